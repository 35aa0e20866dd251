"""MI355X (gfx950) implementation of the multi-RHS Dirac-operator hot path of
Duerr, arXiv:2112.14640: Wilson, Brillouin and staggered applies, their
adjoints, Brillouin link construction, CG / BiCGstab (plain and mixed
precision) and link gradients, all in the HIP library ``libdirac.so``.

``paper_2112_14640_amd.dirac`` is the torch-facing binding and
``paper_2112_14640_amd.autograd`` the differentiable front end.
"""
from . import _lib  # noqa: F401

__all__ = ["dirac", "autograd", "build"]
