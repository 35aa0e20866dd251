"""Plain FP64 CPU oracle for the Dirac-operator hot path.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
bench's CPU-baseline leg may import this package.  The product library never
calls it and has no fallback to it.

Everything here is written from the paper's definitions (Duerr,
"Fast and flexible implementations of Wilson, Brillouin and Susskind fermions
in lattice QCD", arXiv:2112.14640) in complex128 NumPy, vectorised over sites
but with no blocking, fusion or reordering beyond what the definitions state:

* ``gamma``      chiral gamma matrices (App. A)
* ``lattice``    site indexing, neighbour shifts, boundary signs, staggered phases
* ``wilson``     D_W (Eqs. def_wils, def_sder, def_wlap, app_wils) and its adjoint
* ``brillouin``  W links (Tab. off-axis) and D_B (Eqs. def_bril, def_ider, def_blap, app_bril)
* ``staggered``  D_S (Eq. def_stag) and its adjoint
* ``clover``     clover-leaf field strength and the clover term C (Sec. 4, Eq. def_clov)
* ``laplace``    the embedded Wilson and Brillouin Laplacians -Delta/2 + m^2/2 (Eqs. app_wlap, app_blap)
* ``stout``      stout smearing of the links (Sec. 2; rho = 0.12, three steps by default)
* ``dense``      brute-force dense matrices assembled from the operator-level definitions
* ``solvers``    CG / BiCGstab (Sec. 9) and the CG-Lanczos spectrum estimate
* ``force``      link gradients ("fermion force") of Dirac bilinears and solves

Array conventions are those of ``synthetic_inputs``: gauge (Nt,Nz,Ny,Nx,4,Nc,Nc),
Wilson-type vectors (Nt,Nz,Ny,Nx,Nc,4,Nv), staggered vectors (Nt,Nz,Ny,Nx,Nc,Nv).
Direction mu = 0,1,2,3 is x,y,z,t (the paper's 1..4).
"""
