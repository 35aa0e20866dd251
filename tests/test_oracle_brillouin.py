"""Pins for the Brillouin oracle: link census and transport, dense definition, free field, symmetries."""
import itertools
import os

import numpy as np
import pytest

import synthetic_inputs as si
from oracle.brillouin import (CENTER, LAMBDA, RHO, brillouin_apply, brillouin_apply_dagger, brillouin_apply_sites,
                              brillouin_links, brillouin_links_all, direction, direction_index, free_brillouin_symbol,
                              hops, link_from_stored)
from oracle.dense import brillouin_dense
from oracle.gamma import GAMMA, GAMMA5
from oracle.lattice import all_sites, flat_index, site_field
from tests.oracle_helpers import (assert_same_spectrum, flip_t_boundary, gauge_rotate_links,
                                  gauge_rotate_wilson_vector, momenta, plane_wave, rel_err)


def _golden(golden_dir):
    vals = {}
    census = []
    with open(os.path.join(golden_dir, "brillouin_weights.txt")) as f:
        for ln in f:
            if not ln.strip() or ln.startswith("#"):
                continue
            k, *v = ln.split()
            if k == "census":
                census.append(tuple(int(x) for x in v))
            else:
                vals[k] = [float(x) for x in v]
    return vals, census


def test_constants_and_census(golden_dir):
    vals, census = _golden(golden_dir)
    np.testing.assert_allclose(RHO[1:], np.array(vals["rho_num"]) / vals["rho_den"][0], rtol=1e-15)
    np.testing.assert_allclose(LAMBDA, np.array(vals["lambda_num"]) / vals["lambda_den"][0], rtol=1e-15)
    np.testing.assert_allclose(-0.5 * LAMBDA[0], vals["center_weight"][0])
    counts = {}
    for i in range(81):
        if i != CENTER:
            counts[hops(direction(i))] = counts.get(hops(direction(i)), 0) + 1
    for k, terms, paths in census:
        assert counts[k] == terms
        assert len(list(itertools.permutations(range(k)))) == paths
    assert all(direction_index(direction(i)) == i for i in range(81))
    assert np.all(direction(CENTER) == 0)
    for i in range(81):
        assert np.all(direction(80 - i) == -direction(i))


def test_links_unit_field_and_one_hop():
    dims, nc = (2, 2, 2, 4), 3
    V1 = si.gauge_field(None, dims, nc, "unit")
    w = brillouin_links_all(V1)
    np.testing.assert_allclose(w, np.broadcast_to(np.eye(nc), w.shape), atol=1e-15)
    rng = np.random.default_rng(1)
    V = si.gauge_field(rng, dims, nc, "haar")
    w = brillouin_links_all(V)
    vs = site_field(V)
    coords = all_sites(dims)
    for mu in range(4):
        d = np.zeros(4, dtype=int)
        d[mu] = 1
        np.testing.assert_allclose(w[:, direction_index(d)], vs[:, mu], atol=1e-15)
        back = vs[flat_index(coords - d, dims), mu]
        np.testing.assert_allclose(w[:, direction_index(-d)], np.conj(np.swapaxes(back, -1, -2)), atol=1e-15)


def test_two_hop_by_hand():
    dims, nc = (4, 4, 2, 4), 2
    rng = np.random.default_rng(2)
    V = si.gauge_field(rng, dims, nc, "haar")
    w = brillouin_links_all(V, sites=np.array([[1, 2, 0, 3]]))
    # W_{+x+y}(n) = [V_x(n) V_y(n+x) + V_y(n) V_x(n+y)] / 2 at n = (1,2,0,3)
    expect = 0.5 * (V[3, 0, 2, 1, 0] @ V[3, 0, 2, 2, 1] + V[3, 0, 2, 1, 1] @ V[3, 0, 3, 1, 0])
    np.testing.assert_allclose(w[0, direction_index([1, 1, 0, 0])], expect, atol=1e-15)
    # W_{+x-t}(n) = [V_x(n) V_t(n+x-t)^dag + V_t(n-t)^dag V_x(n-t)] / 2
    dag = lambda a: np.conj(a.T)
    expect = 0.5 * (V[3, 0, 2, 1, 0] @ dag(V[2, 0, 2, 2, 3]) + dag(V[2, 0, 2, 1, 3]) @ V[2, 0, 2, 1, 0])
    np.testing.assert_allclose(w[0, direction_index([1, 0, 0, -1])], expect, atol=1e-15)


def test_links_reverse_relation_and_unitarity():
    dims, nc = (2, 2, 4, 2), 3
    rng = np.random.default_rng(3)
    V = si.gauge_field(rng, dims, nc, "haar")
    w = brillouin_links_all(V)
    coords = all_sites(dims)
    for i in range(81):
        d = direction(i)
        shifted = w[flat_index(coords - d, dims), i]
        np.testing.assert_allclose(w[:, 80 - i], np.conj(np.swapaxes(shifted, -1, -2)), atol=1e-14)
    unitary = 0
    for i in range(40):
        prod = w[:, i] @ np.conj(np.swapaxes(w[:, i], -1, -2))
        if np.allclose(prod, np.eye(nc), atol=1e-12):
            unitary += 1
    assert unitary == 4  # only the on-axis W are special unitary (Tab. off-axis caption)


def test_links_pure_gauge_and_covariance():
    dims, nc = (2, 4, 2, 4), 2
    rng = np.random.default_rng(4)
    g = si.gauge_transform(rng, dims, nc)
    V1 = si.gauge_field(None, dims, nc, "unit")
    w = brillouin_links_all(gauge_rotate_links(V1, g))
    gs = site_field(g)
    coords = all_sites(dims)
    for i in range(81):
        d = direction(i)
        expect = gs @ np.conj(np.swapaxes(gs[flat_index(coords + d, dims)], -1, -2))
        np.testing.assert_allclose(w[:, i], expect, atol=1e-14)
    V = si.gauge_field(rng, dims, nc, "haar")
    w0 = brillouin_links_all(V)
    wg = brillouin_links_all(gauge_rotate_links(V, g))
    for i in range(81):
        d = direction(i)
        expect = gs @ w0[:, i] @ np.conj(np.swapaxes(gs[flat_index(coords + d, dims)], -1, -2))
        np.testing.assert_allclose(wg[:, i], expect, atol=1e-14)


def _cols(psi):
    return psi.reshape(-1, psi.shape[-1])


@pytest.mark.parametrize("dims,nc,apbc", [((2, 2, 2, 2), 2, True), ((2, 2, 2, 4), 3, False),
                                          ((4, 4, 2, 4), 2, True)])
def test_stencil_equals_dense_definition(dims, nc, apbc):
    rng = np.random.default_rng(12)
    V = si.gauge_field(rng, dims, nc, "haar")
    psi = si.wilson_vector(rng, dims, nc, 2)
    wall = brillouin_links_all(V)
    w40 = brillouin_links(V)
    d = brillouin_dense(wall, dims, 0.11, apbc)
    np.testing.assert_allclose(_cols(brillouin_apply(w40, psi, 0.11, apbc)), d @ _cols(psi), atol=1e-12)
    np.testing.assert_allclose(_cols(brillouin_apply_dagger(w40, psi, 0.11, apbc)), d.conj().T @ _cols(psi),
                               atol=1e-12)


def _closed_form_symbol(p, m):
    """m + 2(1 - prod cos^2(p/2)) + i sum_mu gamma_mu sin p_mu prod_{nu != mu} (2 + cos p_nu)/3."""
    s = (m + 2.0 * (1.0 - np.prod(np.cos(p / 2) ** 2))) * np.eye(4, dtype=complex)
    for mu in range(4):
        f = np.prod([(2 + np.cos(p[nu])) / 3 for nu in range(4) if nu != mu])
        s = s + 1j * np.sin(p[mu]) * f * GAMMA[mu]
    return s


def test_free_symbol_closed_form():
    rng = np.random.default_rng(13)
    for _ in range(20):
        p = rng.uniform(-np.pi, np.pi, 4)
        np.testing.assert_allclose(free_brillouin_symbol(p, 0.05), _closed_form_symbol(p, 0.05), atol=1e-14)
    # spectrum edge Re z = 2 + m (Sec. 9) at p = (pi,pi,pi,pi); zero mode m at p = 0
    np.testing.assert_allclose(free_brillouin_symbol(np.full(4, np.pi), 0.01), 2.01 * np.eye(4), atol=1e-14)
    np.testing.assert_allclose(free_brillouin_symbol(np.zeros(4), 0.01), 0.01 * np.eye(4), atol=1e-14)


@pytest.mark.parametrize("apbc", [True, False])
def test_free_field_plane_waves(apbc):
    dims, nc, m = (4, 2, 2, 4), 1, 0.03
    V = si.gauge_field(None, dims, nc, "unit")
    w40 = brillouin_links(V)
    rng = np.random.default_rng(14)
    for p in momenta(dims, apbc)[::5]:
        chi = si.complex_gaussian(rng, (nc, 4, 1))
        psi = plane_wave(dims, p, chi)
        expect = plane_wave(dims, p, np.einsum("st,atr->asr", _closed_form_symbol(p, m), chi))
        np.testing.assert_allclose(brillouin_apply(w40, psi, m, apbc), expect, atol=1e-13)


def test_free_spectrum_dense():
    dims, nc, m = (2, 2, 4, 4), 1, 0.05
    V = si.gauge_field(None, dims, nc, "unit")
    ev = np.linalg.eigvals(brillouin_dense(brillouin_links_all(V), dims, m, True))
    expect = []
    for p in momenta(dims, True):
        s = _closed_form_symbol(p, m)
        expect += list(np.linalg.eigvals(s))
    assert_same_spectrum(ev, np.array(expect))


def test_gamma5_hermiticity_and_covariance():
    dims, nc = (2, 4, 2, 4), 2
    rng = np.random.default_rng(15)
    V = si.gauge_field(rng, dims, nc, "haar")
    psi = si.wilson_vector(rng, dims, nc, 2)
    w40 = brillouin_links(V)
    g5 = lambda f: np.einsum("st,...atr->...asr", GAMMA5, f)
    np.testing.assert_allclose(brillouin_apply_dagger(w40, psi, 0.2), g5(brillouin_apply(w40, g5(psi), 0.2)),
                               atol=1e-13)
    g = si.gauge_transform(rng, dims, nc)
    wg = brillouin_links(gauge_rotate_links(V, g))
    lhs = brillouin_apply(wg, gauge_rotate_wilson_vector(g, psi), 0.2)
    rhs = gauge_rotate_wilson_vector(g, brillouin_apply(w40, psi, 0.2))
    np.testing.assert_allclose(lhs, rhs, atol=1e-13)


def test_antiperiodic_equals_flipped_links_and_sampled_sites():
    dims, nc = (2, 2, 2, 4), 2
    rng = np.random.default_rng(16)
    V = si.gauge_field(rng, dims, nc, "haar")
    psi = si.wilson_vector(rng, dims, nc, 3)
    a = brillouin_apply(brillouin_links(V), psi, 0.1, True)
    b = brillouin_apply(brillouin_links(flip_t_boundary(V)), psi, 0.1, False)
    np.testing.assert_allclose(a, b, atol=1e-14)
    sites = np.array([[0, 1, 1, 3], [1, 0, 0, 0]])
    sub = brillouin_apply(brillouin_links(V), psi, 0.1, True, sites=sites)
    for k, (x, y, z, t) in enumerate(sites):
        np.testing.assert_allclose(sub[k], a[t, z, y, x], atol=1e-14)
    coords = all_sites(dims)
    w40 = brillouin_links(V)
    wall = brillouin_links_all(V)
    for i in (0, 39, 41, 80, 13, 67):
        np.testing.assert_allclose(link_from_stored(w40, coords, i, dims), wall[:, i], atol=1e-14)


def test_random_links_stencil_matches_dense_for_arbitrary_w():
    """The apply is defined for any stored W (not only path averages): dense check with random W."""
    dims, nc = (2, 2, 2, 4), 2
    rng = np.random.default_rng(17)
    nx, ny, nz, nt = dims
    w40 = si.complex_gaussian(rng, (nt, nz, ny, nx, 40, nc, nc))
    coords = all_sites(dims)
    wall = np.zeros((coords.shape[0], 81, nc, nc), dtype=complex)
    wall[:, CENTER] = np.eye(nc)
    for i in range(81):
        if i != CENTER:
            wall[:, i] = link_from_stored(w40, coords, i, dims)
    psi = si.wilson_vector(rng, dims, nc, 2)
    d = brillouin_dense(wall, dims, 0.07, True)
    assert rel_err(_cols(brillouin_apply(w40, psi, 0.07)), d @ _cols(psi)) < 1e-13


def test_apply_from_links_at_sites_and_fp32_storage():
    """The sampled-site form (81 links per site from the path averages, no stored array) gives the
    stored-link apply; complex64 storage is evaluated in FP64 (same values as its complex128 copy)."""
    dims, nc = (4, 2, 2, 4), 3
    rng = np.random.default_rng(18)
    V = si.gauge_field(rng, dims, nc, "haar")
    psi = si.wilson_vector(rng, dims, nc, 2)
    sites = np.array([[0, 0, 0, 0], [3, 1, 1, 3], [2, 0, 1, 1]])
    w81 = brillouin_links_all(V, sites=sites)
    for dag, full in ((False, brillouin_apply), (True, brillouin_apply_dagger)):
        ref = full(brillouin_links(V), psi, 0.05, True, sites=sites)
        got = brillouin_apply_sites(w81, psi, 0.05, sites, True, dagger=dag)
        np.testing.assert_allclose(got, ref, atol=1e-14)
    v32, p32 = V.astype(np.complex64), psi.astype(np.complex64)
    a = brillouin_apply_sites(brillouin_links_all(v32, sites=sites), p32, 0.05, sites)
    b = brillouin_apply_sites(brillouin_links_all(v32.astype(complex), sites=sites), p32.astype(complex), 0.05, sites)
    assert a.dtype == np.complex128
    np.testing.assert_array_equal(a, b)
