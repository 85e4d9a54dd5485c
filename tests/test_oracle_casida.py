"""Pins of the oracle's pair-space operators (Eqs. 2-4, definition of P_nm).

* an analytic two-orbital system (constant and cosine orbitals) whose single
  Hartree element is 4 pi / (|G|^2 V_box), which fixes the dV factor and the
  kernel normalisation;
* K built with the explicit-DFT Poisson on a tiny grid;
* structural facts: K symmetric PSD, C SPD with lambda_min(C) >= (min Delta)^2,
  kernel scale 0 gives Omega = Delta exactly;
* the coupling vector of a pair (n, m) = (v', c') is the K column of that
  pair times Delta^1/2 (two different formulas for the same integral);
* matrix-free C x equals the dense C times x.
"""
import numpy as np
import pytest

import gw_inputs as gi
from oracle import casida, poisson
from oracle.sigma import Problem


def tiny_system(grid=(8, 8, 8), box=6.0, n_occ=3, n_emp=5, seed=11, smooth=0.0):
    wl = gi.workload("grid24_v8c32", name="tiny", seed=seed, grid=grid, box=box,
                     n_occ=n_occ, n_emp=n_emp, smooth_sigma=smooth)
    return gi.make_system(wl)


def test_generator_orbitals_are_grid_orthonormal():
    s = tiny_system()
    gram = s.phi @ s.phi.T * s.wl.dv
    assert np.max(np.abs(gram - np.eye(s.wl.n_orb))) < 1e-13


def test_analytic_plane_wave_pair():
    """phi_v = 1/sqrt(V), phi_c = sqrt(2/V) cos(G.r): (vc|vc) = 4 pi / (G^2 V)."""
    shape, h = (12, 10, 8), 0.5
    vol = np.prod(shape) * h ** 3
    x = np.arange(shape[0])[:, None, None] * h
    gx = 2 * np.pi * 2 / (shape[0] * h)
    phv = np.full(shape, 1 / np.sqrt(vol)).reshape(-1)
    phc = (np.sqrt(2 / vol) * np.cos(gx * x) * np.ones(shape)).reshape(-1)
    phi = np.stack([phv, phc])
    k, asym = casida.hartree_matrix(phi, 1, shape, h)
    assert k.shape == (1, 1)
    expect = 4 * np.pi / (gx ** 2 * vol)
    assert abs(k[0, 0] - expect) <= 1e-12 * expect
    # (vv|vc): the density phi_v^2 is constant, so its potential vanishes
    eri = casida.eri_vc(phi, 0, 0, 1, shape, h)
    assert abs(eri[0]) < 1e-14


def test_k_symmetric_psd_and_c_spd():
    s = tiny_system()
    pr = Problem(s.phi, s.energies_ev, s.wl.n_occ, s.wl.grid, s.wl.h)
    assert pr.k_asym < 1e-13
    ek = np.linalg.eigvalsh(pr.K)
    assert ek[0] >= -1e-14 * ek[-1]
    om2, _ = pr.eig()
    assert om2[0] >= np.min(pr.delta) ** 2 * (1 - 1e-13)
    assert np.all(pr.delta > 0)


def test_k_matches_explicit_dft_build():
    s = tiny_system(grid=(4, 6, 4), box=3.0, n_occ=2, n_emp=3)
    phi, nocc, shape, h = s.phi, s.wl.n_occ, s.wl.grid, s.wl.h
    dv = h ** 3
    k, _ = casida.hartree_matrix(phi, nocc, shape, h)
    pairs = [(v, c) for v in range(nocc) for c in range(nocc, s.wl.n_orb)]
    kb = np.empty_like(k)
    for i, (v, c) in enumerate(pairs):
        for j, (v2, c2) in enumerate(pairs):
            vpot = poisson.poisson_bruteforce(phi[v2] * phi[c2], shape, h)
            kb[i, j] = dv * np.sum(phi[v] * phi[c] * vpot)
    assert np.max(np.abs(k - kb)) <= 1e-12 * np.max(np.abs(kb))


def test_zero_kernel_gives_delta():
    s = tiny_system()
    pr = Problem(s.phi, s.energies_ev, s.wl.n_occ, s.wl.grid, s.wl.h, kernel_scale=0.0)
    om2, z = pr.eig()
    assert np.allclose(np.sort(om2), np.sort(pr.delta ** 2), rtol=1e-14, atol=0)


def test_coupling_equals_k_column():
    s = tiny_system()
    pr = Problem(s.phi, s.energies_ev, s.wl.n_occ, s.wl.grid, s.wl.h)
    nocc, nc = s.wl.n_occ, s.wl.n_emp
    for v2, c2 in [(0, 0), (2, 4), (1, 3)]:
        n, m = v2, nocc + c2
        p = casida.coupling_vector(s.phi, n, m, nocc, s.wl.grid, s.wl.h, pr.delta)
        col = pr.K[:, v2 * nc + c2] * np.sqrt(pr.delta)
        assert np.max(np.abs(p - col)) <= 1e-12 * np.max(np.abs(col))
        # (nm|vc) = (mn|vc)
        p2 = casida.coupling_vector(s.phi, m, n, nocc, s.wl.grid, s.wl.h, pr.delta)
        assert np.max(np.abs(p - p2)) <= 1e-14 * np.max(np.abs(p))
    # the batched builder agrees with the one-at-a-time builder
    m = s.qp_states[0]
    pm = pr.coupling(m)
    for n in range(s.wl.n_orb):
        p = casida.coupling_vector(s.phi, n, m, nocc, s.wl.grid, s.wl.h, pr.delta)
        assert np.max(np.abs(pm[n] - p)) <= 1e-12 * max(np.max(np.abs(p)), 1e-30)


def test_matrix_free_c_matches_dense():
    s = tiny_system()
    pr = Problem(s.phi, s.energies_ev, s.wl.n_occ, s.wl.grid, s.wl.h)
    x = gi.random_pair_vectors(3, s.wl.n_vc, 5)
    cx = pr.apply_c(x)
    dense = x @ pr.C.T
    assert np.max(np.abs(cx - dense)) <= 1e-12 * np.max(np.abs(dense))
