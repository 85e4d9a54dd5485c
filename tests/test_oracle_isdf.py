"""Pins of the oracle's ISDF factorisation of K.

* with as many generic points as pairs the fit is exact, so K_ISDF = K;
* the fitted pair densities interpolate: (zeta C)(r_mu) = Z(r_mu) at every
  interpolation point;
* M and K_ISDF are symmetric positive semidefinite;
* on smooth orbitals the error of K_ISDF and of Sigma falls as points are added.
"""
import numpy as np

import gw_inputs as gi
from oracle import casida
from oracle import isdf as I
from oracle.sigma import Problem


def sys_(n_occ=2, n_emp=4, grid=(8, 8, 8), box=6.0, seed=11):
    wl = gi.workload("grid24_v8c32", name="tiny", seed=seed, grid=grid, box=box,
                     n_occ=n_occ, n_emp=n_emp, smooth_sigma=1.0)
    return wl, gi.make_system(wl)


def test_exact_when_points_equal_pairs():
    wl, s = sys_()
    nvc = wl.n_occ * wl.n_emp
    pts = gi.random_grid_points(nvc, wl.n_r, seed=3)
    k_ex, _ = casida.hartree_matrix(s.phi, wl.n_occ, wl.grid, wl.h)
    k_is = I.k_isdf(s.phi, wl.n_occ, wl.grid, wl.h, pts)
    assert np.max(np.abs(k_is - k_ex)) <= 1e-9 * np.max(np.abs(k_ex))


def test_interpolates_at_points():
    wl, s = sys_(n_occ=3, n_emp=6)
    pts = gi.random_grid_points(10, wl.n_r, seed=4)
    cmat, zeta, _ = I.isdf_factors(s.phi, wl.n_occ, wl.grid, wl.h, pts)
    z = casida.pair_densities(s.phi, wl.n_occ)       # [N_vc, N_r]
    fit_at_pts = (zeta.T @ cmat)[pts]                # [N_mu, N_vc]
    assert np.max(np.abs(fit_at_pts - z[:, pts].T)) <= 1e-10 * np.max(np.abs(z))


def test_symmetric_psd():
    wl, s = sys_(n_occ=3, n_emp=6)
    pts = gi.random_grid_points(12, wl.n_r, seed=5)
    _, _, m = I.isdf_factors(s.phi, wl.n_occ, wl.grid, wl.h, pts)
    k = I.k_isdf(s.phi, wl.n_occ, wl.grid, wl.h, pts)
    for a in (m, k):
        assert np.max(np.abs(a - a.T)) <= 1e-12 * np.max(np.abs(a))
        assert np.min(np.linalg.eigvalsh(a)) >= -1e-10 * np.max(np.abs(a))


def test_error_falls_with_points():
    wl, s = sys_(n_occ=3, n_emp=8, grid=(10, 10, 10), box=7.0)
    k_ex, _ = casida.hartree_matrix(s.phi, wl.n_occ, wl.grid, wl.h)
    pr = Problem(s.phi, s.energies_ev, wl.n_occ, wl.grid, wl.h)
    om = np.linspace(-10, 10, 21)
    m = int(s.qp_states[0])
    ref = pr.sigma_exact(m, om, 0.3)
    errs_k, errs_s = [], []
    for n_mu in (6, 12, 24):
        pts = gi.random_grid_points(n_mu, wl.n_r, seed=6)
        k_is = I.k_isdf(s.phi, wl.n_occ, wl.grid, wl.h, pts)
        errs_k.append(np.linalg.norm(k_is - k_ex) / np.linalg.norm(k_ex))
        ip = I.IsdfProblem(s.phi, s.energies_ev, wl.n_occ, wl.grid, wl.h, pts)
        errs_s.append(np.max(np.abs(ip.sigma_exact(m, om, 0.3) - ref)) / np.max(np.abs(ref)))
    assert errs_k[0] > errs_k[1] > errs_k[2]
    assert errs_s[2] < errs_s[0]
    assert errs_k[2] < 1e-6           # 24 = N_vc points: exact again
