"""Pins of the oracle's exchange self-energy and quasiparticle solve.

* for an empty orbital m = c, (vc|vc) is the diagonal element K_{vc,vc} of the
  dense Hartree matrix (built from all pair densities at once);
* (vm|vm) > 0 (positive Coulomb kernel), so Sigma^ex_mm < 0;
* on a tiny grid the FFT Poisson route equals explicit DFT matrices;
* the graphical QP solve reproduces the closed-form root and renormalisation
  factor of a linear Re Sigma^corr(w) = a + b w, picks the root nearest e_m
  when there are several, and reports none when f never changes sign.
"""
import numpy as np

import gw_inputs as gi
from oracle import casida
from oracle import exchange as X
from oracle.poisson import poisson_bruteforce
from oracle.sigma import HARTREE_EV


def _sys(grid=(8, 8, 8), box=6.0, n_occ=3, n_emp=5, seed=11):
    wl = gi.workload("grid24_v8c32", name="tiny", seed=seed, grid=grid, box=box,
                     n_occ=n_occ, n_emp=n_emp, smooth_sigma=1.0)
    return wl, gi.make_system(wl)


def test_exchange_integral_is_hartree_diagonal():
    wl, s = _sys()
    k, _ = casida.hartree_matrix(s.phi, wl.n_occ, wl.grid, wl.h)
    nc = wl.n_emp
    for v in range(wl.n_occ):
        for c in (0, 2, 4):
            m = wl.n_occ + c
            got = X.exchange_integral(s.phi, v, m, wl.grid, wl.h)
            assert abs(got - k[v * nc + c, v * nc + c]) <= 1e-12 * abs(got)


def test_positive_integrals_negative_sigma_x():
    wl, s = _sys()
    for m in range(wl.n_occ + wl.n_emp):
        for v in range(wl.n_occ):
            assert X.exchange_integral(s.phi, v, m, wl.grid, wl.h) > 0.0
        assert X.sigma_x(s.phi, wl.n_occ, m, wl.grid, wl.h) < 0.0


def test_fft_route_equals_dft_matrices():
    wl, s = _sys(grid=(4, 6, 4), box=4.0, n_occ=2, n_emp=2)
    v, m = 1, 3
    rho = s.phi[v] * s.phi[m]
    brute = wl.h ** 3 * np.sum(rho * poisson_bruteforce(rho, wl.grid, wl.h))
    assert abs(X.exchange_integral(s.phi, v, m, wl.grid, wl.h) - brute) <= 1e-12 * abs(brute)


def test_qp_solve_linear_self_energy():
    w = np.linspace(-20, 20, 401)
    a, b = 0.7, -0.25
    sc = a + b * w + 0.01j
    eps, sx, vxc = -5.0, -3.0, -2.5
    e, z = X.qp_solve(w, sc, eps, sx, vxc)
    assert abs(e - (eps + sx + a - vxc) / (1 - b)) <= 1e-12
    assert abs(z - 1.0 / (1.0 - b)) <= 1e-12


def test_qp_solve_nearest_root_and_no_root():
    w = np.linspace(-10, 10, 2001)
    # Re Sigma = 3 sin(w): several roots of -1 + 3 sin(w) - w; the nearest to e_m = -1
    sc = 3.0 * np.sin(w)
    e, _ = X.qp_solve(w, sc, -1.0, 0.0, 0.0)
    f = lambda x: -1.0 + 3.0 * np.sin(x) - x
    roots = [x for x in np.linspace(-10, 10, 200001)[:-1]
             if f(x) * f(x + 1e-4) <= 0]
    nearest = min(roots, key=lambda r: abs(r + 1.0))
    assert abs(e - nearest) <= 1e-3
    e2, z2 = X.qp_solve(w, np.full(len(w), 50.0), 0.0, 0.0, 0.0)
    assert np.isnan(e2) and np.isnan(z2)
