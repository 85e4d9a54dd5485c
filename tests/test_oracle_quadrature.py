"""Pins of the oracle's Lanczos-on-C Gauss quadrature.

* run to full length (L = N_vc) it reproduces Eq. 7 with the exact
  eigenpairs of C (no polynomial, so no fit error);
* the quadrature integrates x^j exactly for j < 2L: sum_k w_k theta_k^j =
  P^T C^j P;
* nodes and weights equal the poles and residues of the continued fraction
  (Eq. 14) of the same tridiagonal;
* at equal cost in C-products it beats the polynomial method, whose error
  floor is the fit of sqrt by p_g.
"""
import numpy as np

import gw_inputs as gi
import oracle
from oracle import quadrature as Q
from oracle import sigma as S
from oracle.sigma import Problem


def tiny(n_occ=2, n_emp=4, seed=11):
    wl = gi.workload("grid24_v8c32", name="tiny", seed=seed, grid=(8, 8, 8), box=6.0,
                     n_occ=n_occ, n_emp=n_emp, smooth_sigma=1.0)
    s = gi.make_system(wl)
    return s, Problem(s.phi, s.energies_ev, wl.n_occ, wl.grid, wl.h)


def rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def test_full_length_is_exact():
    s, pr = tiny()
    om = np.linspace(-12, 12, 25)
    m = int(s.qp_states[0])
    exact = pr.sigma_exact(m, om, 0.2)
    got = Q.sigma_quadrature(pr, m, om, 0.2, pr.delta.size)
    assert rel(got, exact) <= 1e-10


def test_moments_exact():
    s, pr = tiny(n_occ=3, n_emp=5)
    m = int(s.qp_states[1])
    L = 5
    for (a, b, n2), p in zip(Q.lanczos_coeffs_c(pr, m, L, n_list=[0, 6]),
                             pr.coupling(m, [0, 6])):
        th, w = Q.gauss_nodes_weights(a, b, n2)
        v = p.copy()
        for j in range(2 * L):
            assert abs(np.sum(w * th ** j) - p @ v) <= 1e-9 * abs(p @ v)
            v = pr.C @ v


def test_nodes_weights_match_continued_fraction():
    s, pr = tiny()
    m = int(s.qp_states[0])
    (a, b, n2), = Q.lanczos_coeffs_c(pr, m, 6, n_list=[3])
    th, w = Q.gauss_nodes_weights(a, b, n2)
    zetas = np.array([0.0, -0.3 + 0.01j, 1.5 + 0.2j])
    quad = np.array([np.sum(w / (z - th)) for z in zetas])
    assert rel(quad, S.continued_fraction(a, b, n2, zetas)) <= 1e-12


def test_beats_polynomial_at_equal_cost():
    s, pr = tiny(n_occ=4, n_emp=12)                       # N_vc = 48
    om = np.linspace(-10, 10, 41)
    m = int(s.qp_states[0])
    lo, hi = oracle.default_interval(pr)
    exact = pr.sigma_exact(m, om, 0.2)
    g = 7
    poly = pr.sigma_lanczos(m, om, 0.2, 3, lo, hi, g)      # 3 D-steps = 21 C-products
    quad = Q.sigma_quadrature(pr, m, om, 0.2, 3 * g)       # 21 C-steps
    assert rel(quad, exact) < 0.2 * rel(poly, exact)
