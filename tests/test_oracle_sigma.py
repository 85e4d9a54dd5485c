"""Pins of the oracle's Sigma_c (Eqs. 7, 9-14).

* the three closed forms (Eq. 7 sum over poles, Eq. 11 per-n form, Eq. 12
  resolvent by dense linear solves) agree: an algebraic identity evaluated by
  different routes;
* the single-pair system (N_v = N_c = 1) reduces to the textbook one-pole
  RPA self-energy Omega = sqrt(Delta^2 + 2 Delta K), W^2 = (nm|vc)^2 Delta / Omega;
* Lanczos (Eq. 13): moments ||P||^2 (T^j)_00 = P^T D^j P for j < 2L; a run of
  full length reproduces the exact resolvent; breakdown ends the recurrence;
* continued fraction (Eq. 14) = dense tridiagonal solve = Gauss quadrature;
* Im Sigma(w, n) has the sign of eta_n, and z Sigma(w, n) -> <P|D^-1|P> for
  large |w|;
* the error falls with the polynomial degree g and with the Lanczos length L
  (the synthetic analogue of the paper's convergence study).
"""
import numpy as np
import pytest

import gw_inputs as gi
import oracle
from oracle import chebyshev as CH
from oracle import sigma as S
from oracle.sigma import HARTREE_EV, Problem


def tiny(grid=(8, 8, 8), box=6.0, n_occ=3, n_emp=5, seed=11, smooth=1.0):
    wl = gi.workload("grid24_v8c32", name="tiny", seed=seed, grid=grid, box=box,
                     n_occ=n_occ, n_emp=n_emp, smooth_sigma=smooth)
    s = gi.make_system(wl)
    pr = Problem(s.phi, s.energies_ev, wl.n_occ, wl.grid, wl.h)
    return s, pr


def test_hartree_constant():
    assert HARTREE_EV == 27.211386245988


def test_three_closed_forms_agree():
    s, pr = tiny()
    om2, z = pr.eig()
    om = np.sqrt(om2)
    dmat = (z * om) @ z.T
    w_ha = np.linspace(-1.0, 1.0, 41)
    d_ha = 0.01
    m = s.qp_states[0]
    pm = pr.coupling(m)
    for n in range(pr.n_orb):
        w = (pm[n] @ z) ** 2
        e7 = S.sigma_n_poles(w_ha, pr.eps[n], pr.eta(n), d_ha, w, om)
        e11 = S.sigma_n_eq11(w_ha, pr.eps[n], pr.eta(n), d_ha, w, om)
        e12 = S.sigma_n_resolvent_dense(dmat, pm[n], w_ha, pr.eps[n], pr.eta(n), d_ha)
        scale = np.max(np.abs(e7))
        assert np.max(np.abs(e7 - e11)) <= 1e-12 * scale
        assert np.max(np.abs(e7 - e12)) <= 1e-10 * scale


def test_single_pair_textbook_pole():
    """N_v = N_c = 1: one pole at Omega = sqrt(Delta^2 + 2 Delta K)."""
    s, pr = tiny(n_occ=1, n_emp=1)
    d = pr.delta[0]
    k = pr.K[0, 0]
    big_om = np.sqrt(d * d + 2 * d * k)
    m = 0
    omega_ev = np.linspace(-15, 15, 31)
    eta_ev = 0.1
    w_ha, d_ha = omega_ev / HARTREE_EV, eta_ev / HARTREE_EV
    expect = np.zeros(len(w_ha), dtype=complex)
    for n in range(2):
        knm = oracle.casida.eri_vc(pr.phi, n, m, 1, pr.shape, pr.h)[0]
        w2 = knm ** 2 * d / big_om
        eta_n = 1.0 if n == 0 else -1.0
        expect += w2 / (w_ha - pr.eps[n] + eta_n * (big_om - 1j * d_ha))
    expect *= HARTREE_EV
    got = pr.sigma_exact(m, omega_ev, eta_ev)
    assert np.max(np.abs(got - expect)) <= 1e-12 * np.max(np.abs(expect))
    # the method with one Lanczos step: the interval is tight around Omega^2,
    # so p_7 reproduces sqrt to rounding
    lo, hi = d * d, big_om ** 2 * (1 + 1e-3)
    gl = pr.sigma_lanczos(m, omega_ev, eta_ev, 1, lo, hi, 7)
    assert np.max(np.abs(gl - expect)) <= 1e-9 * np.max(np.abs(expect))


def _random_spd(n, seed, lo=0.1, hi=1.0):
    rng = np.random.default_rng(seed)
    q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    ev = np.sort(rng.uniform(lo, hi, n))
    return 0.5 * ((q * ev) @ q.T + ((q * ev) @ q.T).T), rng.standard_normal(n)


def test_lanczos_moments():
    a_mat, p = _random_spd(30, 5)
    for L in (1, 3, 6):
        a, b, nrm2 = S.lanczos(lambda v: a_mat @ v, p, L)
        assert len(a) == L and len(b) == L - 1
        t = S.tridiag_matrix(a, b)
        tj = np.eye(L)
        dj = p.copy()
        for j in range(2 * L):
            lhs = nrm2 * tj[0, 0]
            rhs = p @ dj
            assert abs(lhs - rhs) <= 1e-11 * abs(rhs), (L, j)
            tj = tj @ t
            dj = a_mat @ dj


def test_full_length_lanczos_is_exact_resolvent():
    a_mat, p = _random_spd(15, 6)
    a, b, nrm2 = S.lanczos(lambda v: a_mat @ v, p, 15)
    for zeta in (0.0, 0.3 + 0.01j, -2.0 + 0.5j, 5.0 + 1e-3j):
        exact = p @ np.linalg.solve(zeta * np.eye(15) - a_mat, p.astype(complex))
        got = S.continued_fraction(a, b, nrm2, zeta)
        assert abs(got - exact) <= 1e-10 * abs(exact)


def test_breakdown_and_zero_start():
    a_mat, p = _random_spd(6, 7)
    a, b, nrm2 = S.lanczos(lambda v: a_mat @ v, p, 20)
    assert len(a) == 6 and len(b) == 5
    # start vector in an invariant subspace of dimension 2
    d = np.diag([0.2, 0.5, 0.9, 1.3])
    a2, b2, _ = S.lanczos(lambda v: d @ v, np.array([1.0, 0, 2.0, 0]), 10)
    assert len(a2) == 2
    a3, b3, n3 = S.lanczos(lambda v: d @ v, np.zeros(4), 10)
    assert n3 == 0 and len(a3) == 0
    s = S.sigma_n_from_tridiag(a3, b3, n3, np.array([0.1, 0.2]), 0.0, 1.0, 0.01)
    assert np.all(s == 0)


def test_continued_fraction_dense_and_quadrature():
    rng = np.random.default_rng(8)
    L = 9
    a = rng.uniform(0.1, 1.0, L)
    b = rng.uniform(0.05, 0.3, L - 1)
    nrm2 = 2.7
    zetas = np.array([0.0, 0.4 + 0.02j, -1.0 + 0.3j, 2.0 + 1e-4j])
    cf = S.continued_fraction(a, b, nrm2, zetas)
    dense = S.tridiag_resolvent_dense(a, b, nrm2, zetas)
    th, u = np.linalg.eigh(S.tridiag_matrix(a, b))
    wq = nrm2 * u[0] ** 2
    quad = np.array([np.sum(wq / (z - th)) for z in zetas])
    assert np.max(np.abs(cf - dense)) <= 1e-12 * np.max(np.abs(dense))
    assert np.max(np.abs(cf - quad)) <= 1e-12 * np.max(np.abs(quad))


@pytest.fixture(scope="module")
def small_case():
    s = gi.make_system("grid24_v8c32")
    wl = s.wl
    pr = Problem(s.phi, s.energies_ev, wl.n_occ, wl.grid, wl.h)
    lo, hi = oracle.default_interval(pr)
    return s, pr, lo, hi


def test_sign_and_asymptote(small_case):
    s, pr, lo, hi = small_case
    m = s.qp_states[1]
    coeffs = pr.lanczos_coeffs(m, 32, lo, hi, 7)
    w_ha = s.omega_ev / HARTREE_EV
    d_ha = s.wl.eta / HARTREE_EV
    dg = pr.dg_matrix(lo, hi, 7)
    pm = pr.coupling(m)
    for n in range(0, pr.n_orb, 3):
        a, b, nrm2 = coeffs[n]
        sig = S.sigma_n_from_tridiag(a, b, nrm2, w_ha, pr.eps[n], pr.eta(n), d_ha)
        assert np.all(np.sign(sig.imag) == pr.eta(n))
        big = np.array([1e7, -1e7])
        sz = S.sigma_n_from_tridiag(a, b, nrm2, big, pr.eps[n], pr.eta(n), d_ha)
        zz = S.z_of(big, pr.eps[n], pr.eta(n), d_ha)
        expect = pm[n] @ np.linalg.solve(dg, pm[n])
        assert np.max(np.abs(sz * zz - expect)) <= 1e-5 * expect


def test_routes_agree_and_converge(small_case):
    s, pr, lo, hi = small_case
    m = s.qp_states[0]
    om, eta = s.omega_ev, s.wl.eta
    sl = pr.sigma_lanczos(m, om, eta, 64, lo, hi, 7)
    sm = pr.sigma_lanczos(m, om, eta, 64, lo, hi, 7, route="measure")
    sf = pr.sigma_lanczos(m, om, eta, 64, lo, hi, 7, route="matfree")
    scale = np.max(np.abs(sl))
    assert np.max(np.abs(sl - sm)) <= 1e-11 * scale
    assert np.max(np.abs(sl - sf)) <= 1e-11 * scale
    # convergence in L towards Sigma_Dg, and in g towards Sigma_exact
    sdg = pr.sigma_dg(m, om, eta, lo, hi, 7)
    errs_l = [np.max(np.abs(pr.sigma_lanczos(m, om, eta, L, lo, hi, 7, route="measure") - sdg))
              for L in (4, 16, 64)]
    assert errs_l[0] > errs_l[1] > errs_l[2]
    sx = pr.sigma_exact(m, om, eta)
    errs_g = [np.max(np.abs(pr.sigma_dg(m, om, eta, lo, hi, g) - sx)) for g in (3, 7, 12, 20)]
    assert all(x > y for x, y in zip(errs_g, errs_g[1:]))
    # full-dimension Lanczos equals the L -> N_vc limit
    s_full = pr.sigma_lanczos(m, om, eta, pr.delta.size, lo, hi, 7, route="measure")
    assert np.max(np.abs(s_full - sdg)) <= 1e-9 * np.max(np.abs(sdg))


def test_zero_kernel_sigma_closed_form():
    """K = 0: Omega_s = Delta_s and Z = I, so P_nm has no coupling and
    Sigma vanishes identically (every (nm|vc) is scaled by the kernel)."""
    s, _ = tiny()
    pr0 = Problem(s.phi, s.energies_ev, s.wl.n_occ, s.wl.grid, s.wl.h, kernel_scale=0.0)
    sig = pr0.sigma_exact(s.qp_states[0], np.linspace(-5, 5, 11), 0.1)
    assert np.max(np.abs(sig)) == 0.0
