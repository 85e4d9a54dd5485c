"""Pins of the oracle's Tamm-Dancoff Sigma_c (B = 0 in the Casida matrix).

* eigendecomposition route (Eq. 7 with the eigenpairs of A) = explicit
  resolvent solves <k|(z_n + eta_n A)^-1|k> (no eigendecomposition);
* the single-pair system reduces to one pole at Delta + (vc|vc) with residue
  (nm|vc)^2;
* Lanczos on A run to full length reproduces the exact result; the dense and
  matrix-free routes agree;
* weak coupling: with the Coulomb kernel scaled by s -> 0 both TDA and the
  full method reduce to s^2 sum_n sum_vc (nm|vc)^2 / (w - e_n + eta_n (Delta_vc
  - i delta)) (Omega -> Delta, eigenvectors -> unit vectors), so TDA / s^2,
  RPA / s^2 and that double sum agree to O(s);
* Im Sigma(w, n) has the sign of eta_n.
"""
import numpy as np

import gw_inputs as gi
import oracle
from oracle import tda as T
from oracle.sigma import HARTREE_EV, Problem, occupation_sign


def tiny(n_occ=3, n_emp=5, seed=11, scale=1.0, grid=(8, 8, 8), box=6.0):
    wl = gi.workload("grid24_v8c32", name="tiny", seed=seed, grid=grid, box=box,
                     n_occ=n_occ, n_emp=n_emp, smooth_sigma=1.0)
    s = gi.make_system(wl)
    pr = Problem(s.phi, s.energies_ev, wl.n_occ, wl.grid, wl.h, kernel_scale=scale)
    return s, pr


def rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def test_eigh_equals_resolvent_solves():
    s, pr = tiny()
    om = np.linspace(-12, 12, 25)
    m = int(s.qp_states[0])
    a = T.sigma_tda_exact(pr, m, om, 0.2)
    b = T.sigma_tda_dense_resolvent(pr, m, om, 0.2)
    assert np.max(np.abs(a)) > 1e-3
    assert rel(a, b) <= 1e-11


def test_single_pair_pole():
    s, pr = tiny(n_occ=1, n_emp=1)
    om_s = pr.delta[0] + pr.K[0, 0]
    om = np.linspace(-15, 15, 31)
    w_ha, d_ha = om / HARTREE_EV, 0.1 / HARTREE_EV
    m = 0
    expect = np.zeros(len(om), dtype=complex)
    for n in range(2):
        k = oracle.casida.eri_vc(pr.phi, n, m, 1, pr.shape, pr.h)[0]
        eta = 1.0 if n == 0 else -1.0
        expect += k * k / (w_ha - pr.eps[n] + eta * (om_s - 1j * d_ha))
    expect *= HARTREE_EV
    assert rel(T.sigma_tda_exact(pr, m, om, 0.1), expect) <= 1e-12
    assert rel(T.sigma_tda_lanczos(pr, m, om, 0.1, 1), expect) <= 1e-12


def test_full_length_lanczos_and_routes():
    s, pr = tiny(n_occ=2, n_emp=4)
    nvc = 8
    om = np.linspace(-10, 10, 21)
    m = int(s.qp_states[1])
    exact = T.sigma_tda_exact(pr, m, om, 0.3)
    full = T.sigma_tda_lanczos(pr, m, om, 0.3, nvc)
    assert rel(full, exact) <= 1e-10
    dense = T.lanczos_coeffs_tda(pr, m, 6, n_list=[0, 5])
    mfree = T.lanczos_coeffs_tda(pr, m, 6, n_list=[0, 5], route="matfree")
    for (a1, b1, n1), (a2, b2, n2) in zip(dense, mfree):
        assert rel(a2, a1) <= 1e-11 and rel(b2, b1) <= 1e-10 and abs(n2 - n1) <= 1e-12 * n1
    # a short run converges towards the exact result
    e4 = rel(T.sigma_tda_lanczos(pr, m, om, 0.3, 2), exact)
    e7 = rel(T.sigma_tda_lanczos(pr, m, om, 0.3, 6), exact)
    assert e7 < e4


def test_weak_coupling_limit_matches_full_method():
    sc = 1e-4
    s, pr = tiny(scale=sc)
    om = np.linspace(-9, 9, 19)
    m = int(s.qp_states[0])
    w_ha, d_ha = om / HARTREE_EV, 0.2 / HARTREE_EV
    # s^2 sum_n sum_vc (nm|vc)_1^2 / (w - e_n + eta_n (Delta_vc - i delta))
    k1 = T.eri_vectors(pr, m) / sc
    ref = np.zeros(len(om), dtype=complex)
    for n in range(pr.n_orb):
        eta = occupation_sign(n, pr.n_occ)
        ref += np.sum(k1[n][None, :] ** 2 /
                      (w_ha[:, None] - pr.eps[n] + eta * (pr.delta[None, :] - 1j * d_ha)), axis=1)
    ref *= HARTREE_EV
    tda = T.sigma_tda_exact(pr, m, om, 0.2) / sc ** 2
    rpa = pr.sigma_exact(m, om, 0.2) / sc ** 2
    assert rel(tda, ref) <= 1e-3
    assert rel(rpa, ref) <= 1e-3
    # and at full coupling the two differ (B matters)
    s1, pr1 = tiny()
    assert rel(T.sigma_tda_exact(pr1, m, om, 0.2), pr1.sigma_exact(m, om, 0.2)) > 1e-3


def test_sign_of_imaginary_part():
    s, pr = tiny()
    om = np.linspace(-20, 20, 41)
    m = int(s.qp_states[0])
    d_ha = 0.1 / HARTREE_EV
    coeffs = T.lanczos_coeffs_tda(pr, m, 8)
    for n, (a, b, n2) in enumerate(coeffs):
        eta = occupation_sign(n, pr.n_occ)
        sig = T.sigma_n_tda_from_tridiag(a, b, n2, om / HARTREE_EV, pr.eps[n], eta, d_ha)
        assert np.all(eta * sig.imag >= 0)
