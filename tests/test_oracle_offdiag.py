"""Pins of the oracle's off-diagonal self-energy Sigma_mm'.

* with m' = m the exact form reduces to the diagonal Eq. 7 of the (separately
  pinned) diagonal oracle, and the polarised Lanczos route to the diagonal
  Lanczos route;
* Sigma_mm' = Sigma_m'm (exact and Lanczos);
* run to full length (L = N_vc) the polarised Lanczos route equals the
  pole sum with p_g(C) eigenvalues and residue products W_nm W_nm' (an
  eigendecomposition, not a recurrence);
* at short lengths it converges towards that limit.
"""
import numpy as np

import gw_inputs as gi
import oracle
from oracle import offdiag as O
from oracle.sigma import Problem


def tiny(n_occ=2, n_emp=4, seed=11):
    wl = gi.workload("grid24_v8c32", name="tiny", seed=seed, grid=(8, 8, 8), box=6.0,
                     n_occ=n_occ, n_emp=n_emp, smooth_sigma=1.0)
    s = gi.make_system(wl)
    return s, Problem(s.phi, s.energies_ev, wl.n_occ, wl.grid, wl.h)


def rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def test_diagonal_reduction():
    s, pr = tiny()
    om = np.linspace(-12, 12, 25)
    m = int(s.qp_states[0])
    assert rel(O.sigma_exact_offdiag(pr, m, m, om, 0.2), pr.sigma_exact(m, om, 0.2)) <= 1e-13
    lo, hi = oracle.default_interval(pr)
    diag = pr.sigma_lanczos(m, om, 0.2, 5, lo, hi, 7)
    assert rel(O.sigma_lanczos_offdiag(pr, m, m, om, 0.2, 5, lo, hi, 7), diag) <= 1e-12


def test_symmetric():
    s, pr = tiny(n_occ=3, n_emp=5)
    om = np.linspace(-10, 10, 21)
    m, m2 = int(s.qp_states[0]), int(s.qp_states[1])
    assert m != m2
    a = O.sigma_exact_offdiag(pr, m, m2, om, 0.3)
    assert np.max(np.abs(a)) > 1e-3
    assert rel(O.sigma_exact_offdiag(pr, m2, m, om, 0.3), a) <= 1e-13
    lo, hi = oracle.default_interval(pr)
    b = O.sigma_lanczos_offdiag(pr, m, m2, om, 0.3, 6, lo, hi, 7)
    assert rel(O.sigma_lanczos_offdiag(pr, m2, m, om, 0.3, 6, lo, hi, 7), b) <= 1e-12


def test_full_length_equals_pole_sum():
    s, pr = tiny()
    om = np.linspace(-12, 12, 25)
    m, m2 = int(s.qp_states[0]), int(s.qp_states[1])
    lo, hi = oracle.default_interval(pr)
    ref = O.sigma_dg_offdiag(pr, m, m2, om, 0.2, lo, hi, 7)
    assert np.max(np.abs(ref)) > 1e-3
    got = O.sigma_lanczos_offdiag(pr, m, m2, om, 0.2, pr.delta.size, lo, hi, 7)
    assert rel(got, ref) <= 1e-9
    got_m = O.sigma_lanczos_offdiag(pr, m, m2, om, 0.2, pr.delta.size, lo, hi, 7,
                                    route="measure")
    assert rel(got_m, ref) <= 1e-9


def test_converges_with_length():
    s, pr = tiny(n_occ=3, n_emp=8)
    om = np.linspace(-10, 10, 41)
    m, m2 = int(s.qp_states[0]), int(s.qp_states[0]) + 1
    lo, hi = oracle.default_interval(pr)
    ref = O.sigma_dg_offdiag(pr, m, m2, om, 0.3, lo, hi, 7)
    errs = [rel(O.sigma_lanczos_offdiag(pr, m, m2, om, 0.3, L, lo, hi, 7), ref)
            for L in (2, 6, 14)]
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-3
