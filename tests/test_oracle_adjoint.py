"""Pins of the oracle's derivatives of Sigma_c (used to check the GPU VJP).

* the closed-form Daleckii-Krein gradient of the L -> N_vc limit with respect
  to every orbital energy equals central finite differences of that limit;
* Lanczos run to full dimension (exact Krylov space) has the same derivative;
* the explicit z_n dependence: d Sigma(w, n)/d e_n at fixed C and P equals
  -d Sigma(w, n)/d w.
"""
import numpy as np

import gw_inputs as gi
import oracle
from oracle import adjoint as A
from oracle.sigma import HARTREE_EV, Problem


def tiny(n_occ=2, n_emp=3, seed=21):
    wl = gi.workload("grid24_v8c32", name="tiny", seed=seed, grid=(8, 8, 8), box=5.0,
                     n_occ=n_occ, n_emp=n_emp, smooth_sigma=1.0)
    s = gi.make_system(wl)
    pr = Problem(s.phi, s.energies_ev, wl.n_occ, wl.grid, wl.h)
    lo, hi = oracle.default_interval(pr, margin=0.05)
    return s, wl, lo, hi


def test_dk_energy_gradient_matches_fd():
    s, wl, lo, hi = tiny()
    qp = s.qp_states
    om = np.linspace(-10, 10, 7)
    rng = np.random.default_rng(3)
    G = rng.standard_normal((len(qp), len(om))) + 1j * rng.standard_normal((len(qp), len(om)))
    fwd = lambda e: A.loss(A.sigma_dg_states(s.phi, e, wl.n_occ, wl.grid, wl.h, qp, om, 0.3,
                                              lo, hi, 7), G)
    grad = A.dk_energy_gradient(s.phi, s.energies_ev, wl.n_occ, wl.grid, wl.h, qp, om, 0.3,
                                lo, hi, 7, G)
    for a in range(wl.n_orb):
        e1 = np.zeros(wl.n_orb)
        e1[a] = 1.0
        fd = A.fd_directional(fwd, s.energies_ev, e1, 1e-4)
        assert abs(fd - grad[a]) <= 1e-6 * max(1.0, np.max(np.abs(grad))), (a, fd, grad[a])
    d = rng.standard_normal(wl.n_orb)
    assert abs(A.fd_directional(fwd, s.energies_ev, d, 1e-4) - grad @ d) <= 1e-6 * np.sum(np.abs(grad))


def test_full_length_lanczos_has_the_same_derivative():
    s, wl, lo, hi = tiny()
    qp = s.qp_states[:1]
    om = np.linspace(-8, 8, 5)
    G = np.ones((1, len(om))) * (0.3 - 0.7j)
    nvc = wl.n_vc
    fl = lambda e: A.loss(A.sigma_states(s.phi, e, wl.n_occ, wl.grid, wl.h, qp, om, 0.3, nvc,
                                          lo, hi, 7, reorth="full"), G)
    fd_ = lambda e: A.loss(A.sigma_dg_states(s.phi, e, wl.n_occ, wl.grid, wl.h, qp, om, 0.3,
                                              lo, hi, 7), G)
    d = np.random.default_rng(4).standard_normal(wl.n_orb)
    a = A.fd_directional(fl, s.energies_ev, d, 1e-4)
    b = A.fd_directional(fd_, s.energies_ev, d, 1e-4)
    assert abs(a - b) <= 1e-6 * abs(b)


def test_explicit_energy_dependence_is_minus_omega_derivative():
    s, wl, lo, hi = tiny()
    pr = Problem(s.phi, s.energies_ev, wl.n_occ, wl.grid, wl.h)
    m = int(s.qp_states[0])
    coeffs = pr.lanczos_coeffs(m, 5, lo, hi, 7)
    n = 3
    a, b, n2 = coeffs[n]
    from oracle import sigma as S
    om = np.linspace(-5, 5, 9) / HARTREE_EV
    d = 0.3 / HARTREE_EV
    h = 1e-6
    de = (S.sigma_n_from_tridiag(a, b, n2, om, pr.eps[n] + h, pr.eta(n), d)
          - S.sigma_n_from_tridiag(a, b, n2, om, pr.eps[n] - h, pr.eta(n), d)) / (2 * h)
    dw = (S.sigma_n_from_tridiag(a, b, n2, om + h, pr.eps[n], pr.eta(n), d)
          - S.sigma_n_from_tridiag(a, b, n2, om - h, pr.eps[n], pr.eta(n), d)) / (2 * h)
    assert np.max(np.abs(de + dw)) <= 1e-6 * np.max(np.abs(dw))
