"""Tamm-Dancoff variant of Sigma_c (oracle; test infrastructure only).

The paper's closing discussion notes that setting B = 0 in the RPA Casida
matrix leaves the Hermitian matrix A alone, so a standard Lanczos run on A
serves.  Written out with the paper's notation:

* A_{vc,v'c'} = (e_c - e_v) delta_vv' delta_cc' + (vc|v'c')   (Casida A, RPA),
  A X^s = X^s Omega_s with orthonormal X^s.
* The residue of the pole s for the pair (n, m) is <k_nm|X^s>^2, where
  (k_nm)_vc = (nm|vc): the TDA transition density has no (Delta/Omega)^1/2
  factor, unlike W^s_nm of the full method.
* Eq. 7 then reads
      Sigma_mm(w) = sum_n sum_s <k_nm|X^s>^2 / (w - e_n + eta_n (Omega_s - i delta)).
* With z_n = w - e_n - i eta_n delta, the denominator is
  z_n + eta_n Omega_s = -eta_n (-eta_n z_n - Omega_s), so
      Sigma_mm(w, n) = -eta_n R_A(-eta_n z_n),
      R_A(zeta) = <k_nm|(zeta - A)^-1|k_nm>,
  one resolvent per (m, n) instead of the difference of two in Eq. 12, and
  no square root: L Lanczos steps on A from k_nm and the continued fraction
  of Eq. 14 give R_A.

Readings: the same kernel, normalisation, units, reorthogonalisation and
breakdown rules as the full method (see ``sigma``).
"""
from __future__ import annotations

import numpy as np

from . import casida
from .sigma import (HARTREE_EV, Problem, continued_fraction, lanczos, occupation_sign, z_of)


def tda_matrix(pr: Problem) -> np.ndarray:
    """Dense A = Delta + K (Casida A with the RPA kernel)."""
    return np.diag(pr.delta) + pr.K


def eri_vectors(pr: Problem, m: int, n_list=None) -> np.ndarray:
    """(k_nm)_vc = (nm|vc) for every n (or n_list), shape [len, N_vc]."""
    ns = range(pr.n_orb) if n_list is None else list(n_list)
    return np.array([casida.eri_vc(pr.phi, n, m, pr.n_occ, pr.shape, pr.h, pr.scale)
                     for n in ns])


def sigma_tda_exact(pr: Problem, m: int, omega_ev, delta_ev) -> np.ndarray:
    """Eq. 7 in the TDA from the eigenpairs of A (eV)."""
    om, x = np.linalg.eigh(tda_matrix(pr))
    k = eri_vectors(pr, m)
    w_all = (k @ x) ** 2
    w_ha = np.asarray(omega_ev, dtype=np.float64) / HARTREE_EV
    d_ha = delta_ev / HARTREE_EV
    tot = np.zeros(len(w_ha), dtype=np.complex128)
    for n in range(pr.n_orb):
        eta = occupation_sign(n, pr.n_occ)
        den = (w_ha[:, None] - pr.eps[n] + eta * (om[None, :] - 1j * d_ha))
        tot += np.sum(w_all[n][None, :] / den, axis=1)
    return tot * HARTREE_EV


def sigma_tda_dense_resolvent(pr: Problem, m: int, omega_ev, delta_ev) -> np.ndarray:
    """The same quantity by explicit solves, Sigma(w, n) = <k|(z_n + eta_n A)^-1|k>
    (no eigendecomposition; a pin for sigma_tda_exact)."""
    a = tda_matrix(pr)
    k = eri_vectors(pr, m)
    w_ha = np.asarray(omega_ev, dtype=np.float64) / HARTREE_EV
    d_ha = delta_ev / HARTREE_EV
    eye = np.eye(a.shape[0])
    tot = np.zeros(len(w_ha), dtype=np.complex128)
    for n in range(pr.n_orb):
        eta = occupation_sign(n, pr.n_occ)
        for i, w in enumerate(w_ha):
            z = w - pr.eps[n] - 1j * eta * d_ha
            tot[i] += k[n] @ np.linalg.solve(z * eye + eta * a, k[n].astype(np.complex128))
    return tot * HARTREE_EV


def lanczos_coeffs_tda(pr: Problem, m: int, n_lanczos: int, reorth="full", n_list=None,
                       route="dense"):
    """(a, b, ||k||^2) for every n (or n_list): Lanczos on A from k_nm.
    route "dense" uses the dense A; "matfree" applies A x = Delta x + K x with
    the matrix-free Coulomb product."""
    ks = eri_vectors(pr, m, n_list)
    out = []
    if route == "dense":
        a = tda_matrix(pr)
        for k in ks:
            out.append(lanczos(lambda v: a @ v, k, n_lanczos, reorth))
    elif route == "matfree":
        for k in ks:
            out.append(lanczos(lambda v: pr.delta * v + casida.apply_k(
                pr.phi, pr.n_occ, pr.shape, pr.h, v, pr.scale), k, n_lanczos, reorth))
    else:
        raise ValueError(route)
    return out


def sigma_n_tda_from_tridiag(a, b, norm2, omega, e_n, eta_n, delta):
    """Sigma_mm(w, n) = -eta_n R_A(-eta_n z_n) from the Lanczos coefficients."""
    z = z_of(omega, e_n, eta_n, delta)
    if norm2 == 0.0 or len(a) == 0:
        return np.zeros_like(z)
    return -eta_n * continued_fraction(a, b, norm2, -eta_n * z)


def sigma_tda_lanczos(pr: Problem, m: int, omega_ev, delta_ev, n_lanczos: int,
                      reorth="full", route="dense") -> np.ndarray:
    """The Lanczos TDA result summed over n (Eq. 10), eV."""
    coeffs = lanczos_coeffs_tda(pr, m, n_lanczos, reorth, route=route)
    w_ha = np.asarray(omega_ev, dtype=np.float64) / HARTREE_EV
    d_ha = delta_ev / HARTREE_EV
    tot = np.zeros(len(w_ha), dtype=np.complex128)
    for n, (a, b, nrm2) in enumerate(coeffs):
        tot += sigma_n_tda_from_tridiag(a, b, nrm2, w_ha, pr.eps[n],
                                        occupation_sign(n, pr.n_occ), d_ha)
    return tot * HARTREE_EV
