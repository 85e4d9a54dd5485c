"""Sigma_c by Lanczos on C and Gauss quadrature (oracle; test infrastructure
only).

Eq. 11 writes Sigma_mm(w, n) as a sum over the eigenpairs (Omega_s^2, Z^s) of
C of <P|Z^s>^2 f(Omega_s^2) with

    f(x) = [1/sqrt(x) - 1/(sqrt(x) + eta_n z_n)] / z_n,

i.e. the spectral measure of C seen from P_nm integrated against f.  The
method of the paper replaces sqrt by a polynomial p_g so that the measure of
D = p_g(C) can be probed by Lanczos on D (Eqs. 12-14).  The same measure can
instead be probed directly: L Lanczos steps on C from P give the tridiagonal
T_L; its eigenvalues theta_k (Ritz values) and the squared first components
of its eigenvectors u_k define the L-point Gauss quadrature

    Sigma_mm(w, n) ~ ||P||^2 sum_k u_k(0)^2 f(theta_k),

which is exact for any f when L = N_vc and otherwise for polynomials of
degree < 2L.  No polynomial fit of the square root is involved.
"""
from __future__ import annotations

import numpy as np

from .sigma import HARTREE_EV, Problem, lanczos, occupation_sign, tridiag_matrix, z_of


def gauss_nodes_weights(a, b, norm2):
    """(theta_k, w_k = ||P||^2 u_k(0)^2) of the tridiagonal (a, b) by eigh."""
    if len(a) == 0 or norm2 == 0.0:
        return np.zeros(0), np.zeros(0)
    th, u = np.linalg.eigh(tridiag_matrix(np.asarray(a), np.asarray(b)))
    return th, norm2 * u[0] ** 2


def sigma_n_quadrature(theta, w, omega, e_n, eta_n, delta):
    """sum_k w_k [1/sqrt(theta_k) - 1/(sqrt(theta_k) + eta_n z_n)] / z_n."""
    z = z_of(omega, e_n, eta_n, delta)
    if len(theta) == 0:
        return np.zeros_like(z)
    om = np.sqrt(theta)[None, :]
    zz = z[:, None]
    return np.sum(w[None, :] * (1.0 / om - 1.0 / (om + eta_n * zz)), axis=1) / z


def lanczos_coeffs_c(pr: Problem, m: int, n_steps: int, reorth="full", n_list=None):
    """(a, b, ||P||^2) of Lanczos on C from P_nm for every n (or n_list)."""
    ns = list(range(pr.n_orb)) if n_list is None else list(n_list)
    pm = pr.coupling(m, ns)
    c = pr.C
    return [lanczos(lambda v: c @ v, pm[i], n_steps, reorth) for i in range(len(ns))]


def sigma_quadrature(pr: Problem, m: int, omega_ev, delta_ev, n_steps: int,
                     reorth="full") -> np.ndarray:
    """Sigma_mm(w) by Lanczos on C + Gauss quadrature, summed over n, eV."""
    w_ha = np.asarray(omega_ev, dtype=np.float64) / HARTREE_EV
    d_ha = delta_ev / HARTREE_EV
    tot = np.zeros(len(w_ha), dtype=np.complex128)
    for n, (a, b, n2) in enumerate(lanczos_coeffs_c(pr, m, n_steps, reorth)):
        th, w = gauss_nodes_weights(a, b, n2)
        tot += sigma_n_quadrature(th, w, w_ha, pr.eps[n], occupation_sign(n, pr.n_occ), d_ha)
    return tot * HARTREE_EV
