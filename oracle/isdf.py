"""Interpolative separable density fitting of the pair densities
(oracle; test infrastructure only).

The paper factorises the pair products with auxiliary functions zeta_mu
(Eq. 15), phi_n phi_m(r) ~ sum_mu zeta_mu(r) C^mu_nm, so that the Coulomb
integrals become (kl|nm) ~ sum_ab (a|b) C^a_kl C^b_nm with the two-centre
integrals (a|b) (Eqs. 16-17), and names the interpolative separable variant
(ISDF).  Written out here:

* interpolation points r_mu (given; chosen by the caller);
* coefficients are the pair products at the points,
  C^mu_vc = phi_v(r_mu) phi_c(r_mu);
* the auxiliary functions are the least-squares fit of the pair-density
  matrix Z[r, vc] = phi_v(r) phi_c(r) by zeta C:  zeta = Z C^T (C C^T)^-1;
* (a|b) = dV sum_r zeta_a(r) V[zeta_b](r) with the same periodic kernel as K;
* K_ISDF = C^T M C replaces K inside C = Delta^2 + 2 Delta^1/2 K Delta^1/2.

Reading (the paper does not spell these out): only the (vc|v'c') integrals of
K are fitted; the coupling integrals (nm|vc) of P_nm stay exact on the grid.
"""
from __future__ import annotations

import numpy as np

from . import casida
from .poisson import poisson
from .sigma import Problem


def isdf_factors(phi, n_occ, shape, h, points, scale=1.0):
    """(Cmat [N_mu, N_vc], zeta [N_mu, N_r], M [N_mu, N_mu]) for the points."""
    points = np.asarray(points)
    z = casida.pair_densities(phi, n_occ)           # [N_vc, N_r]
    cmat = z[:, points].T                           # [N_mu, N_vc]
    zc = z.T @ cmat.T                               # Z C^T  [N_r, N_mu]
    cct = cmat @ cmat.T                             # C C^T  [N_mu, N_mu]
    zeta = np.linalg.solve(cct, zc.T)               # (C C^T)^-1 (Z C^T)^T = zeta^T
    vz = poisson(zeta, shape, h, scale)
    m = (h ** 3) * (zeta @ vz.T)
    return cmat, zeta, 0.5 * (m + m.T)


def k_isdf(phi, n_occ, shape, h, points, scale=1.0):
    """Dense K_ISDF = C^T M C."""
    cmat, _, m = isdf_factors(phi, n_occ, shape, h, points, scale)
    return cmat.T @ m @ cmat


class IsdfProblem(Problem):
    """A Problem whose K is the ISDF factorisation (the coupling vectors stay
    exact)."""

    def __init__(self, phi, energies_ev, n_occ, shape, h, points, kernel_scale=1.0):
        self.points = np.asarray(points)
        super().__init__(phi, energies_ev, n_occ, shape, h, kernel_scale, dense=True)

    def build_dense(self):
        self._k = k_isdf(self.phi, self.n_occ, self.shape, self.h, self.points, self.scale)
        self.k_asym = 0.0
        self._c = casida.casida_c(self.delta, self._k)

    def apply_c(self, x):
        return self.C @ x
