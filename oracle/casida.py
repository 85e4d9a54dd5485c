"""Pair-space operators of the reduced Casida problem (oracle; test only).

Definitions followed (paper, Eqs. 2-4 and the definition of P_nm before
Eq. 9), for real orbitals of a finite system:

* pairs (v, c), v occupied, c empty, flattened v-major: index v*N_c + c;
* Delta_vc = e_c - e_v  (diagonal of A - B, Eq. 2);
* K_{vc,v'c'} = (vc|v'c') = dV sum_r phi_v phi_c(r) V[phi_v' phi_c'](r)
  (Eqs. 2-3; for real orbitals (vc|c'v') = (vc|v'c'), so A = Delta + K and
  B = K);
* C = (A-B)^1/2 (A+B) (A-B)^1/2 = Delta^2 + 2 Delta^1/2 K Delta^1/2 (Eq. 4),
  because A - B = Delta is diagonal;
* (P_nm)_vc = (nm|vc) (e_c - e_v)^1/2 with
  (nm|vc) = dV sum_r phi_v phi_c(r) V[phi_n phi_m](r).

Reading (spin): the formulas carry no spin factor; K is used as printed.
``scale`` multiplies the Coulomb kernel (1 = as printed; 0 switches the
coupling off, the pin Omega = Delta).
"""
from __future__ import annotations

import numpy as np

from .poisson import poisson


def delta_pairs(eps_ha: np.ndarray, n_occ: int) -> np.ndarray:
    """Delta_vc = e_c - e_v, flattened v-major, hartree."""
    ev = eps_ha[:n_occ]
    ec = eps_ha[n_occ:]
    return (ec[None, :] - ev[:, None]).reshape(-1)


def pair_densities(phi: np.ndarray, n_occ: int) -> np.ndarray:
    """B[(v,c), r] = phi_v(r) phi_c(r), shape [N_vc, N_r]."""
    pv = phi[:n_occ]
    pc = phi[n_occ:]
    return (pv[:, None, :] * pc[None, :, :]).reshape(-1, phi.shape[1])


def hartree_matrix(phi: np.ndarray, n_occ: int, shape, h: float,
                   scale: float = 1.0, symmetrize: bool = True):
    """Dense K (Eqs. 2-3).  Returns (K, asymmetry) where asymmetry is
    ||K - K^T|| / ||K|| before symmetrisation."""
    dv = h ** 3
    b = pair_densities(phi, n_occ)
    vb = poisson(b, shape, h, scale)
    k = dv * (b @ vb.T)
    nrm = np.linalg.norm(k)
    asym = np.linalg.norm(k - k.T) / nrm if nrm > 0 else 0.0
    if symmetrize:
        k = 0.5 * (k + k.T)
    return k, asym


def casida_c(delta: np.ndarray, k: np.ndarray) -> np.ndarray:
    """C = Delta^2 + 2 Delta^1/2 K Delta^1/2 (Eq. 4)."""
    s = np.sqrt(delta)
    return np.diag(delta ** 2) + 2.0 * (s[:, None] * k * s[None, :])


def apply_k(phi: np.ndarray, n_occ: int, shape, h: float, x: np.ndarray,
            scale: float = 1.0) -> np.ndarray:
    """(K x)_vc for pair vectors x [..., N_vc] without forming K: by
    linearity of the integral, sum_{v'c'} (vc|v'c') x_{v'c'} equals
    dV sum_r phi_v phi_c(r) V[rho_x](r) with rho_x = sum x_{v'c'} phi_v' phi_c'."""
    dv = h ** 3
    nv = n_occ
    nc = phi.shape[0] - n_occ
    pv, pc = phi[:nv], phi[nv:]
    xs = x.reshape(x.shape[:-1] + (nv, nc))
    # rho_x(r) = sum_v phi_v(r) sum_c phi_c(r) x_vc
    rho = np.einsum("...vc,cr,vr->...r", xs, pc, pv, optimize=True)
    vpot = poisson(rho, shape, h, scale)
    out = dv * np.einsum("vr,...r,cr->...vc", pv, vpot, pc, optimize=True)
    return out.reshape(x.shape)


def apply_c(phi, n_occ, shape, h, delta, x, scale=1.0):
    """C x = Delta^2 x + 2 Delta^1/2 K (Delta^1/2 x) (Eq. 4), matrix-free."""
    s = np.sqrt(delta)
    return delta ** 2 * x + 2.0 * s * apply_k(phi, n_occ, shape, h, s * x, scale)


def eri_vc(phi: np.ndarray, n: int, m: int, n_occ: int, shape, h: float,
           scale: float = 1.0) -> np.ndarray:
    """(nm|vc) = dV sum_r phi_v(r) phi_c(r) V[phi_n phi_m](r) for all pairs
    (v, c), flattened v-major.  The sum over r is the matrix product
    (phi_v V) phi_c^T, so pair densities are never stored."""
    dv = h ** 3
    vnm = poisson(phi[n] * phi[m], shape, h, scale)
    pv, pc = phi[:n_occ], phi[n_occ:]
    return dv * ((pv * vnm[None, :]) @ pc.T).reshape(-1)


def coupling_vector(phi, n, m, n_occ, shape, h, delta, scale=1.0):
    """(P_nm)_vc = (nm|vc) (e_c - e_v)^1/2 (definition before Eq. 9)."""
    return eri_vc(phi, n, m, n_occ, shape, h, scale) * np.sqrt(delta)


def coupling_vectors_for_state(phi, m, n_occ, shape, h, delta, scale=1.0, n_list=None):
    """P_nm for every orbital n (the n-sum of Eq. 10), or for the n in n_list,
    shape [len, N_vc]."""
    ns = range(phi.shape[0]) if n_list is None else list(n_list)
    sd = np.sqrt(delta)
    return np.array([eri_vc(phi, n, m, n_occ, shape, h, scale) * sd for n in ns])
