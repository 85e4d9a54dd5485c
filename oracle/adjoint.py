"""Derivatives of Sigma_c for checking the GPU vector-Jacobian product
(oracle; test infrastructure only).

The scalar differentiated is

    l = sum_{q, w} Re( conj(G_qw) Sigma_q(w) )        (Sigma in eV)

for given complex cotangents G.  Conventions: orbitals are free variables
(no orthonormality constraint), occupations are fixed, and the Chebyshev
interval [lo, hi] with its coefficients is held fixed.

* ``fd_directional``: central finite difference of any forward along a
  direction (the plain definition of a directional derivative).
* ``dk_energy_gradient``: closed-form gradient with respect to every orbital
  energy of the L -> N_vc limit Sigma_Dg (poles at p_g(Omega_s^2)), by the
  Daleckii-Krein formula for the derivative of a matrix function:
  d[P^T F(C) P] = (Z^T P)^T (F^[1] o Z^T dC Z) (Z^T P) with the first divided
  differences F^[1]_st = (F(l_s) - F(l_t)) / (l_s - l_t) (F'(l_s) when equal),
  plus the explicit dependence of z_n and of P_nm = (nm|vc) Delta^1/2 on the
  energies.  Used at tiny sizes to pin the finite differences.
"""
from __future__ import annotations

import numpy as np

from . import chebyshev
from .sigma import HARTREE_EV, Problem, occupation_sign


def loss(sig, G) -> float:
    return float(np.sum(np.real(np.conj(G) * sig)))


def sigma_states(phi, eps_ev, n_occ, shape, h, qp, omega_ev, delta_ev, n_lanczos, lo, hi,
                 g, reorth="none", route="dense"):
    """Sigma_q(w) (eV) for every QP state in qp by the Lanczos method."""
    pr = Problem(phi, eps_ev, n_occ, shape, h, dense=(route != "matfree"))
    return np.array([pr.sigma_lanczos(int(m), omega_ev, delta_ev, n_lanczos, lo, hi, g,
                                      reorth=reorth, route=route) for m in qp])


def sigma_dg_states(phi, eps_ev, n_occ, shape, h, qp, omega_ev, delta_ev, lo, hi, g):
    """The L -> N_vc limit (exact p_g(C) resolvent) for every QP state."""
    pr = Problem(phi, eps_ev, n_occ, shape, h)
    return np.array([pr.sigma_dg(int(m), omega_ev, delta_ev, lo, hi, g) for m in qp])


def fd_directional(fun, x, dx, step):
    """(f(x + step dx) - f(x - step dx)) / (2 step)."""
    return (fun(x + step * dx) - fun(x - step * dx)) / (2.0 * step)


def _divided_differences(fvals, dfvals, lam):
    d = lam[:, None] - lam[None, :]
    num = fvals[:, None] - fvals[None, :]
    same = np.abs(d) <= 1e-13 * np.maximum(np.abs(lam[:, None]), 1e-300)
    out = np.where(same, 0.5 * (dfvals[:, None] + dfvals[None, :]),
                   num / np.where(same, 1.0, d))
    return out


def dk_energy_gradient(phi, eps_ev, n_occ, shape, h, qp, omega_ev, delta_ev, lo, hi, g, G):
    """d l / d eps_a (per eV) for the L -> N_vc limit, all a."""
    pr = Problem(phi, eps_ev, n_occ, shape, h)
    nv, nc = n_occ, pr.n_orb - n_occ
    delta = pr.delta
    sd = np.sqrt(delta)
    om2, z = pr.eig()
    c = chebyshev.sqrt_coeffs(lo, hi, g)
    lam = chebyshev.eval_scalar(c, lo, hi, om2)
    # p'(x) from the Chebyshev series: d/dx T_j(t) = j U_{j-1}(t) dt/dx
    t = (2 * om2 - (hi + lo)) / (hi - lo)
    u_prev, u_cur = np.zeros_like(t), np.ones_like(t)   # U_{-1}, U_0
    dlam = np.zeros_like(t)
    for j in range(1, g + 1):
        dlam += c[j] * j * u_cur
        u_prev, u_cur = u_cur, 2 * t * u_cur - u_prev
    dlam *= 2.0 / (hi - lo)
    w_ha = np.asarray(omega_ev) / HARTREE_EV
    d_ha = delta_ev / HARTREE_EV
    k = pr.K
    grad = np.zeros(pr.n_orb)
    # dC / d eps_a and dP / d eps_a through Delta (dDelta_vc/d eps_a = [a=c] - [a=v])
    ddelta = np.zeros((pr.n_orb, nv * nc))
    for v in range(nv):
        for cc in range(nc):
            ddelta[v, v * nc + cc] -= 1.0
            ddelta[nv + cc, v * nc + cc] += 1.0
    for qi, m in enumerate(qp):
        pm = pr.coupling(int(m))
        kv = pm / sd[None, :]                  # (nm|vc)
        for n in range(pr.n_orb):
            eta = occupation_sign(n, n_occ)
            y = z.T @ pm[n]
            for wi, om in enumerate(w_ha):
                zz = om - pr.eps[n] - 1j * eta * d_ha
                cfac = np.conj(G[qi, wi]) * HARTREE_EV
                f = (1.0 / lam - 1.0 / (lam + eta * zz)) / zz
                # dF/dx through lam(x) = p(x)
                dfl = (-1.0 / lam ** 2 + 1.0 / (lam + eta * zz) ** 2) / zz
                df = dfl * dlam
                f1 = _divided_differences(f, df, om2)
                # explicit z dependence: dz/d eps_n = -1
                dfz = (-(1.0 / lam - 1.0 / (lam + eta * zz)) / zz ** 2
                       + (eta / (lam + eta * zz) ** 2) / zz)
                grad[n] += np.real(cfac * (-np.sum(y * y * dfz)))
                # through Delta: C and P
                for a in range(pr.n_orb):
                    dd = ddelta[a]
                    if not np.any(dd):
                        continue
                    dsd = dd / (2 * sd)
                    dc = (np.diag(2 * delta * dd)
                          + 2 * (dsd[:, None] * k * sd[None, :] + sd[:, None] * k * dsd[None, :]))
                    dcz = z.T @ dc @ z
                    term = y @ (f1 * dcz) @ y
                    dp = kv[n] * dsd
                    term += 2 * (z.T @ dp) @ (f * y)
                    grad[a] += np.real(cfac * term)
    return grad / HARTREE_EV
