"""Exchange self-energy and quasiparticle energies (oracle; test
infrastructure only).

* Sigma^ex_mm = - sum_v (vm|vm), the frequency-independent part of
  <phi_m|Sigma^GW(w)|phi_m> = Sigma^ex_mm + Sigma^corr_mm(w) (the paper's
  self-energy split), with (vm|vm) = dV sum_r phi_v phi_m(r) V[phi_v phi_m](r)
  on the grid and the same periodic kernel as the pair integrals of the
  correlation part.
* Quasiparticle equation solved graphically on the frequency grid:
  E = e_m + Sigma^ex_mm + Re Sigma^corr_mm(E) - v_xc, i.e. the zeros of
  f(w) = e_m + Sigma^ex + Re Sigma^corr(w) - v_xc - w, located by sign changes
  between neighbouring grid points and linear interpolation; the root nearest
  to e_m is the quasiparticle energy, Z = 1 / (1 - d Re Sigma^corr / dw) there
  (slope of the interpolating segment).  v_xc comes from the mean-field
  calculation (not available here; callers pass it, 0 by default).  Energies
  in eV.
"""
from __future__ import annotations

import numpy as np

from .poisson import poisson
from .sigma import HARTREE_EV


def exchange_integral(phi, v, m, shape, h, scale=1.0) -> float:
    """(vm|vm) in hartree."""
    rho = phi[v] * phi[m]
    return float((h ** 3) * np.sum(rho * poisson(rho, shape, h, scale)))


def sigma_x(phi, n_occ, m, shape, h, scale=1.0) -> float:
    """Sigma^ex_mm = -sum_{v < n_occ} (vm|vm), eV."""
    return -HARTREE_EV * sum(exchange_integral(phi, v, m, shape, h, scale)
                             for v in range(n_occ))


def qp_solve(omega_ev, sigma_c_ev, eps_ev, sigma_x_ev, vxc_ev=0.0):
    """(E_qp, Z) from the graphical solution on the grid; (nan, nan) when
    f(w) changes sign nowhere on the grid."""
    w = np.asarray(omega_ev, dtype=np.float64)
    f = eps_ev + sigma_x_ev + np.real(np.asarray(sigma_c_ev)) - vxc_ev - w
    best = None
    for i in range(len(w) - 1):
        f0, f1 = f[i], f[i + 1]
        if f0 == 0.0:
            root, seg = w[i], i
        elif f0 * f1 < 0.0:
            root, seg = w[i] - f0 * (w[i + 1] - w[i]) / (f1 - f0), i
        else:
            continue
        if best is None or abs(root - eps_ev) < abs(best[0] - eps_ev):
            best = (root, seg)
    if best is None:
        return float("nan"), float("nan")
    root, i = best
    i = min(i, len(w) - 2)
    slope = (np.real(sigma_c_ev[i + 1]) - np.real(sigma_c_ev[i])) / (w[i + 1] - w[i])
    return float(root), float(1.0 / (1.0 - slope))
