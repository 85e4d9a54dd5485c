"""Off-diagonal self-energy elements Sigma_mm'(omega) (oracle; test
infrastructure only).

The paper evaluates the diagonal elements and points to a band Lanczos for
off-diagonal ones (its closing remarks on Meyer and Pal's band method).
Written out here:

* exact: Eq. 7 with the squared residue |W^s_nm|^2 replaced by the product
  W^s_nm W^s_nm' of the residues of the two states (the same pole energies
  Omega_s; W^s_nm = P_nm . Z^s / sqrt(Omega_s) as in Eq. 9);
* with D replaced by p_g(C): the same, with poles at p_g(Omega_s^2);
* the method: Sigma(omega, n) of Eqs. 12 and 14 is a quadratic form
  F_n(P) = P^T f_n(D) P in the start vector, so the bilinear form follows
  from two quadratic forms, P^T f q = [F(P + q) - F(P - q)] / 4, each
  computed by the Lanczos route of the diagonal elements from the start
  vector P_nm + P_nm' or P_nm - P_nm'.  (Reading: the polarisation identity
  in place of a block recurrence; both give the same bilinear form, this one
  with two scalar recurrences.)
"""
from __future__ import annotations

import numpy as np

from . import chebyshev
from .sigma import (HARTREE_EV, Problem, lanczos, sigma_n_from_tridiag, sigma_n_poles,
                    stieltjes)


def _sum_poles(pr: Problem, m, m2, omega_ev, delta_ev, lam, om2z):
    z = om2z
    w_all = (pr.coupling(m) @ z) * (pr.coupling(m2) @ z)
    w_ha = np.asarray(omega_ev) / HARTREE_EV
    d_ha = delta_ev / HARTREE_EV
    tot = np.zeros(len(w_ha), dtype=np.complex128)
    for n in range(pr.n_orb):
        tot += sigma_n_poles(w_ha, pr.eps[n], pr.eta(n), d_ha, w_all[n], lam)
    return tot * HARTREE_EV


def sigma_exact_offdiag(pr: Problem, m, m2, omega_ev, delta_ev):
    """Eq. 7 with W^s_nm W^s_nm' and the exact eigenpairs of C (eV)."""
    om2, z = pr.eig()
    return _sum_poles(pr, m, m2, omega_ev, delta_ev, np.sqrt(om2), z)


def sigma_dg_offdiag(pr: Problem, m, m2, omega_ev, delta_ev, lo, hi, g):
    """As sigma_exact_offdiag with D = p_g(C): poles at p_g(Omega_s^2)."""
    om2, z = pr.eig()
    lam = chebyshev.eval_scalar(chebyshev.sqrt_coeffs(lo, hi, g), lo, hi, om2)
    return _sum_poles(pr, m, m2, omega_ev, delta_ev, lam, z)


def sigma_lanczos_offdiag(pr: Problem, m, m2, omega_ev, delta_ev, n_lanczos, lo, hi, g,
                          reorth="full", route="dense"):
    """The method's Sigma_mm' (eV): per n, Lanczos on p_g(C) from
    P_nm + P_nm' and from P_nm - P_nm', continued fractions, and a quarter of
    the difference, summed over n."""
    pa, pb = pr.coupling(m), pr.coupling(m2)
    w_ha = np.asarray(omega_ev) / HARTREE_EV
    d_ha = delta_ev / HARTREE_EV
    c = chebyshev.sqrt_coeffs(lo, hi, g)
    if route == "dense":
        dg = chebyshev.eval_matrix(c, lo, hi, pr.C)
        coeffs = lambda v: lanczos(lambda x: dg @ x, v, n_lanczos, reorth)
    elif route == "measure":
        om2, z = pr.eig()
        lam = chebyshev.eval_scalar(c, lo, hi, om2)
        coeffs = lambda v: stieltjes(lam, (v @ z) ** 2, n_lanczos, reorth)
    else:
        raise ValueError(route)
    tot = np.zeros(len(w_ha), dtype=np.complex128)
    for n in range(pr.n_orb):
        sp = sigma_n_from_tridiag(*coeffs(pa[n] + pb[n]), w_ha, pr.eps[n], pr.eta(n), d_ha)
        sm = sigma_n_from_tridiag(*coeffs(pa[n] - pb[n]), w_ha, pr.eps[n], pr.eta(n), d_ha)
        tot += (sp - sm) / 4.0
    return tot * HARTREE_EV
