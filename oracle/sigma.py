"""Correlation self-energy Sigma_c(omega): closed forms and the Lanczos method
(oracle; test infrastructure only).

Notation (paper): QP state m, summed intermediate state n, occupation sign
eta_n = +1 (occupied) / -1 (empty), broadening delta > 0,
z_n = omega - e_n - i eta_n delta (Eq. 11).

* Eq. 7:  Sigma_mm(w) = sum_n sum_s (W^s_nm)^2 / (w - e_n + eta_n (Omega_s - i delta)),
  with W^s_nm = <P_nm|Z^s> Omega_s^-1/2 (Eq. 9).
* Eq. 11: Sigma_mm(w, n) = (1/z_n) sum_s <P|Z^s>^2 [1/Omega_s - 1/(Omega_s + eta_n z_n)].
* Eq. 12: Sigma_mm(w, n) = (1/z_n) <P| D^-1 - (D + eta_n z_n)^-1 |P>.
* Eq. 13: L Lanczos steps on D from P give the tridiagonal D_L (a_k, b_k).
* Eq. 14: <P|(zeta - D)^-1|P> ~ ||P||^2 / (zeta - a_0 - b_1^2/(zeta - a_1 - ...)).

Assembly of Eq. 12 from the continued fraction.  With
R(zeta) = <P|(zeta - D)^-1|P>,  R(0) = -<P|D^-1|P> and
R(-eta_n z_n) = -<P|(D + eta_n z_n)^-1|P>, so

    Sigma_mm(w, n) = [R(-eta_n z_n) - R(0)] / z_n.

Both evaluation points lie off the spectrum of D (Im(-eta_n z_n) = +delta,
and 0 lies below the positive spectrum), so the continued fraction never
divides by zero.

Readings: Eq. 14 is printed without the ||P||^2 factor and with "z -" missing
at its third level; it is read as the standard Haydock fraction.  L (the
``n_lanczos`` argument) is the number of D-matvecs, i.e. the number of
diagonal entries a_0..a_{L-1}.  The fraction is truncated plainly (no
terminator).  Reorthogonalisation is not described in the paper (it notes only
that resolvents do not suffer from ghost eigenvalues); "full" is two-pass
classical Gram-Schmidt against all previous Lanczos vectors, done after the
three-term update and before the norm.  Breakdown: the recurrence ends when
b_{k+1} <= 1e-12 * max_{j<=k} |a_j|; ||P|| = 0 gives Sigma(w, n) = 0.
"""
from __future__ import annotations

import numpy as np

from . import casida, chebyshev

HARTREE_EV = 27.211386245988
BREAKDOWN_REL = 1e-12


def occupation_sign(n: int, n_occ: int) -> float:
    """eta_n: +1 for occupied, -1 for empty orbitals (text after Eq. 7)."""
    return 1.0 if n < n_occ else -1.0


def z_of(omega, e_n, eta_n, delta):
    """z_n = omega - e_n - i eta_n delta (text after Eq. 11)."""
    return np.asarray(omega, dtype=np.float64) - e_n - 1j * eta_n * delta


# ---------------------------------------------------------------- closed forms
def sigma_n_poles(omega, e_n, eta_n, delta, w, lam):
    """Eq. 7 for one n.  w_s = <P_nm|Z^s>^2, lam_s = pole energy Omega_s;
    (W^s)^2 = w_s / lam_s (Eq. 9)."""
    om = np.asarray(omega, dtype=np.float64)[:, None]
    wsq = (w / lam)[None, :]
    den = om - e_n + eta_n * (lam[None, :] - 1j * delta)
    return np.sum(wsq / den, axis=1)


def sigma_n_eq11(omega, e_n, eta_n, delta, w, lam):
    """Eq. 11 for one n."""
    z = z_of(omega, e_n, eta_n, delta)[:, None]
    term = 1.0 / lam[None, :] - 1.0 / (lam[None, :] + eta_n * z)
    return np.sum(w[None, :] * term, axis=1) / z[:, 0]


def sigma_n_resolvent_dense(dmat, p, omega, e_n, eta_n, delta):
    """Eq. 12 for one n with explicit linear solves on the dense matrix D."""
    n = dmat.shape[0]
    eye = np.eye(n)
    base = p @ np.linalg.solve(dmat, p)
    out = np.empty(len(omega), dtype=np.complex128)
    for i, z in enumerate(z_of(omega, e_n, eta_n, delta)):
        shifted = p.astype(np.complex128) @ np.linalg.solve(dmat + eta_n * z * eye, p.astype(np.complex128))
        out[i] = (base - shifted) / z
    return out


# ---------------------------------------------------------------- Lanczos (Eq. 13)
def lanczos(matvec, p, n_steps: int, reorth: str = "full"):
    """Lanczos tridiagonalisation of a symmetric operator from start vector p.

    Returns (a, b, norm2): a = [a_0..a_{L'-1}], b = [b_1..b_{L'-1}],
    norm2 = ||p||^2, with L' <= n_steps (shorter only on breakdown).

    Step k: w = D q_k; a_k = q_k.w; w -= a_k q_k + b_k q_{k-1};
    [reorthogonalise]; b_{k+1} = ||w||; q_{k+1} = w / b_{k+1}.
    """
    p = np.asarray(p, dtype=np.float64)
    norm2 = float(p @ p)
    if norm2 == 0.0 or n_steps <= 0:
        return np.zeros(0), np.zeros(0), norm2
    q = p / np.sqrt(norm2)
    q_prev = np.zeros_like(q)
    b_k = 0.0
    basis = [q]
    a_list, b_list = [], []
    amax = 0.0
    for k in range(n_steps):
        w = matvec(q)
        a_k = float(q @ w)
        a_list.append(a_k)
        amax = max(amax, abs(a_k))
        if k == n_steps - 1:
            break
        w = w - a_k * q - b_k * q_prev
        if reorth == "full":
            qm = np.array(basis)
            for _ in range(2):
                w = w - qm.T @ (qm @ w)
        elif reorth == "local":
            for _ in range(2):
                w = w - q * (q @ w)
                w = w - q_prev * (q_prev @ w)
        elif reorth != "none":
            raise ValueError(reorth)
        b_next = float(np.sqrt(w @ w))
        if b_next <= BREAKDOWN_REL * amax:
            break
        b_list.append(b_next)
        q_prev, q = q, w / b_next
        b_k = b_next
        basis.append(q)
    return np.array(a_list), np.array(b_list), norm2


def stieltjes(lam, w, n_steps: int, reorth: str = "full"):
    """Lanczos on the discrete measure sum_s w_s delta(x - lam_s): the
    recurrence on diag(lam) from start vector sqrt(w).  In exact arithmetic
    identical to Lanczos on D from P when lam, w are D's eigenvalues and the
    squared overlaps <P|Z^s>^2."""
    lam = np.asarray(lam, dtype=np.float64)
    return lanczos(lambda v: lam * v, np.sqrt(np.asarray(w, dtype=np.float64)),
                   n_steps, reorth)


# ---------------------------------------------------------------- Eq. 14
def continued_fraction(a, b, norm2, zeta):
    """R(zeta) = ||P||^2 / (zeta - a_0 - b_1^2/(zeta - a_1 - ...)), by the
    backward recurrence t = zeta - a_{L-1}; t = zeta - a_k - b_{k+1}^2 / t."""
    zeta = np.asarray(zeta, dtype=np.complex128)
    if len(a) == 0:
        return np.zeros_like(zeta)
    t = zeta - a[-1]
    for k in range(len(a) - 2, -1, -1):
        t = zeta - a[k] - b[k] ** 2 / t
    return norm2 / t


def tridiag_matrix(a, b):
    return np.diag(a) + np.diag(b, 1) + np.diag(b, -1)


def tridiag_resolvent_dense(a, b, norm2, zeta):
    """||P||^2 [(zeta - T)^-1]_00 by explicit solves (pin for Eq. 14)."""
    t = tridiag_matrix(a, b)
    n = len(a)
    e0 = np.zeros(n)
    e0[0] = 1.0
    out = np.empty(np.size(zeta), dtype=np.complex128)
    for i, z in enumerate(np.atleast_1d(zeta)):
        out[i] = norm2 * np.linalg.solve(z * np.eye(n) - t, e0.astype(np.complex128))[0]
    return out


def sigma_n_from_tridiag(a, b, norm2, omega, e_n, eta_n, delta):
    """Sigma_mm(w, n) = [R(-eta_n z_n) - R(0)] / z_n  (Eq. 12 with Eq. 14)."""
    z = z_of(omega, e_n, eta_n, delta)
    if norm2 == 0.0 or len(a) == 0:
        return np.zeros_like(z)
    r0 = continued_fraction(a, b, norm2, 0.0)
    rz = continued_fraction(a, b, norm2, -eta_n * z)
    return (rz - r0) / z


# ---------------------------------------------------------------- a full problem
class Problem:
    """All oracle quantities of one system (hartree internally)."""

    def __init__(self, phi, energies_ev, n_occ, shape, h, kernel_scale=1.0,
                 dense=True):
        self.phi = np.asarray(phi, dtype=np.float64)
        self.n_occ = int(n_occ)
        self.n_orb = self.phi.shape[0]
        self.shape = tuple(shape)
        self.h = float(h)
        self.dv = self.h ** 3
        self.scale = float(kernel_scale)
        self.eps = np.asarray(energies_ev, dtype=np.float64) / HARTREE_EV
        self.delta = casida.delta_pairs(self.eps, self.n_occ)
        self._k = None
        self._c = None
        self._eig = None
        self.k_asym = None
        if dense:
            self.build_dense()

    # dense operators ------------------------------------------------------
    def build_dense(self):
        self._k, self.k_asym = casida.hartree_matrix(
            self.phi, self.n_occ, self.shape, self.h, self.scale)
        self._c = casida.casida_c(self.delta, self._k)

    @property
    def K(self):
        if self._k is None:
            self.build_dense()
        return self._k

    @property
    def C(self):
        if self._c is None:
            self.build_dense()
        return self._c

    def eig(self):
        """(Omega_s^2, Z) from eigh of C (Eq. 4)."""
        if self._eig is None:
            self._eig = np.linalg.eigh(self.C)
        return self._eig

    def coupling(self, m, n_list=None):
        """[N_orb, N_vc] array of P_nm for all n (or [len(n_list), N_vc])."""
        return casida.coupling_vectors_for_state(
            self.phi, m, self.n_occ, self.shape, self.h, self.delta, self.scale, n_list)

    def apply_c(self, x):
        return casida.apply_c(self.phi, self.n_occ, self.shape, self.h,
                              self.delta, x, self.scale)

    def eta(self, n):
        return occupation_sign(n, self.n_occ)

    # Sigma, sum over n (Eq. 10), in eV -------------------------------------
    def sigma_exact(self, m, omega_ev, delta_ev):
        """Eq. 7 with the exact eigenpairs of C (the physics reference)."""
        om2, z = self.eig()
        om = np.sqrt(om2)
        pm = self.coupling(m)
        w_all = (pm @ z) ** 2
        w_ha = np.asarray(omega_ev) / HARTREE_EV
        d_ha = delta_ev / HARTREE_EV
        tot = np.zeros(len(w_ha), dtype=np.complex128)
        for n in range(self.n_orb):
            tot += sigma_n_poles(w_ha, self.eps[n], self.eta(n), d_ha, w_all[n], om)
        return tot * HARTREE_EV

    def sigma_dg(self, m, omega_ev, delta_ev, lo, hi, g):
        """Eq. 12 with D replaced by p_g(C) exactly (the L -> N_vc limit):
        poles at lam_s = p_g(Omega_s^2) with residues w_s / lam_s."""
        om2, z = self.eig()
        c = chebyshev.sqrt_coeffs(lo, hi, g)
        lam = chebyshev.eval_scalar(c, lo, hi, om2)
        pm = self.coupling(m)
        w_all = (pm @ z) ** 2
        w_ha = np.asarray(omega_ev) / HARTREE_EV
        d_ha = delta_ev / HARTREE_EV
        tot = np.zeros(len(w_ha), dtype=np.complex128)
        for n in range(self.n_orb):
            tot += sigma_n_poles(w_ha, self.eps[n], self.eta(n), d_ha, w_all[n], lam)
        return tot * HARTREE_EV

    def dg_matrix(self, lo, hi, g):
        """Dense D_g = p_g(C)."""
        c = chebyshev.sqrt_coeffs(lo, hi, g)
        return chebyshev.eval_matrix(c, lo, hi, self.C)

    def lanczos_coeffs(self, m, n_lanczos, lo, hi, g, reorth="full",
                       route="dense", n_list=None):
        """(a, b, ||P||^2) for every n (or n_list) of QP state m.

        route "dense":   Lanczos on the dense D_g = p_g(C) from P_nm (Eq. 13).
        route "measure": Stieltjes recurrence on the spectral measure of D_g
                         seen from P_nm (same result in exact arithmetic).
        route "matfree": Lanczos on p_g(C) applied by the Chebyshev recurrence
                         with matrix-free C x (for sizes where C is too big).
        """
        ns = list(range(self.n_orb)) if n_list is None else list(n_list)
        pm = self.coupling(m, ns)
        out = []
        if route == "dense":
            dg = self.dg_matrix(lo, hi, g)
            for i, _ in enumerate(ns):
                out.append(lanczos(lambda v: dg @ v, pm[i], n_lanczos, reorth))
        elif route == "measure":
            om2, z = self.eig()
            c = chebyshev.sqrt_coeffs(lo, hi, g)
            lam = chebyshev.eval_scalar(c, lo, hi, om2)
            for i, _ in enumerate(ns):
                out.append(stieltjes(lam, (pm[i] @ z) ** 2, n_lanczos, reorth))
        elif route == "matfree":
            c = chebyshev.sqrt_coeffs(lo, hi, g)
            for i, _ in enumerate(ns):
                out.append(lanczos(lambda v: chebyshev.apply(c, lo, hi, self.apply_c, v),
                                   pm[i], n_lanczos, reorth))
        else:
            raise ValueError(route)
        return out

    def sigma_lanczos(self, m, omega_ev, delta_ev, n_lanczos, lo, hi, g,
                      reorth="full", route="dense"):
        """Sigma_L: the method's result, Lanczos + continued fraction,
        summed over n (Eq. 10), eV."""
        coeffs = self.lanczos_coeffs(m, n_lanczos, lo, hi, g, reorth, route)
        w_ha = np.asarray(omega_ev) / HARTREE_EV
        d_ha = delta_ev / HARTREE_EV
        tot = np.zeros(len(w_ha), dtype=np.complex128)
        for n, (a, b, nrm2) in enumerate(coeffs):
            tot += sigma_n_from_tridiag(a, b, nrm2, w_ha, self.eps[n], self.eta(n), d_ha)
        return tot * HARTREE_EV

    def spectral_bounds(self):
        om2, _ = self.eig()
        return float(om2[0]), float(om2[-1])


def default_interval(problem: Problem, margin: float = 1e-3):
    """The interval used by tests: lo = (min Delta)^2, a rigorous lower bound
    since K is PSD, and hi = max Omega^2 (1 + margin) from the eigenvalues."""
    lo = float(np.min(problem.delta) ** 2)
    _, top = problem.spectral_bounds()
    return lo, top * (1.0 + margin)
