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


# ---------------------------------------------------------------------------
# Interpolation-point selection.
#
# The paper names ISDF but not how its points are chosen.  Reading: the
# weighted K-means (centroidal Voronoi) selection of the ISDF literature,
# written out so that every decision is exact and reproducible:
#
# * weight w(r) = (sum_v phi_v(r)^2)(sum_c phi_c(r)^2), each sum taken in
#   orbital order, then quantised to integers W(r) = floor(w / max w * 2^30 +
#   1/2) so that cluster sums are exact in any order;
# * assignment: every grid point to the nearest centroid under the periodic
#   minimum-image distance in bohr (ties to the lower centroid index);
# * update: centroid = nearest grid point to it + (sum W D) / (sum W), D the
#   integer displacement of each member from that grid point wrapped into
#   [-n/2, n/2) per axis; empty clusters keep their centroid;
# * stop when an assignment repeats the previous one, or after max_iter
#   updates;
# * the point of each non-empty cluster is its member nearest the centroid
#   (ties to the lower grid index); points are returned in increasing order.

KMEANS_QBITS = 30


def kmeans_weights(phi, n_occ):
    """w(r) = (sum_v phi_v^2)(sum_c phi_c^2) for phi [N_orb, N_r]."""
    a = np.zeros(phi.shape[1])
    b = np.zeros(phi.shape[1])
    for v in range(n_occ):
        a = a + phi[v] * phi[v]
    for c in range(n_occ, phi.shape[0]):
        b = b + phi[c] * phi[c]
    return a * b


def quantise_weights(w):
    return np.floor(w / np.max(w) * 2.0 ** KMEANS_QBITS + 0.5).astype(np.int64)


def _grid_coords(shape):
    idx = np.arange(int(np.prod(shape)))
    x, rem = np.divmod(idx, shape[1] * shape[2])
    y, z = np.divmod(rem, shape[2])
    return np.stack([x, y, z], axis=1)              # [N_r, 3] int64


def _assign(coords, cent, shape, spacing):
    """Nearest centroid of every grid point: (labels, squared distance)."""
    best = np.full(coords.shape[0], np.inf)
    lab = np.zeros(coords.shape[0], dtype=np.int64)
    cf = coords.astype(np.float64)
    for k in range(cent.shape[0]):
        d2 = None
        for a in range(3):
            n = float(shape[a])
            dx = cf[:, a] - cent[k, a]
            dx = (dx - n * np.floor(dx / n + 0.5)) * spacing[a]
            d2 = dx * dx if d2 is None else d2 + dx * dx
        upd = d2 < best
        best[upd] = d2[upd]
        lab[upd] = k
    return lab, best


def kmeans_points(w, shape, spacing, init_points, max_iter):
    """Interpolation points by weighted K-means; returns (points, n_assign).

    w: [N_r] weights; shape: (n_x, n_y, n_z); spacing: bohr per axis;
    init_points: grid indices of the initial centroids."""
    pts, _, n_assign = kmeans(w, shape, spacing, init_points, max_iter)
    return pts, n_assign


def kmeans(w, shape, spacing, init_points, max_iter):
    """(points, final centroids [K, 3] in grid units, number of assignments)."""
    W = quantise_weights(w)
    coords = _grid_coords(shape)
    cent = coords[np.asarray(init_points)].astype(np.float64)
    K = cent.shape[0]
    prev = None
    n_assign = 0
    for it in range(max_iter + 1):
        lab, best = _assign(coords, cent, shape, spacing)
        n_assign += 1
        if prev is not None and np.array_equal(lab, prev):
            break
        if it == max_iter:
            break
        prev = lab
        rc = np.floor(cent + 0.5)
        s0 = np.zeros(K, dtype=np.int64)
        np.add.at(s0, lab, W)
        new = cent.copy()
        for a in range(3):
            n = shape[a]
            D = coords[:, a] - rc[lab, a].astype(np.int64)
            D = (D + n // 2) % n - n // 2
            s1 = np.zeros(K, dtype=np.int64)
            np.add.at(s1, lab, W * D)
            na = rc[:, a] + s1.astype(np.float64) / np.where(s0 > 0, s0, 1).astype(np.float64)
            na = na - float(n) * np.floor(na / float(n))
            new[:, a] = np.where(s0 > 0, na, cent[:, a])
        cent = new
    pts = []
    for k in range(K):
        members = np.nonzero(lab == k)[0]
        if members.size:
            pts.append(int(members[np.argmin(best[members])]))
    return np.sort(np.array(pts, dtype=np.int64)), cent, n_assign


# ---------------------------------------------------------------------------
# Interpolation points by column-pivoted QR (the selection the ISDF
# literature pairs with the interpolative decomposition).  The pair-density
# matrix Z[(vc), r] = phi_v(r) phi_c(r) is too large to pivot directly, so it
# is sketched: with caller-given random matrices Gv [N_v, p] and Gc [N_c, p]
# (the random numbers are inputs, not drawn here),
#     S[k, r] = (sum_v Gv[v, k] phi_v(r)) (sum_c Gc[c, k] phi_c(r)),
# i.e. S = Gv^T Z-rows combined through the Khatri-Rao structure of Z; its
# column space follows Z's.  The points are the first n_mu pivots of
# column-pivoted Gram-Schmidt on S (Businger-Golub pivoting): at each step
# the column (grid point) with the largest residual 2-norm is taken (ties to
# the lower index), normalised, and projected out of every column.

def qrcp_sketch(phi, n_occ, gv, gc):
    """S [p, N_r] = (Gv^T phi_v) * (Gc^T phi_c), elementwise."""
    pv, pc = phi[:n_occ], phi[n_occ:]
    return (np.asarray(gv).T @ pv) * (np.asarray(gc).T @ pc)


def qrcp_pivots(s, n_mu):
    """First n_mu pivots (grid indices, in pivot order) of column-pivoted
    Gram-Schmidt on s [p, N_r]; also the residual norms at each pivot."""
    r = np.array(s, dtype=np.float64, copy=True)
    taken = np.zeros(r.shape[1], dtype=bool)
    piv, rdiag = [], []
    for _ in range(n_mu):
        nrm = np.einsum("kr,kr->r", r, r)
        nrm[taken] = -1.0
        j = int(np.argmax(nrm))           # first index of the maximum
        # a zero residual (sketch rank exhausted) is taken without projecting
        q = r[:, j] / np.sqrt(nrm[j]) if nrm[j] > 0.0 else np.zeros(r.shape[0])
        r -= np.outer(q, q @ r)
        r[:, j] = 0.0
        taken[j] = True
        piv.append(j)
        rdiag.append(float(np.sqrt(nrm[j])))
    return np.array(piv), np.array(rdiag)


def qrcp_points(phi, n_occ, n_mu, gv, gc):
    """Interpolation points (increasing grid indices) by QRCP of the sketch."""
    piv, _ = qrcp_pivots(qrcp_sketch(phi, n_occ, gv, gc), n_mu)
    return np.sort(piv)
