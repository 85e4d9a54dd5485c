"""Pins of the oracle's ISDF factorisation of K.

* with as many generic points as pairs the fit is exact, so K_ISDF = K;
* the fitted pair densities interpolate: (zeta C)(r_mu) = Z(r_mu) at every
  interpolation point;
* M and K_ISDF are symmetric positive semidefinite;
* on smooth orbitals the error of K_ISDF and of Sigma falls as points are added.
"""
import numpy as np

import gw_inputs as gi
from oracle import casida
from oracle import isdf as I
from oracle.sigma import Problem


def sys_(n_occ=2, n_emp=4, grid=(8, 8, 8), box=6.0, seed=11):
    wl = gi.workload("grid24_v8c32", name="tiny", seed=seed, grid=grid, box=box,
                     n_occ=n_occ, n_emp=n_emp, smooth_sigma=1.0)
    return wl, gi.make_system(wl)


def test_exact_when_points_equal_pairs():
    wl, s = sys_()
    nvc = wl.n_occ * wl.n_emp
    pts = gi.random_grid_points(nvc, wl.n_r, seed=3)
    k_ex, _ = casida.hartree_matrix(s.phi, wl.n_occ, wl.grid, wl.h)
    k_is = I.k_isdf(s.phi, wl.n_occ, wl.grid, wl.h, pts)
    assert np.max(np.abs(k_is - k_ex)) <= 1e-9 * np.max(np.abs(k_ex))


def test_interpolates_at_points():
    wl, s = sys_(n_occ=3, n_emp=6)
    pts = gi.random_grid_points(10, wl.n_r, seed=4)
    cmat, zeta, _ = I.isdf_factors(s.phi, wl.n_occ, wl.grid, wl.h, pts)
    z = casida.pair_densities(s.phi, wl.n_occ)       # [N_vc, N_r]
    fit_at_pts = (zeta.T @ cmat)[pts]                # [N_mu, N_vc]
    assert np.max(np.abs(fit_at_pts - z[:, pts].T)) <= 1e-10 * np.max(np.abs(z))


def test_symmetric_psd():
    wl, s = sys_(n_occ=3, n_emp=6)
    pts = gi.random_grid_points(12, wl.n_r, seed=5)
    _, _, m = I.isdf_factors(s.phi, wl.n_occ, wl.grid, wl.h, pts)
    k = I.k_isdf(s.phi, wl.n_occ, wl.grid, wl.h, pts)
    for a in (m, k):
        assert np.max(np.abs(a - a.T)) <= 1e-12 * np.max(np.abs(a))
        assert np.min(np.linalg.eigvalsh(a)) >= -1e-10 * np.max(np.abs(a))


def test_error_falls_with_points():
    wl, s = sys_(n_occ=3, n_emp=8, grid=(10, 10, 10), box=7.0)
    k_ex, _ = casida.hartree_matrix(s.phi, wl.n_occ, wl.grid, wl.h)
    pr = Problem(s.phi, s.energies_ev, wl.n_occ, wl.grid, wl.h)
    om = np.linspace(-10, 10, 21)
    m = int(s.qp_states[0])
    ref = pr.sigma_exact(m, om, 0.3)
    errs_k, errs_s = [], []
    for n_mu in (6, 12, 24):
        pts = gi.random_grid_points(n_mu, wl.n_r, seed=6)
        k_is = I.k_isdf(s.phi, wl.n_occ, wl.grid, wl.h, pts)
        errs_k.append(np.linalg.norm(k_is - k_ex) / np.linalg.norm(k_ex))
        ip = I.IsdfProblem(s.phi, s.energies_ev, wl.n_occ, wl.grid, wl.h, pts)
        errs_s.append(np.max(np.abs(ip.sigma_exact(m, om, 0.3) - ref)) / np.max(np.abs(ref)))
    assert errs_k[0] > errs_k[1] > errs_k[2]
    assert errs_s[2] < errs_s[0]
    assert errs_k[2] < 1e-6           # 24 = N_vc points: exact again


# ---- interpolation-point selection (weighted K-means) ----

def test_kmeans_finds_isolated_weights():
    """All weight on K isolated grid points, centroids started one cell away
    (across the periodic boundary for some): every centroid moves onto its
    point and the points come back exactly; the move changes the cells once,
    so the third assignment is the first to repeat."""
    shape = (10, 12, 8)
    n_r = int(np.prod(shape))
    heavy = [(0, 0, 0), (5, 6, 4), (9, 11, 7), (2, 9, 1), (7, 3, 6)]
    start = [(9, 0, 0), (5, 7, 4), (0, 11, 7), (2, 9, 2), (7, 3, 5)]
    idx = lambda p: (p[0] * shape[1] + p[1]) * shape[2] + p[2]
    w = np.full(n_r, 0.0)
    for p in heavy:
        w[idx(p)] = 1.0 + 0.25 * idx(p) / n_r
    pts, n_assign = I.kmeans_points(w, shape, (0.4, 0.4, 0.4), [idx(p) for p in start], 10)
    assert list(pts) == sorted(idx(p) for p in heavy)
    assert n_assign == 3


def test_kmeans_uniform_lattice():
    """Uniform weight on an 8^3 grid, eight centroids on the lattice of
    spacing 4.  Per axis, the points 2 and 6 are equidistant from 0 and 4 and
    go to the lower centroid index, so the cells are {6, 7, 0, 1, 2} and
    {3, 4, 5} per axis, both centred on their centroid: nothing moves, the
    second assignment repeats the first, and each point is its lattice site.
    A second case on a 6-point ring with weights 1, 2, 3, 4, 5, 8 (exact after
    quantisation) follows the hand-computed Lloyd iterates: cells {4, 5, 0, 1}
    and {2, 3} give centroids 5 and 2 + 4/7, then cells {4, 5, 0} and
    {1, 2, 3} give 5 - 4/14 and 3 - 7/9, which the third assignment keeps."""
    shape = (8, 8, 8)
    trip = [(a, b, c) for a in (0, 4) for b in (0, 4) for c in (0, 4)]
    lat = [a * 64 + b * 8 + c for a, b, c in trip]
    pts, cent, n_assign = I.kmeans(np.ones(512), shape, (0.3, 0.3, 0.3), lat, 10)
    assert list(pts) == sorted(lat)
    assert np.array_equal(cent, np.array(trip, dtype=float))
    assert n_assign == 2

    w = np.array([1.0, 2.0, 3.0, 4.0, 5.0, 8.0])
    pts, cent, n_assign = I.kmeans(w, (6, 1, 1), (0.5, 0.5, 0.5), [0, 2], 10)
    assert n_assign == 3
    assert list(pts) == [2, 5]
    assert abs(cent[0, 0] - (5 - 4 / 14)) <= 1e-14 and abs(cent[1, 0] - (3 - 7 / 9)) <= 1e-14
    assert np.all(cent[:, 1:] == 0.0)


def test_kmeans_assignment_is_nearest_image():
    """Against a brute-force distance over all 27 periodic images on a small
    anisotropic grid with random centroids."""
    rng = np.random.default_rng(4)
    shape, spacing = (5, 7, 6), (0.3, 0.45, 0.35)
    coords = I._grid_coords(shape)
    cent = rng.uniform(0, 1, size=(6, 3)) * np.array(shape)
    lab, best = I._assign(coords, cent, shape, spacing)
    for r in range(coords.shape[0]):
        d = []
        for k in range(cent.shape[0]):
            imgs = [sum(((coords[r, a] - cent[k, a] + s[a] * shape[a]) * spacing[a]) ** 2
                        for a in range(3))
                    for s in np.ndindex(3, 3, 3) for s in [tuple(x - 1 for x in s)]]
            d.append(min(imgs))
        assert lab[r] == int(np.argmin(d))
        assert abs(best[r] - min(d)) <= 1e-12 * max(min(d), 1.0)


def test_kmeans_points_beat_random_points():
    """On smooth orbitals the K-means points (started from random ones) fit
    K better than the random points themselves, at two point counts."""
    wl, s = sys_(n_occ=4, n_emp=16, grid=(12, 12, 12), box=7.0, seed=9)
    k_ex, _ = casida.hartree_matrix(s.phi, wl.n_occ, wl.grid, wl.h)
    w = I.kmeans_weights(s.phi, wl.n_occ)
    for n_mu in (24, 40):
        init = gi.random_grid_points(n_mu, wl.n_r, seed=3)
        pts, _ = I.kmeans_points(w, wl.grid, (wl.h,) * 3, init, 30)
        err = lambda p: np.linalg.norm(I.k_isdf(s.phi, wl.n_occ, wl.grid, wl.h, p) - k_ex)
        assert err(pts) < 0.9 * err(init)


# ------------------------------------------------------------------ QRCP points
def _gauss(shape, seed):
    return np.random.default_rng(seed).standard_normal(shape)


def test_qrcp_sketch_is_khatri_rao_projection():
    """S[k, r] = sum_vc Gv[v, k] Gc[c, k] Z[(vc), r], by brute force."""
    wl, s = sys_(n_occ=2, n_emp=3, grid=(6, 6, 6), box=5.0)
    gv, gc = _gauss((2, 5), 1), _gauss((3, 5), 2)
    z = casida.pair_densities(s.phi, wl.n_occ)          # [(vc), r]
    w = np.array([[gv[v, k] * gc[c, k] for v in range(2) for c in range(3)] for k in range(5)])
    assert np.max(np.abs(I.qrcp_sketch(s.phi, wl.n_occ, gv, gc) - w @ z)) <= 1e-13 * np.max(np.abs(z))


def test_qrcp_pivots_match_lapack():
    """Column-pivoted Gram-Schmidt picks the same pivots as LAPACK's pivoted
    Householder QR (dgeqp3) on a generic matrix, with |R_jj| equal."""
    import scipy.linalg as sl
    a = _gauss((12, 60), 5) * np.linspace(0.2, 3.0, 60)[None, :]
    piv, rd = I.qrcp_pivots(a, 12)
    _, rr, p = sl.qr(a, pivoting=True, mode="economic")
    assert np.array_equal(piv, p[:12])
    assert np.max(np.abs(rd - np.abs(np.diag(rr)))) <= 1e-12 * rd[0]


def test_qrcp_exact_at_full_rank():
    """With as many pivots as pairs (and a sketch at least that wide), the
    QRCP points carry the whole column space of Z: K_ISDF = K."""
    wl, s = sys_()
    nvc = wl.n_occ * wl.n_emp
    pts = I.qrcp_points(s.phi, wl.n_occ, nvc, _gauss((wl.n_occ, nvc + 4), 7),
                        _gauss((wl.n_emp, nvc + 4), 8))
    assert len(set(pts.tolist())) == nvc
    k_ex, _ = casida.hartree_matrix(s.phi, wl.n_occ, wl.grid, wl.h)
    k_is = I.k_isdf(s.phi, wl.n_occ, wl.grid, wl.h, pts)
    assert np.max(np.abs(k_is - k_ex)) <= 1e-9 * np.max(np.abs(k_ex))


def test_qrcp_points_beat_random_points():
    wl, s = sys_(n_occ=4, n_emp=16, grid=(12, 12, 12), box=7.0, seed=9)
    k_ex, _ = casida.hartree_matrix(s.phi, wl.n_occ, wl.grid, wl.h)
    err = lambda p: np.linalg.norm(I.k_isdf(s.phi, wl.n_occ, wl.grid, wl.h, p) - k_ex)
    for n_mu in (24, 40):
        pts = I.qrcp_points(s.phi, wl.n_occ, n_mu, _gauss((wl.n_occ, n_mu + 8), 1),
                            _gauss((wl.n_emp, n_mu + 8), 2))
        assert err(pts) < 0.9 * err(gi.random_grid_points(n_mu, wl.n_r, seed=3))
