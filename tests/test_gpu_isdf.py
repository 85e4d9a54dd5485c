"""GPU ISDF product (gwl_isdf_setup, GWL_KEY_ISDF) against the oracle.

* C x with the ISDF factorisation: FP64 <= 1e-10 relative to the oracle's
  dense C_ISDF on a smooth case and on the ragged case;
* Sigma through the whole path: FP64 <= 1e-8 relative (smooth orbitals,
  N_mu = 4 N_orb seeded random points); the mixed precision is refused;
* turning ISDF off restores the grid product; bad points and enabling
  without a setup are errors;
* K-means interpolation points equal the oracle's bit for bit (isotropic and
  anisotropic boxes, repeated initial centroids, a single pass) and fit C
  better than the random points they start from.
"""
import numpy as np
import pytest

import gw_inputs as gi
import oracle
from oracle import isdf as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(*a):
    print("[case]", *a, flush=True)


def relerr(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / max(np.max(np.abs(b)), 1e-300))


class Case:
    def __init__(self, base, n_mu_per_orb=4, **kw):
        self.wl = gi.workload(base, **kw)
        self.sys = gi.make_system(self.wl)
        self.points = gi.random_grid_points(n_mu_per_orb * self.wl.n_orb, self.wl.n_r, seed=21)
        self.pr = I.IsdfProblem(self.sys.phi, self.sys.energies_ev, self.wl.n_occ,
                                self.wl.grid, self.wl.h, self.points)
        self.lo, self.hi = oracle.default_interval(self.pr)


def make_ctx(case, precision="fp64", **kw):
    import paper_2310_20103_amd as G
    wl = case.wl
    ctx = G.Context(case.sys.phi, case.sys.energies_ev, wl.n_occ, wl.grid,
                    tuple(n * wl.h for n in wl.grid), precision=precision,
                    poly_degree=wl.poly_degree, poly_lo=case.lo, poly_hi=case.hi, **kw)
    ctx.isdf_setup(case.points)
    return ctx


@pytest.fixture(scope="module")
def smooth():
    _say("isdf smooth case 24^3, 8+32, 160 points")
    return Case("grid24_v8c32", name="smooth", smooth_sigma=1.0, n_lanczos=24, n_omega=41)


@pytest.fixture(scope="module")
def ragged():
    _say("isdf ragged case 12x18x8, 5+19, 96 points")
    return Case("grid24_v8c32", name="ragged", seed=77, grid=(12, 18, 8), box=7.0, n_occ=5,
                n_emp=19, smooth_sigma=1.0, n_lanczos=12, n_omega=21)


@pytest.mark.parametrize("which", ["smooth", "ragged"])
def test_apply_c_fp64(request, which):
    import paper_2310_20103_amd as G
    case = request.getfixturevalue(which)
    _say("isdf apply_c fp64", which)
    x = gi.random_pair_vectors(3, case.wl.n_vc, seed=5)
    with make_ctx(case) as ctx:
        assert ctx.query(G.KEY_ISDF) == 1 and ctx.query(G.KEY_ISDF_NMU) == len(case.points)
        got = ctx.apply_c(torch.tensor(x, device="cuda")).cpu().numpy()
    assert relerr(got, x @ case.pr.C.T) <= 1e-10


def test_sigma_fp64_mixed_refused(smooth):
    import paper_2310_20103_amd as G
    _say("isdf sigma fp64; mixed refused")
    wl = smooth.wl
    with make_ctx(smooth) as ctx:
        got64 = ctx.sigma_c(smooth.sys.qp_states, smooth.sys.omega_ev, wl.eta, wl.n_lanczos)
        ctx.set_precision("mixed")
        with pytest.raises(G.GwlError):
            ctx.sigma_c(smooth.sys.qp_states[:1], smooth.sys.omega_ev, wl.eta, 4)
    for i, m in enumerate(smooth.sys.qp_states):
        ref = smooth.pr.sigma_lanczos(int(m), smooth.sys.omega_ev, wl.eta, wl.n_lanczos,
                                      smooth.lo, smooth.hi, wl.poly_degree)
        assert np.max(np.abs(ref)) > 0.1
        assert relerr(got64[i], ref) <= 1e-8


def test_isdf_with_quadrature_and_offdiag(smooth):
    """The ISDF product under the other Sigma routes: Lanczos on C with Gauss
    quadrature, and the off-diagonal element, against the oracle on the same
    ISDF operator (FP64 <= 1e-8 relative)."""
    from oracle import offdiag as O
    from oracle import quadrature as Q
    _say("isdf + quadrature, isdf + off-diagonal")
    wl = smooth.wl
    m, m2 = int(smooth.sys.qp_states[0]), int(smooth.sys.qp_states[-1])
    om = smooth.sys.omega_ev
    with make_ctx(smooth) as ctx:
        off = ctx.sigma_c_offdiag(m, m2, om, wl.eta, 10)
        ctx.set_quadrature(True)
        quad = ctx.sigma_c([m], om, wl.eta, 20)[0]
    ref_off = O.sigma_lanczos_offdiag(smooth.pr, m, m2, om, wl.eta, 10, smooth.lo, smooth.hi,
                                      wl.poly_degree)
    ref_quad = Q.sigma_quadrature(smooth.pr, m, om, wl.eta, 20)
    assert np.max(np.abs(ref_off)) > 1e-3 and np.max(np.abs(ref_quad)) > 0.1
    assert relerr(off, ref_off) <= 1e-8
    assert relerr(quad, ref_quad) <= 1e-8


def test_switch_off_and_errors(smooth):
    import paper_2310_20103_amd as G
    _say("isdf off / errors")
    wl = smooth.wl
    grid = oracle.Problem(smooth.sys.phi, smooth.sys.energies_ev, wl.n_occ, wl.grid, wl.h)
    x = gi.random_pair_vectors(2, wl.n_vc, seed=6)
    with make_ctx(smooth) as ctx:
        ctx.set_isdf(False)
        got = ctx.apply_c(torch.tensor(x, device="cuda")).cpu().numpy()
        assert relerr(got, x @ grid.C.T) <= 1e-11
        with pytest.raises(G.GwlError):
            ctx.isdf_setup([5, 3, 9])                        # not increasing
        with pytest.raises(G.GwlError):
            ctx.isdf_setup([0, wl.n_r])                      # out of range
    ctx2 = G.Context(smooth.sys.phi, smooth.sys.energies_ev, wl.n_occ, wl.grid,
                     tuple(n * wl.h for n in wl.grid), poly_lo=smooth.lo, poly_hi=smooth.hi)
    try:
        with pytest.raises(G.GwlError):
            ctx2.set_isdf(True)
    finally:
        ctx2.close()


@pytest.mark.parametrize("which", ["smooth", "ragged"])
def test_kmeans_points_match_oracle(request, which):
    """gwl_isdf_kmeans gives the oracle's points and assignment count bit for
    bit (integer results of exactly reproduced FP64 decisions); the ragged
    grid runs in an anisotropic box (spacing differs per axis)."""
    import paper_2310_20103_amd as G
    case = request.getfixturevalue(which)
    wl = case.wl
    _say("isdf kmeans vs oracle", which)
    box = tuple(n * wl.h for n in wl.grid) if which == "smooth" else (7.0, 9.1, 5.3)
    spacing = tuple(b / n for b, n in zip(box, wl.grid))
    init = gi.random_grid_points(len(case.points), wl.n_r, seed=31)
    ref, ref_n = I.kmeans_points(I.kmeans_weights(case.sys.phi, wl.n_occ), wl.grid, spacing,
                                 init, 25)
    with G.Context(case.sys.phi, case.sys.energies_ev, wl.n_occ, wl.grid, box,
                   poly_lo=case.lo, poly_hi=case.hi) as ctx:
        got, got_n = ctx.isdf_kmeans(init, 25)
    assert got_n == ref_n
    assert np.array_equal(got, ref)


def test_kmeans_many_centroids():
    """More centroids than one LDS chunk of the assignment kernel (1024):
    1100 centroids on a 16^3 grid, bit for bit against the oracle."""
    import paper_2310_20103_amd as G
    _say("isdf kmeans, 1100 centroids on 16^3")
    wl = gi.workload("grid24_v8c32", name="km1100", seed=41, grid=(16, 16, 16), box=8.0,
                     n_occ=4, n_emp=12, smooth_sigma=1.0)
    s = gi.make_system(wl)
    box = tuple(n * wl.h for n in wl.grid)
    spacing = tuple(b / n for b, n in zip(box, wl.grid))
    init = gi.random_grid_points(1100, wl.n_r, seed=42)
    ref, ref_n = I.kmeans_points(I.kmeans_weights(s.phi, wl.n_occ), wl.grid, spacing, init, 10)
    with G.Context(s.phi, s.energies_ev, wl.n_occ, wl.grid, box) as ctx:
        got, got_n = ctx.isdf_kmeans(init, 10)
    assert got_n == ref_n
    assert np.array_equal(got, ref)


def test_kmeans_edges(smooth):
    """Repeated initial centroids leave clusters empty (fewer points), a
    single assignment pass at max_iter = 0, and bad arguments are errors."""
    import paper_2310_20103_amd as G
    wl = smooth.wl
    _say("isdf kmeans edges")
    spacing = tuple((n * wl.h) / n for n in wl.grid)
    w = I.kmeans_weights(smooth.sys.phi, wl.n_occ)
    init = [17, 17, 4000, 9000, 9000, 12000]
    with make_ctx(smooth) as ctx:
        for it in (0, 3):
            got, got_n = ctx.isdf_kmeans(init, it)
            ref, ref_n = I.kmeans_points(w, wl.grid, spacing, init, it)
            assert got_n == ref_n and np.array_equal(got, ref)
        assert ctx.isdf_kmeans(init, 0)[1] == 1 and len(ctx.isdf_kmeans(init, 0)[0]) == 4
        with pytest.raises(G.GwlError):
            ctx.isdf_kmeans([0, wl.n_r], 5)
        with pytest.raises(G.GwlError):
            ctx.isdf_kmeans([1, 2], -1)


def test_kmeans_points_fit_better(smooth):
    """C x with ISDF on the K-means points is closer to the grid product than
    with the random points they started from (same count)."""
    wl = smooth.wl
    _say("isdf kmeans fit vs random")
    grid = oracle.Problem(smooth.sys.phi, smooth.sys.energies_ev, wl.n_occ, wl.grid, wl.h)
    x = gi.random_pair_vectors(3, wl.n_vc, seed=8)
    ref = x @ grid.C.T
    with make_ctx(smooth) as ctx:
        pts, _ = ctx.isdf_kmeans(smooth.points, 30)
        err_rand = relerr(ctx.apply_c(torch.tensor(x, device="cuda")).cpu().numpy(), ref)
        ctx.isdf_setup(pts)
        err_km = relerr(ctx.apply_c(torch.tensor(x, device="cuda")).cpu().numpy(), ref)
    assert err_km < 0.9 * err_rand


# ------------------------------------------------------------------ QRCP points
@pytest.mark.parametrize("shape", [((12, 12, 12), 7.0, 4, 16, (24, 40)),
                                   ((16, 12, 8), 6.0, 3, 11, (20, 33))])
def test_qrcp_points_match_oracle(shape):
    """gwl_isdf_qrcp against the oracle's pivoted Gram-Schmidt on the same
    sketch (random factors passed to both): the same point set; with the
    points the ISDF C x fits better than with random ones."""
    import paper_2310_20103_amd as G
    grid, box, n_occ, n_emp, n_mus = shape
    wl = gi.workload("grid24_v8c32", name="qrcp", seed=9, grid=grid, box=box, n_occ=n_occ,
                     n_emp=n_emp, smooth_sigma=1.0)
    s = gi.make_system(wl)
    k_ex, _ = oracle.casida.hartree_matrix(s.phi, wl.n_occ, wl.grid, wl.h)
    with G.Context(s.phi, s.energies_ev, wl.n_occ, wl.grid,
                   tuple(n * wl.h for n in wl.grid)) as c:
        for n_mu in n_mus:
            rng = np.random.default_rng(n_mu)
            gv = rng.standard_normal((n_occ, n_mu + 8))
            gc = rng.standard_normal((n_emp, n_mu + 8))
            _say(f"qrcp grid {grid}, {n_occ}+{n_emp}, n_mu {n_mu}")
            got = c.isdf_qrcp(gv, gc, n_mu)
            ref = I.qrcp_points(s.phi, wl.n_occ, n_mu, gv, gc)
            assert np.array_equal(got, ref)
            err = lambda p: np.linalg.norm(I.k_isdf(s.phi, wl.n_occ, wl.grid, wl.h, p) - k_ex)
            assert err(got) < 0.9 * err(gi.random_grid_points(n_mu, wl.n_r, seed=3))
        # the points feed the ISDF product directly
        c.isdf_setup(got)
        c.set_option(G.KEY_ISDF, 1)
        assert c.query(G.KEY_ISDF_NMU) == n_mus[-1]
        with pytest.raises(G.GwlError):
            c.isdf_qrcp(gv, gc, gv.shape[1] + 1)   # more points than sketch columns
