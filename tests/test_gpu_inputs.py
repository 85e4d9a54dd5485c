"""GPU parity on the input forms of the large configuration and on a smooth,
headline-shaped case, each against the FP64 CPU oracle element by element.

* FP32 orbitals (orb_dtype 4), handed over from host memory and from device
  memory: C x and the coupling vectors P_nm (FP64 <= 1e-11 relative) and
  Sigma (FP64 <= 1e-8 relative; mixed <= 1e-3 eV on smooth orbitals), the
  oracle running on the same FP32-rounded orbital values in FP64.
* Grids with a 128-point edge along x, y or z (the FFT line length of the
  128^3 configuration): the Poisson solve (FP64 1e-12, FP32 2e-6 relative)
  and C x (FP64 1e-11; mixed 1e-3, its coupling part 2e-2).
* grid32_v32c128 with smooth orbitals (low-pass width 1 bohr before the QR):
  the headline case's shape scaled to a size the oracle diagonalises
  (N_vc = 4096), where Sigma is eV-sized and the 1 meV bar on the mixed path
  binds; FP64 <= 1e-8 relative and mixed <= 1e-3 eV against the oracle's
  Lanczos Sigma (its spectral-measure route) for all four QP states.
* A NaN or an infinity among the orbital values (FP64 or FP32, host or
  device) is refused at setup, where the orbitals are packed on the GPU.
"""
import numpy as np
import pytest

import gw_inputs as gi
import oracle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(*a):
    print("[case]", *a, flush=True)


def relerr(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / max(np.max(np.abs(b)), 1e-300))


def _box(wl):
    return tuple(n * wl.h for n in wl.grid)


def _ctx(orbitals, eps, wl, lo, hi, precision="fp64", **kw):
    import paper_2310_20103_amd as G
    return G.Context(orbitals, eps, wl.n_occ, wl.grid, _box(wl), precision=precision,
                     poly_degree=wl.poly_degree, poly_lo=lo, poly_hi=hi, **kw)


# ------------------------------------------------------------------ FP32 orbitals
@pytest.fixture(scope="module")
def f32case():
    _say("fp32 orbitals: smooth 24^3, 8+32")
    wl = gi.workload("grid24_v8c32", name="f32", smooth_sigma=1.0, n_lanczos=48, n_omega=101)
    s = gi.make_system(wl)
    phi32 = s.phi.astype(np.float32)
    pr = oracle.Problem(phi32.astype(np.float64), s.energies_ev, wl.n_occ, wl.grid, wl.h)
    lo, hi = oracle.default_interval(pr)
    return wl, s, phi32, pr, lo, hi


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("where", ["host", "device"])
def test_non_finite_orbitals_refused(f32case, dtype, where):
    import paper_2310_20103_amd as G
    wl, s, phi32, pr, lo, hi = f32case
    _say("non-finite orbital values refused,", np.dtype(dtype).name, where)
    for bad in (np.nan, np.inf):
        phi = s.phi.astype(dtype)
        phi[wl.n_occ + 3, 1234] = bad  # a conduction orbital, away from the row ends
        src = phi if where == "host" else torch.from_numpy(phi).cuda()
        with pytest.raises(G.GwlError, match="non-finite orbital value"):
            _ctx(src, s.energies_ev, wl, lo, hi)


@pytest.mark.parametrize("where", ["host", "device"])
def test_fp32_orbitals_products(f32case, where):
    wl, s, phi32, pr, lo, hi = f32case
    _say("fp32 orbitals C x and coupling vectors from", where)
    orb = phi32 if where == "host" else torch.tensor(phi32, device="cuda")
    with _ctx(orb, s.energies_ev, wl, lo, hi) as c:
        x = gi.random_pair_vectors(5, wl.n_vc, seed=41)
        got = c.apply_c(torch.tensor(x, device="cuda")).cpu().numpy()
        assert relerr(got, x @ pr.C.T) <= 1e-11
        m = int(s.qp_states[0])
        n = np.arange(wl.n_orb)
        p = c.coupling(np.full_like(n, m), n).cpu().numpy()
        assert relerr(p, pr.coupling(m)) <= 1e-11


@pytest.mark.parametrize("where", ["host", "device"])
def test_fp32_orbitals_sigma(f32case, where):
    wl, s, phi32, pr, lo, hi = f32case
    orb = phi32 if where == "host" else torch.tensor(phi32, device="cuda")
    om = s.omega_ev
    for prec in ("fp64", "mixed"):
        _say("fp32 orbitals sigma", where, prec)
        with _ctx(orb, s.energies_ev, wl, lo, hi, precision=prec) as c:
            got = c.sigma_c(s.qp_states, om, wl.eta, wl.n_lanczos)
        for i, m in enumerate(s.qp_states):
            ref = pr.sigma_lanczos(int(m), om, wl.eta, wl.n_lanczos, lo, hi, wl.poly_degree,
                                   route="measure")
            err = float(np.max(np.abs(got[i] - ref)))
            _say(f"  m={m}: max|Sigma| {np.max(np.abs(ref)):.3e} eV, err {err:.2e} eV, "
                 f"rel {relerr(got[i], ref):.2e}")
            if prec == "fp64":
                assert relerr(got[i], ref) <= 1e-8
            else:
                assert err <= 1e-3


# ------------------------------------------------------------------ 128-point edges
@pytest.mark.parametrize("grid", [(128, 12, 8), (12, 128, 8), (8, 12, 128)])
def test_grid_with_128_point_edge(grid):
    wl = gi.workload("grid24_v8c32", name="edge128", seed=61, grid=grid, box=0.375 * grid[0],
                     n_occ=4, n_emp=12, n_qp_occ=1, n_qp_emp=1, n_lanczos=8, n_omega=9)
    _say("grid", grid, "h 0.375 bohr, 4+12 orbitals")
    s = gi.make_system(wl)
    pr = oracle.Problem(s.phi, s.energies_ev, wl.n_occ, wl.grid, wl.h)
    lo, hi = oracle.default_interval(pr)
    f = gi.random_fields(6, wl.n_r, seed=62)
    ref_v = oracle.poisson.poisson(f, wl.grid, wl.h)
    x = gi.random_pair_vectors(4, wl.n_vc, seed=63)
    ref_c = x @ pr.C.T
    dk = ref_c - pr.delta ** 2 * x
    for prec, tol_v in (("fp64", 1e-12), ("mixed", 2e-6)):
        with _ctx(s.phi, s.energies_ev, wl, lo, hi, precision=prec) as c:
            dt = torch.float64 if prec == "fp64" else torch.float32
            v = c.poisson(torch.tensor(f, dtype=dt, device="cuda"), prec).double().cpu().numpy()
            got = c.apply_c(torch.tensor(x, device="cuda"), prec).cpu().numpy()
        _say(f"  {prec}: poisson {relerr(v, ref_v):.2e}, C x {relerr(got, ref_c):.2e}")
        assert relerr(v, ref_v) <= tol_v
        if prec == "fp64":
            assert relerr(got, ref_c) <= 1e-11
        else:
            assert relerr(got, ref_c) <= 1e-3
            assert relerr(got - pr.delta ** 2 * x, dk) <= 2e-2


# ------------------------------------------------------------------ 2^20 grid points
def test_grid_of_2_20_points_k_panels():
    """128 x 128 x 64 = 2^20 points: the mixed second GEMM reads its FP16
    orbitals from K panels (rows of N_rp values below 2^20 points), in the
    MFMA kernel and in the plain-FMA kernel; C x against the oracle."""
    import paper_2310_20103_amd as G
    grid = (128, 128, 64)
    wl = gi.workload("grid24_v8c32", name="grid2p20", seed=71, grid=grid, box=0.375 * grid[0],
                     n_occ=4, n_emp=12, n_qp_occ=1, n_qp_emp=1, n_lanczos=8, n_omega=9)
    _say("grid", grid, "(2^20 points), 4+12 orbitals, mixed products from K panels")
    s = gi.make_system(wl)
    pr = oracle.Problem(s.phi, s.energies_ev, wl.n_occ, wl.grid, wl.h)
    lo, hi = oracle.default_interval(pr)
    x = gi.random_pair_vectors(4, wl.n_vc, seed=72)
    ref_c = x @ pr.C.T
    dk = ref_c - pr.delta ** 2 * x
    with _ctx(s.phi, s.energies_ev, wl, lo, hi, precision="mixed") as c:
        for kern in (1, 0):
            c.set_option(G.KEY_KERNELS, kern)
            got = c.apply_c(torch.tensor(x, device="cuda"), "mixed").cpu().numpy()
            _say(f"  kernels {kern}: C x {relerr(got, ref_c):.2e}, "
                 f"K x {relerr(got - pr.delta ** 2 * x, dk):.2e}")
            assert relerr(got, ref_c) <= 1e-3
            assert relerr(got - pr.delta ** 2 * x, dk) <= 2e-2


# ------------------------------------------------------------------ smooth headline-shaped case
def test_smooth_headline_shaped_sigma():
    wl = gi.workload("grid32_v32c128", name="grid32_v32c128_smooth", smooth_sigma=1.0)
    _say("smooth grid32_v32c128: 32^3, 32+128 orbitals, N_vc 4096, L", wl.n_lanczos)
    s = gi.make_system(wl)
    pr = oracle.Problem(s.phi, s.energies_ev, wl.n_occ, wl.grid, wl.h)
    lo, hi = oracle.default_interval(pr)
    om = s.omega_ev
    refs = [pr.sigma_lanczos(int(m), om, wl.eta, wl.n_lanczos, lo, hi, wl.poly_degree,
                             route="measure") for m in s.qp_states]
    for prec in ("fp64", "mixed"):
        with _ctx(s.phi, s.energies_ev, wl, lo, hi, precision=prec) as c:
            got = c.sigma_c(s.qp_states, om, wl.eta, wl.n_lanczos)
        for i, m in enumerate(s.qp_states):
            err = float(np.max(np.abs(got[i] - refs[i])))
            _say(f"  {prec} m={m}: max|Sigma| {np.max(np.abs(refs[i])):.3f} eV, "
                 f"err {err:.2e} eV, rel {relerr(got[i], refs[i]):.2e}")
            assert np.max(np.abs(refs[i])) > 0.05
            if prec == "fp64":
                assert relerr(got[i], refs[i]) <= 1e-8
            else:
                assert err <= 1e-3
