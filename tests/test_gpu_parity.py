"""GPU parity of every step of the path against the FP64 CPU oracle.

Each test calls the HIP library through the C ABI (ctypes binding) and
compares element by element with the oracle on the same seeded inputs.
Tolerances:
  * FP64 kernels (FFT Poisson, coupling vectors, C x, p_g(C) x): 1e-11
    relative to the largest element; FP64 Sigma vs the oracle's Lanczos
    Sigma_L: <= 1e-8 relative (max over omega, per QP state).
  * mixed (BF16 GEMM operands, FP32 accumulation/FFT, FP64 recurrence):
    <= 1e-3 eV absolute against the oracle.
"""
import numpy as np
import pytest

import gw_inputs as gi
import oracle
from oracle import chebyshev as CH
from oracle import sigma as S

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print("[case]", *a, flush=True)


def box_of(wl):
    return tuple(n * wl.h for n in wl.grid)


def make_ctx(sysm, precision="fp64", interval=None, poly_degree_override=None, **kw):
    import paper_2310_20103_amd as G
    wl = sysm.wl
    lo, hi = interval if interval is not None else (0.0, 0.0)
    g = wl.poly_degree if poly_degree_override is None else poly_degree_override
    return G.Context(sysm.phi, sysm.energies_ev, wl.n_occ, wl.grid, box_of(wl),
                     precision=precision, poly_degree=g, poly_lo=lo, poly_hi=hi, **kw)


def relerr(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / max(np.max(np.abs(b)), 1e-300))


class Case:
    def __init__(self, base, **over):
        wl = gi.workload(base, **over)
        self.sys = gi.make_system(wl)
        self.wl = wl
        self.pr = oracle.Problem(self.sys.phi, self.sys.energies_ev, wl.n_occ, wl.grid, wl.h)
        self.lo, self.hi = oracle.default_interval(self.pr)


@pytest.fixture(scope="module")
def small():
    _say("small case grid24_v8c32")
    return Case("grid24_v8c32")


@pytest.fixture(scope="module")
def ragged():
    # grid 12 x 18 x 8 (radices 4*3, 2*3*3, 8), N_v = 5, N_c = 19: every
    # dimension has a ragged tail against the tiles
    _say("ragged case grid 12x18x8, 5+19 orbitals")
    return Case("grid24_v8c32", name="ragged", seed=77, grid=(12, 18, 8), box=6.0,
                n_occ=5, n_emp=19, n_qp_occ=1, n_qp_emp=1, n_lanczos=24, n_omega=33)


@pytest.fixture(scope="module")
def smooth():
    _say("smooth stress variant of the small case")
    return Case("grid24_v8c32", name="smooth", smooth_sigma=1.0)


@pytest.fixture(scope="module")
def ctx_small(small):
    c = make_ctx(small.sys, interval=(small.lo, small.hi))
    yield c
    c.close()


@pytest.fixture(scope="module")
def ctx_ragged(ragged):
    c = make_ctx(ragged.sys, interval=(ragged.lo, ragged.hi))
    yield c
    c.close()


# ------------------------------------------------------------------ FFT Poisson
@pytest.mark.parametrize("which", ["small", "ragged"])
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("mixed", 2e-6)])
def test_poisson(request, which, precision, tol):
    case = request.getfixturevalue(which)
    ctx = request.getfixturevalue("ctx_" + which)
    wl = case.wl
    _say("poisson", which, precision)
    f = gi.random_fields(5, wl.n_r, seed=3)
    ref = oracle.poisson.poisson(f, wl.grid, wl.h)
    dt = torch.float64 if precision == "fp64" else torch.float32
    got = ctx.poisson(torch.tensor(f, dtype=dt, device="cuda"), precision).double().cpu().numpy()
    assert relerr(got, ref) <= tol


# ------------------------------------------------------------------ coupling vectors
@pytest.mark.parametrize("which", ["small", "ragged"])
def test_coupling(request, which):
    case = request.getfixturevalue(which)
    ctx = request.getfixturevalue("ctx_" + which)
    _say("coupling", which)
    m = int(case.sys.qp_states[0])
    ref = case.pr.coupling(m)
    n = np.arange(case.wl.n_orb)
    got = ctx.coupling(np.full_like(n, m), n).cpu().numpy()
    assert relerr(got, ref) <= 1e-11


# ------------------------------------------------------------------ C x and p_g(C) x
@pytest.mark.parametrize("which", ["small", "ragged"])
def test_apply_c_fp64(request, which):
    case = request.getfixturevalue(which)
    ctx = request.getfixturevalue("ctx_" + which)
    _say("apply_c fp64", which)
    x = gi.random_pair_vectors(7, case.wl.n_vc, seed=4)
    ref = x @ case.pr.C.T
    got = ctx.apply_c(torch.tensor(x, device="cuda")).cpu().numpy()
    assert relerr(got, ref) <= 1e-11


@pytest.mark.parametrize("which", ["small", "ragged"])
def test_apply_c_mixed(request, which):
    case = request.getfixturevalue(which)
    ctx = request.getfixturevalue("ctx_" + which)
    _say("apply_c mixed", which)
    x = gi.random_pair_vectors(3, case.wl.n_vc, seed=5)
    ref = x @ case.pr.C.T
    got = ctx.apply_c(torch.tensor(x, device="cuda"), "mixed").cpu().numpy()
    assert relerr(got, ref) <= 1e-3
    # the coupling part alone to BF16 accuracy
    dk = ref - case.pr.delta ** 2 * x
    gk = got - case.pr.delta ** 2 * x
    assert relerr(gk, dk) <= 2e-2


@pytest.mark.parametrize("which", ["small", "ragged"])
def test_pair_density(request, which):
    """The first GEMM with its fused row-dot alone (gwl_pair_density):
    rho_b = (Delta^1/2 x_b) B with B[(v,c), r] = phi_v(r) phi_c(r), the oracle's
    pair densities.  Mixed: three FP16 factors per term (unit roundoff 2^-11
    each), FP32 sums."""
    from oracle import casida as CA
    case = request.getfixturevalue(which)
    ctx = request.getfixturevalue("ctx_" + which)
    _say("pair density", which)
    x = gi.random_pair_vectors(5, case.wl.n_vc, seed=8)
    ref = (np.sqrt(case.pr.delta) * x) @ CA.pair_densities(case.sys.phi, case.wl.n_occ)
    for prec, tol in (("fp64", 1e-12), ("mixed", 2e-3)):
        got = ctx.pair_density(torch.tensor(x, device="cuda"), prec).cpu().numpy()
        _say(f"  {prec}: {relerr(got, ref):.2e}")
        assert got.shape == ref.shape
        assert relerr(got, ref) <= tol


@pytest.mark.parametrize("which", ["small", "ragged"])
def test_potential_product(request, which):
    """The second GEMM alone (gwl_potential_product) on seeded potentials:
    y_b,vc = dV sum_r phi_v(r) V_b(r) phi_c(r); and, with V_b the oracle's
    Hartree potential of the pair density of x_b, y_b = K x_b.  Mixed: FP16
    phi_v, phi_c and V_b, their product phi_v V_b rounded to FP16 again, FP32
    sums."""
    from oracle import casida as CA
    from oracle import poisson as PO
    case = request.getfixturevalue(which)
    ctx = request.getfixturevalue("ctx_" + which)
    _say("potential product", which)
    phi, nv = case.sys.phi, case.wl.n_occ
    dv = case.wl.h ** 3
    pv, pc = phi[:nv], phi[nv:]
    v = np.random.default_rng(21).standard_normal((3, phi.shape[1]))
    x = gi.random_pair_vectors(2, case.wl.n_vc, seed=22)
    rho = x @ CA.pair_densities(phi, nv)
    v = np.concatenate([v, PO.poisson(rho, case.wl.grid, case.wl.h)])
    ref = dv * np.einsum("vr,br,cr->bvc", pv, v, pc).reshape(len(v), -1)
    kx = CA.apply_k(phi, nv, case.wl.grid, case.wl.h, x)
    for prec, tol in (("fp64", 1e-12), ("mixed", 3e-3)):
        got = ctx.potential_product(torch.tensor(v, device="cuda"), prec).cpu().numpy()
        _say(f"  {prec}: {relerr(got, ref):.2e}  K x: {relerr(got[3:], kx):.2e}")
        assert got.shape == ref.shape
        assert relerr(got, ref) <= tol
        assert relerr(got[3:], kx) <= tol


def test_component_calls_chunked_and_errors(request):
    """gwl_pair_density and gwl_potential_product over 130 vectors (a batch
    of 128, then 2): the same values as one call per vector (to rounding:
    the split of the grid sum depends on the batch size); no vectors is a
    no-op; the ISDF product refuses both."""
    import paper_2310_20103_amd as G
    from oracle import casida as CA
    case = request.getfixturevalue("ragged")
    ctx = request.getfixturevalue("ctx_ragged")
    _say("component calls over 130 vectors")
    x = gi.random_pair_vectors(130, case.wl.n_vc, seed=23)
    ref = (np.sqrt(case.pr.delta) * x) @ CA.pair_densities(case.sys.phi, case.wl.n_occ)
    rho = ctx.pair_density(torch.tensor(x, device="cuda"), "fp64").cpu().numpy()
    assert relerr(rho, ref) <= 1e-12
    y = ctx.potential_product(torch.tensor(rho, device="cuda"), "fp64").cpu().numpy()
    one = np.concatenate([ctx.potential_product(torch.tensor(rho[i:i + 1], device="cuda"),
                                                "fp64").cpu().numpy() for i in (0, 127, 128, 129)])
    assert relerr(y[[0, 127, 128, 129]], one) <= 1e-12
    empty = ctx.potential_product(torch.zeros((0, case.wl.n_r), dtype=torch.float64,
                                              device="cuda"), "fp64")
    assert tuple(empty.shape) == (0, case.wl.n_vc)
    with make_ctx(case.sys, interval=(case.lo, case.hi)) as c2:
        # 32 spread points (fewer than N_vc = 95, so C C^T is regular)
        c2.isdf_setup(np.linspace(0, case.wl.n_r - 1, 32).astype(np.int32))
        with pytest.raises(G.GwlError, match="ISDF"):
            c2.potential_product(torch.tensor(rho[:2], device="cuda"), "fp64")
        with pytest.raises(G.GwlError, match="ISDF"):
            c2.pair_density(torch.tensor(x[:2], device="cuda"), "fp64")


@pytest.mark.parametrize("n_emp", [100, 150, 260])
def test_apply_c_conduction_k_steps(n_emp):
    """C x with N_c padded to 128, 192 and 320: the K loops of the GEMMs over
    the conduction index run 4, 6 and 10 steps of 32 (the mixed first GEMM
    has a peeled head and tail of two steps each around its main loop)."""
    case = Case("grid24_v8c32", name=f"ksteps{n_emp}", seed=90 + n_emp, grid=(16, 16, 16),
                box=8.0, n_occ=4, n_emp=n_emp, n_qp_occ=1, n_qp_emp=1, n_lanczos=4,
                n_omega=5)
    _say("apply_c conduction K steps", n_emp)
    x = gi.random_pair_vectors(3, case.wl.n_vc, seed=6)
    ref = x @ case.pr.C.T
    dk = ref - case.pr.delta ** 2 * x
    for prec in ("fp64", "mixed"):
        with make_ctx(case.sys, precision=prec, interval=(case.lo, case.hi)) as ctx:
            got = ctx.apply_c(torch.tensor(x, device="cuda"), prec).cpu().numpy()
        if prec == "fp64":
            assert relerr(got, ref) <= 1e-11
        else:
            assert relerr(got, ref) <= 1e-3
            assert relerr(got - case.pr.delta ** 2 * x, dk) <= 2e-2


@pytest.mark.parametrize("which", ["small", "ragged"])
def test_apply_d_fp64(request, which):
    case = request.getfixturevalue(which)
    ctx = request.getfixturevalue("ctx_" + which)
    _say("apply_d fp64", which)
    x = gi.random_pair_vectors(3, case.wl.n_vc, seed=6)
    dg = case.pr.dg_matrix(case.lo, case.hi, case.wl.poly_degree)
    ref = x @ dg.T
    got = ctx.apply_d(torch.tensor(x, device="cuda")).cpu().numpy()
    assert relerr(got, ref) <= 1e-11


# ------------------------------------------------------------------ Lanczos coefficients
def test_lanczos_coefficients(small, ctx_small):
    _say("lanczos coefficients small, 4 pairs x 64 steps")
    m = int(small.sys.qp_states[0])
    ns = [0, 3, 9, 39]
    a, b, n2, ol = ctx_small.lanczos_pairs([m] * 4, ns, [64] * 4)
    ref = small.pr.lanczos_coeffs(m, 64, small.lo, small.hi, small.wl.poly_degree, n_list=ns)
    for i, (ra, rb, rn2) in enumerate(ref):
        assert ol[i] == len(ra)
        assert abs(n2[i] - rn2) <= 1e-12 * rn2
        assert relerr(a[i, :len(ra)], ra) <= 1e-9
        assert relerr(b[i, :len(rb)], rb) <= 1e-9


def test_uneven_lengths_with_refill(small):
    """Lengths 1..64 over 3 slots: slots retire and are refilled mid-run."""
    _say("uneven lengths, block 3")
    ctx = make_ctx(small.sys, interval=(small.lo, small.hi), block=3)
    try:
        m = int(small.sys.qp_states[1])
        ns = [1, 7, 20, 33, 2, 11, 38, 5]
        lens = [1, 5, 64, 17, 3, 40, 9, 26]
        a, b, n2, ol = ctx.lanczos_pairs([m] * len(ns), ns, lens)
        for i, n in enumerate(ns):
            ra, rb, rn2 = small.pr.lanczos_coeffs(m, lens[i], small.lo, small.hi,
                                                  small.wl.poly_degree, n_list=[n])[0]
            assert ol[i] == len(ra) == lens[i]
            assert relerr(a[i, :len(ra)], ra) <= 1e-9
            if len(rb):
                assert relerr(b[i, :len(rb)], rb) <= 1e-9
            assert np.all(a[i, len(ra):] == 0)
    finally:
        ctx.close()


def test_uneven_lengths_mixed_compacted(small):
    """Mixed precision with slots falling idle: the product then runs over
    the busy slots only (rows gathered in the cast, scattered in the combine);
    longest runs are scheduled first."""
    _say("uneven lengths mixed, block 3")
    ctx = make_ctx(small.sys, precision="mixed", interval=(small.lo, small.hi), block=3)
    try:
        m = int(small.sys.qp_states[0])
        ns = [4, 9, 30, 17, 2]
        lens = [6, 40, 12, 25, 3]
        a, b, n2, ol = ctx.lanczos_pairs([m] * len(ns), ns, lens)
        for i, n in enumerate(ns):
            ra, rb, rn2 = small.pr.lanczos_coeffs(m, lens[i], small.lo, small.hi,
                                                  small.wl.poly_degree, n_list=[n])[0]
            assert ol[i] == lens[i]
            # BF16 operands perturb the operator by ~1e-6; later Lanczos
            # coefficients amplify that, the first ones do not
            assert relerr(a[i, :min(8, lens[i])], ra[:8]) <= 1e-5
            assert relerr(a[i, :lens[i]], ra) <= 1e-3
            assert np.all(a[i, lens[i]:] == 0)
    finally:
        ctx.close()


def test_breakdown_short_fraction():
    """N_vc = 6 < L = 12: the recurrence must stop at an invariant subspace."""
    _say("breakdown tiny 2+3")
    case = Case("grid24_v8c32", name="tiny", seed=5, grid=(8, 8, 8), box=5.0, n_occ=2,
                n_emp=3, n_lanczos=12, n_omega=21)
    ctx = make_ctx(case.sys, interval=(case.lo, case.hi))
    try:
        m = int(case.sys.qp_states[0])
        ns = list(range(case.wl.n_orb))
        a, b, n2, ol = ctx.lanczos_pairs([m] * len(ns), ns, [12] * len(ns))
        assert np.all(ol <= 6) and np.all(ol >= 1)
        om = case.sys.omega_ev
        got = ctx.sigma_c([m], om, case.wl.eta, 12)[0]
        ref = case.pr.sigma_lanczos(m, om, case.wl.eta, 12, case.lo, case.hi, case.wl.poly_degree)
        assert relerr(got, ref) <= 1e-9
        # full length reproduces the L -> N_vc limit
        sdg = case.pr.sigma_dg(m, om, case.wl.eta, case.lo, case.hi, case.wl.poly_degree)
        assert relerr(got, sdg) <= 1e-9
    finally:
        ctx.close()


# ------------------------------------------------------------------ Sigma
def test_sigma_fp64_small(small, ctx_small):
    _say("sigma fp64 small L=64")
    wl = small.wl
    got = ctx_small.sigma_c(small.sys.qp_states, small.sys.omega_ev, wl.eta, wl.n_lanczos)
    for i, m in enumerate(small.sys.qp_states):
        ref = small.pr.sigma_lanczos(int(m), small.sys.omega_ev, wl.eta, wl.n_lanczos,
                                     small.lo, small.hi, wl.poly_degree)
        assert relerr(got[i], ref) <= 1e-8
        assert np.all(np.isfinite(got[i]))


def test_sigma_error_falls_with_degree_and_length(small):
    """Analogues of the paper's convergence checks in the polynomial degree g
    and the Lanczos length L (Fig. 1): the GPU's FP64 Sigma approaches the
    exact one as g grows (at L = N_vc, where the recurrence is exhausted) and
    approaches the L -> N_vc limit Sigma_Dg as L grows (g = 7); every point
    matches the oracle's Lanczos Sigma."""
    wl, pr, lo, hi = small.wl, small.pr, small.lo, small.hi
    m = int(small.sys.qp_states[0])
    om = small.sys.omega_ev
    sx = pr.sigma_exact(m, om, wl.eta)
    errs_g = []
    for g in (3, 7, 12):
        _say(f"sigma vs degree g={g}")
        with make_ctx(small.sys, interval=(lo, hi), poly_degree_override=g) as c:
            got = c.sigma_c([m], om, wl.eta, wl.n_vc)[0]
        assert relerr(got, pr.sigma_lanczos(m, om, wl.eta, wl.n_vc, lo, hi, g)) <= 1e-8
        errs_g.append(float(np.max(np.abs(got - sx))))
    assert errs_g[0] > errs_g[1] > errs_g[2], errs_g
    sdg = pr.sigma_dg(m, om, wl.eta, lo, hi, wl.poly_degree)
    errs_l = []
    with make_ctx(small.sys, interval=(lo, hi)) as c:
        for L in (4, 16, 64):
            _say(f"sigma vs length L={L}")
            got = c.sigma_c([m], om, wl.eta, L)[0]
            assert relerr(got, pr.sigma_lanczos(m, om, wl.eta, L, lo, hi, wl.poly_degree)) <= 1e-8
            errs_l.append(float(np.max(np.abs(got - sdg))))
    assert errs_l[0] > errs_l[1] > errs_l[2], errs_l


def test_sigma_fp64_ragged(ragged, ctx_ragged):
    _say("sigma fp64 ragged")
    wl = ragged.wl
    got = ctx_ragged.sigma_c(ragged.sys.qp_states, ragged.sys.omega_ev, wl.eta, wl.n_lanczos)
    for i, m in enumerate(ragged.sys.qp_states):
        ref = ragged.pr.sigma_lanczos(int(m), ragged.sys.omega_ev, wl.eta, wl.n_lanczos,
                                      ragged.lo, ragged.hi, wl.poly_degree)
        assert relerr(got[i], ref) <= 1e-8


def test_sigma_mixed_small(small, ctx_small):
    _say("sigma mixed small")
    wl = small.wl
    ctx_small.set_precision("mixed")
    try:
        got = ctx_small.sigma_c(small.sys.qp_states, small.sys.omega_ev, wl.eta, wl.n_lanczos)
    finally:
        ctx_small.set_precision("fp64")
    for i, m in enumerate(small.sys.qp_states):
        ref = small.pr.sigma_lanczos(int(m), small.sys.omega_ev, wl.eta, wl.n_lanczos,
                                     small.lo, small.hi, wl.poly_degree)
        assert np.max(np.abs(got[i] - ref)) <= 1e-3


def test_sigma_mixed_smooth_stress(smooth):
    """Smooth orbitals give eV-sized Sigma, so the 1 meV bar binds."""
    _say("sigma mixed smooth")
    wl = smooth.wl
    ctx = make_ctx(smooth.sys, precision="mixed", interval=(smooth.lo, smooth.hi))
    try:
        got = ctx.sigma_c(smooth.sys.qp_states, smooth.sys.omega_ev, wl.eta, wl.n_lanczos)
        ctx.set_precision("fp64")
        got64 = ctx.sigma_c(smooth.sys.qp_states, smooth.sys.omega_ev, wl.eta, wl.n_lanczos)
    finally:
        ctx.close()
    for i, m in enumerate(smooth.sys.qp_states):
        ref = smooth.pr.sigma_lanczos(int(m), smooth.sys.omega_ev, wl.eta, wl.n_lanczos,
                                      smooth.lo, smooth.hi, wl.poly_degree)
        assert np.max(np.abs(ref)) > 0.1          # the stress variant is eV-sized
        assert relerr(got64[i], ref) <= 1e-8
        assert np.max(np.abs(got[i] - ref)) <= 1e-3


def test_sigma_from_coeffs(small, ctx_small):
    _say("continued fraction from oracle coefficients")
    m = int(small.sys.qp_states[0])
    ns = list(range(small.wl.n_orb))
    coeffs = small.pr.lanczos_coeffs(m, 20, small.lo, small.hi, small.wl.poly_degree)
    ld = 20
    a = np.zeros((len(ns), ld))
    b = np.zeros((len(ns), ld))
    lens = np.zeros(len(ns), dtype=np.int32)
    n2 = np.zeros(len(ns))
    for i, (ra, rb, rn) in enumerate(coeffs):
        a[i, :len(ra)] = ra
        b[i, :len(rb)] = rb
        lens[i] = len(ra)
        n2[i] = rn
    om = small.sys.omega_ev
    got = ctx_small.sigma_from_coeffs(ns, a, b, n2, lens, om, small.wl.eta)
    for i, n in enumerate(ns):
        ref = S.sigma_n_from_tridiag(a[i, :lens[i]], b[i, :max(lens[i] - 1, 0)], n2[i],
                                     om / oracle.HARTREE_EV, small.pr.eps[n], small.pr.eta(n),
                                     small.wl.eta / oracle.HARTREE_EV) * oracle.HARTREE_EV
        assert relerr(got[i], ref) <= 1e-12


def test_resume_from_coefficient_file(small, ctx_small, tmp_path):
    """Lanczos coefficients from the GPU written to .npz, read back and turned
    into Sigma on a second frequency grid and broadening: the same values as
    from the arrays in memory, bit for bit, and as the oracle's continued
    fraction on the same coefficients."""
    import paper_2310_20103_amd as G
    _say("resume Sigma from a coefficient file")
    m = int(small.sys.qp_states[0])
    ns = list(range(0, small.wl.n_orb, 3))
    L = 12
    a, b, n2, ol = ctx_small.lanczos_pairs([m] * len(ns), ns, [L] * len(ns))
    path = tmp_path / "coeffs.npz"
    lo, hi = ctx_small.interval
    G.save_coefficients(path, [m] * len(ns), ns, a, b, n2, ol, poly_lo=lo, poly_hi=hi,
                        poly_degree=small.wl.poly_degree)
    got, meta = G.load_coefficients(path)
    assert meta["poly_hi"] == hi
    om2 = np.linspace(-30.0, 30.0, 77)
    eta2 = 0.25
    ref = ctx_small.sigma_from_coeffs(ns, a, b, n2, ol, om2, eta2)
    res = ctx_small.sigma_from_coeffs(got["n"], got["alpha"], got["beta"], got["norm2"],
                                      got["lens"], om2, eta2)
    assert np.array_equal(res, ref)
    for i, n in enumerate(ns):
        k = int(ol[i])
        orc = S.sigma_n_from_tridiag(a[i, :k], b[i, :max(k - 1, 0)], n2[i],
                                     om2 / oracle.HARTREE_EV, small.pr.eps[n], small.pr.eta(n),
                                     eta2 / oracle.HARTREE_EV) * oracle.HARTREE_EV
        assert relerr(res[i], orc) <= 1e-12


def test_reorth_modes_close(small):
    _say("reorth none/local vs full")
    wl = small.wl
    ref = small.pr.sigma_lanczos(int(small.sys.qp_states[0]), small.sys.omega_ev, wl.eta,
                                 wl.n_lanczos, small.lo, small.hi, wl.poly_degree)
    for mode in ("local", "none"):
        ctx = make_ctx(small.sys, interval=(small.lo, small.hi), reorth=mode)
        try:
            got = ctx.sigma_c(small.sys.qp_states[:1], small.sys.omega_ev, wl.eta, wl.n_lanczos)[0]
        finally:
            ctx.close()
        assert relerr(got, ref) <= 1e-3


def test_auto_interval_contains_spectrum(small):
    _say("auto interval")
    ctx = make_ctx(small.sys)
    try:
        lo, hi = ctx.interval
    finally:
        ctx.close()
    emin, emax = small.pr.spectral_bounds()
    assert lo <= emin * (1 + 1e-12)
    assert hi >= emax
    assert hi <= 1.1 * emax


def test_determinism(small, ctx_small):
    _say("determinism")
    wl = small.wl
    a = ctx_small.sigma_c(small.sys.qp_states, small.sys.omega_ev[:50], wl.eta, 16)
    b = ctx_small.sigma_c(small.sys.qp_states, small.sys.omega_ev[:50], wl.eta, 16)
    assert np.array_equal(a, b)


# ------------------------------------------------------------------ errors and edges
def test_errors_and_empty(small, ctx_small):
    import paper_2310_20103_amd as G
    _say("errors")
    s = small.sys
    wl = small.wl
    with pytest.raises(G.GwlError) as e:
        G.Context(s.phi, s.energies_ev, 0, wl.grid, wl.box)
    assert e.value.code == -1
    bad_e = s.energies_ev.copy()
    bad_e[wl.n_occ] = -20.0
    with pytest.raises(G.GwlError) as e:
        G.Context(s.phi, bad_e, wl.n_occ, wl.grid, wl.box)
    assert e.value.code == -1
    with pytest.raises(G.GwlError) as e:
        G.Context(np.zeros((4, 7 * 8 * 8)), np.array([-5.0, -4.0, 1.0, 2.0]), 2, (7, 8, 8), 5.0)
    assert e.value.code == -6
    with pytest.raises(G.GwlError):
        ctx_small.sigma_c([wl.n_orb], s.omega_ev, wl.eta, 4)
    with pytest.raises(G.GwlError):
        ctx_small.sigma_c([0], s.omega_ev, 0.0, 4)
    with pytest.raises(G.GwlError):
        ctx_small.sigma_c([0], s.omega_ev, wl.eta, 0)
    out = ctx_small.sigma_c([], s.omega_ev, wl.eta, 4)
    assert out.shape == (0, len(s.omega_ev))
    out = ctx_small.sigma_c([0], [], wl.eta, 4)
    assert out.shape == (1, 0)


# ------------------------------------------------------------------ wide valence space
@pytest.fixture(scope="module")
def wide():
    # N_v = 136 pads to 256: two 128-wide v tiles of the first GEMM (FP32
    # weights from L2, partial densities summed in the FFT's first pass) and
    # the general A loader of the second GEMM
    _say("wide case grid 12^3, 136+12 orbitals")
    return Case("grid24_v8c32", name="wide", seed=55, grid=(12, 12, 12), box=6.0,
                n_occ=136, n_emp=12)


def test_apply_c_wide_valence(wide):
    import paper_2310_20103_amd as G
    _say("apply_c wide valence, fp64 / mixed / plain kernels")
    ctx = make_ctx(wide.sys, interval=(wide.lo, wide.hi))
    try:
        assert ctx.query(G.KEY_N_VC) == 136 * 12
        x = gi.random_pair_vectors(6, wide.wl.n_vc, seed=14)
        ref = x @ wide.pr.C.T
        xt = torch.tensor(x, device="cuda")
        got64 = ctx.apply_c(xt).cpu().numpy()
        gotmx = ctx.apply_c(xt, "mixed").cpu().numpy()
        ctx.set_option(G.KEY_KERNELS, 0)
        plain = ctx.apply_c(xt, "mixed").cpu().numpy()
    finally:
        ctx.close()
    assert relerr(got64, ref) <= 1e-11
    assert relerr(gotmx, ref) <= 1e-3
    dk = ref - wide.pr.delta ** 2 * x
    assert relerr(gotmx - wide.pr.delta ** 2 * x, dk) <= 2e-2
    # the plain kernels round the 16-bit operands in another order: their
    # coupling parts agree to the same 16-bit bar
    d2x = wide.pr.delta ** 2 * x
    assert relerr(gotmx - d2x, plain - d2x) <= 2e-2


def test_sigma_wide_valence(wide):
    _say("sigma wide valence fp64, 2 QP states, L = 8")
    wl = wide.wl
    om = np.linspace(-15, 15, 31)
    ctx = make_ctx(wide.sys, interval=(wide.lo, wide.hi))
    try:
        got = ctx.sigma_c(wide.sys.qp_states, om, wl.eta, 8)
    finally:
        ctx.close()
    for i, m in enumerate(wide.sys.qp_states):
        ref = wide.pr.sigma_lanczos(int(m), om, wl.eta, 8, wide.lo, wide.hi, wl.poly_degree)
        assert relerr(got[i], ref) <= 1e-8


# ------------------------------------------------------------------ kernel variants
@pytest.mark.parametrize("which", ["small", "ragged"])
def test_mfma_matches_plain_kernels(request, which):
    """The MFMA GEMMs against the plain FMA tiles on the same inputs."""
    import paper_2310_20103_amd as G
    case = request.getfixturevalue(which)
    ctx = request.getfixturevalue("ctx_" + which)
    _say("mfma vs plain", which)
    x = torch.tensor(gi.random_pair_vectors(5, case.wl.n_vc, seed=9), device="cuda")
    out = {}
    for kern in (0, 1):
        ctx.set_option(G.KEY_KERNELS, kern)
        out[kern] = {p: ctx.apply_c(x, p).cpu().numpy() for p in ("fp64", "mixed")}
    assert relerr(out[1]["fp64"], out[0]["fp64"]) <= 1e-13
    assert relerr(out[1]["mixed"], out[0]["mixed"]) <= 1e-5
    # both block tiles of the second BF16 GEMM (256 is the default)
    try:
        ctx.set_option(G.KEY_BF16_TILE, 128)
        assert ctx.query(G.KEY_BF16_TILE) == 128
        m128 = ctx.apply_c(x, "mixed").cpu().numpy()
    finally:
        ctx.set_option(G.KEY_BF16_TILE, 256)
    assert relerr(m128, out[0]["mixed"]) <= 1e-5


# ------------------------------------------------------------------ graphs and tuner
def test_graph_replay_matches_eager(small):
    """Each Lanczos step replays the captured p_g(C) graph with eager vector
    kernels and host synchronisation in between; every replay feeds a_k, so
    equal coefficient arrays check every replay against eager launches."""
    import paper_2310_20103_amd as G
    _say("graph replay vs eager")
    m = int(small.sys.qp_states[0])
    ns = list(range(0, small.wl.n_orb, 2))
    out = {}
    for graphs in (0, 1):
        ctx = make_ctx(small.sys, interval=(small.lo, small.hi), block=7)
        try:
            ctx.set_option(G.KEY_GRAPHS, graphs)
            for p in ("fp64", "mixed"):
                ctx.set_precision(p)
                out[(graphs, p)] = ctx.lanczos_pairs([m] * len(ns), ns, [24] * len(ns))
        finally:
            ctx.close()
    for p in ("fp64", "mixed"):
        for a, b in zip(out[(0, p)], out[(1, p)]):
            assert np.array_equal(a, b)


def test_autotuner_mixed_tile(small):
    """The mixed product's tuner also picks the second GEMM's tile; a tile set
    by the caller is kept."""
    import paper_2310_20103_amd as G
    _say("autotuner, mixed tile")
    wl = small.wl
    ctx = make_ctx(small.sys, precision="mixed", interval=(small.lo, small.hi), block=0)
    try:
        got = ctx.sigma_c(small.sys.qp_states[:1], small.sys.omega_ev, wl.eta, 8)
        assert ctx.query(G.KEY_TUNED_TILE) in (128, 256)
        assert ctx.query(G.KEY_BF16_TILE) == ctx.query(G.KEY_TUNED_TILE)
        ctx.set_option(G.KEY_BF16_TILE, 128)
        got128 = ctx.sigma_c(small.sys.qp_states[:1], small.sys.omega_ev, wl.eta, 8)
        assert ctx.query(G.KEY_TUNED_TILE) == 128 and ctx.query(G.KEY_BF16_TILE) == 128
    finally:
        ctx.close()
    ref = small.pr.sigma_lanczos(int(small.sys.qp_states[0]), small.sys.omega_ev, wl.eta, 8,
                                 small.lo, small.hi, wl.poly_degree)
    assert np.max(np.abs(got[0] - ref)) <= 1e-3
    assert np.max(np.abs(got128[0] - ref)) <= 1e-3


def test_autotuner_choice(small, ctx_small):
    import paper_2310_20103_amd as G
    _say("autotuner")
    wl = small.wl
    ctx_small.sigma_c(small.sys.qp_states[:1], small.sys.omega_ev[:4], wl.eta, 2)
    assert ctx_small.query(G.KEY_TUNED_BLOCK) in (32, 64, 128, 256)
    assert 1 <= ctx_small.query(G.KEY_TUNED_SPLITK) <= 32
    assert ctx_small.query(G.KEY_TUNED_TILE) in (128, 256)


# ------------------------------------------------------------------ schedulers
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("reorth", ["full", "local"])
def test_table_scheduler_matches_host_scheduler(small, precision, reorth):
    """The scheduler that uploads its refill schedule once and replays a graph
    of the whole Lanczos step gives bitwise the coefficients of the
    host-driven loop (same kernels in the same order): uneven lengths over
    3 slots, so slots retire, are refilled mid-run and fall idle at the end;
    also with graphs off and on the C route (quadrature); and it matches the
    oracle."""
    import paper_2310_20103_amd as G
    _say("table vs host scheduler", precision, reorth)
    m = int(small.sys.qp_states[0])
    ns = [4, 9, 30, 17, 2, 22, 35, 11]
    lens = [6, 40, 12, 25, 3, 64, 1, 19]
    out = {}
    with make_ctx(small.sys, precision=precision, interval=(small.lo, small.hi), block=3,
                  reorth=reorth) as ctx:
        assert ctx.query(G.KEY_SCHEDULER) == 1
        for sched, graphs in ((1, 1), (0, 1), (1, 0)):
            ctx.set_option(G.KEY_SCHEDULER, sched)
            ctx.set_option(G.KEY_GRAPHS, graphs)
            out[(sched, graphs)] = ctx.lanczos_pairs([m] * len(ns), ns, lens)
            assert ctx.query(G.KEY_LAST_C_MATVECS) == sum(lens) * small.wl.poly_degree
        if precision == "fp64":
            ctx.set_quadrature(True)
            q = {}
            for sched in (1, 0):
                ctx.set_option(G.KEY_SCHEDULER, sched)
                ctx.set_option(G.KEY_GRAPHS, 1)
                q[sched] = ctx.lanczos_pairs([m] * len(ns), ns, lens)
            for x, y in zip(q[1], q[0]):
                assert np.array_equal(x, y)
    ref = out[(0, 1)]
    for key in ((1, 1), (1, 0)):
        for x, y in zip(out[key], ref):
            assert np.array_equal(x, y), key
    a, b, n2, ol = ref
    for i, n in enumerate(ns):
        ra, rb, rn2 = small.pr.lanczos_coeffs(m, lens[i], small.lo, small.hi,
                                              small.wl.poly_degree, n_list=[n])[0]
        assert ol[i] == lens[i]
        if precision == "fp64" and reorth == "full":
            assert relerr(a[i, :lens[i]], ra) <= 1e-9
        else:
            assert relerr(a[i, :min(6, lens[i])], ra[:6]) <= 1e-4
