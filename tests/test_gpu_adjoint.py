"""GPU vector-Jacobian product of Sigma_c (gwl_sigma_c_vjp).

* against central finite differences of the same GPU forward (FP64, no
  reorthogonalisation, fixed interval) along seeded random directions in the
  energies and in the orbital grid values: <= 1e-6 relative;
* against central finite differences of the oracle forward (same algorithm):
  <= 1e-5 relative;
* the energy gradient element by element against the oracle's closed form
  (Daleckii-Krein divided differences through the eigendecomposition of C)
  at L >= N_vc, where the recurrence is exhausted and Sigma_L equals the
  exact p_g(C) resolvent: <= 1e-6 of the largest element;
* 64 sampled orbital-gradient entries (8 per orbital) against central
  differences of the oracle forward in that one grid value: <= 1e-5;
* the forward Sigma returned with the gradient equals gwl_sigma_c;
* two runs agree bitwise;
* a case whose orbital contraction spans several tiles in every direction
  (odd N_v, two 64-wide conduction tiles, 18 grid tiles, two blocks of
  start vectors): directional derivatives against central differences of
  the GPU forward (<= 1e-6) and sampled entries against the oracle's;
* FP32 orbitals: the gradient comes back in FP32, equal to the FP64
  context's gradient on the same (rounded) orbitals, rounded;
* the split form (gwl_sigma_c_vjp_forward, then gwl_sigma_c_vjp_backward,
  twice, with two cotangents) equals the one-call VJP bitwise, over several
  blocks of start vectors, with one and with several checkpoint segments,
  for the full n-sum and a partial one; a backward with no kept forward, or
  after the block size changed, is an error.
"""
import numpy as np
import pytest

import gw_inputs as gi
import oracle
from oracle import adjoint as A

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def tiny():
    _say("adjoint tiny case 3+5 orbitals, grid 8x8x12")
    wl = gi.workload("grid24_v8c32", name="adj", seed=31, grid=(8, 8, 12), box=5.0,
                     n_occ=3, n_emp=5, n_qp_occ=1, n_qp_emp=1, n_lanczos=6, n_omega=9,
                     eta=0.3, smooth_sigma=1.0)
    s = gi.make_system(wl)
    pr = oracle.Problem(s.phi, s.energies_ev, wl.n_occ, wl.grid, wl.h)
    lo, hi = oracle.default_interval(pr, margin=0.05)
    om = np.linspace(-10, 10, wl.n_omega)
    rng = np.random.default_rng(5)
    G = rng.standard_normal((len(s.qp_states), len(om))) + 1j * rng.standard_normal(
        (len(s.qp_states), len(om)))
    return s, wl, lo, hi, om, G


def _box(wl):
    return tuple(n * wl.h for n in wl.grid)


def _ctx(phi, eps, wl, lo, hi, **kw):
    import paper_2310_20103_amd as G
    return G.Context(phi, eps, wl.n_occ, wl.grid, _box(wl), poly_lo=lo, poly_hi=hi,
                     poly_degree=wl.poly_degree, **kw)


def _gpu_loss(phi, eps, wl, lo, hi, qp, om, G):
    with _ctx(phi, eps, wl, lo, hi, reorth="none") as c:
        return A.loss(c.sigma_c(qp, om, wl.eta, wl.n_lanczos), G)


def test_vjp_against_fd_of_gpu_forward(tiny):
    s, wl, lo, hi, om, G = tiny
    qp = s.qp_states
    _say("vjp vs fd (gpu forward)")
    with _ctx(s.phi, s.energies_ev, wl, lo, hi) as c:
        sig, ge, go = c.sigma_c_vjp(qp, om, wl.eta, wl.n_lanczos, G)
        go = go.cpu().numpy()
    with _ctx(s.phi, s.energies_ev, wl, lo, hi, reorth="none") as c:
        ref = c.sigma_c(qp, om, wl.eta, wl.n_lanczos)
    assert np.max(np.abs(sig - ref)) <= 1e-12 * np.max(np.abs(ref))
    rng = np.random.default_rng(6)
    de = rng.standard_normal(wl.n_orb)
    h = 1e-5
    fd = (_gpu_loss(s.phi, s.energies_ev + h * de, wl, lo, hi, qp, om, G)
          - _gpu_loss(s.phi, s.energies_ev - h * de, wl, lo, hi, qp, om, G)) / (2 * h)
    assert abs(fd - ge @ de) <= 1e-6 * abs(fd) + 1e-12, (fd, ge @ de)
    dphi = rng.standard_normal(s.phi.shape) * np.mean(np.abs(s.phi))
    hp = 1e-5
    fdp = (_gpu_loss(s.phi + hp * dphi, s.energies_ev, wl, lo, hi, qp, om, G)
           - _gpu_loss(s.phi - hp * dphi, s.energies_ev, wl, lo, hi, qp, om, G)) / (2 * hp)
    got = float(np.sum(go * dphi))
    assert abs(fdp - got) <= 1e-6 * abs(fdp) + 1e-12, (fdp, got)


def test_vjp_against_oracle_fd(tiny):
    s, wl, lo, hi, om, G = tiny
    qp = s.qp_states
    _say("vjp vs oracle fd")
    with _ctx(s.phi, s.energies_ev, wl, lo, hi) as c:
        _, ge, go = c.sigma_c_vjp(qp, om, wl.eta, wl.n_lanczos, G)
        go = go.cpu().numpy()
    fwd_e = lambda e: A.loss(A.sigma_states(s.phi, e, wl.n_occ, wl.grid, wl.h, qp, om, wl.eta,
                                             wl.n_lanczos, lo, hi, wl.poly_degree), G)
    rng = np.random.default_rng(7)
    de = rng.standard_normal(wl.n_orb)
    fd = A.fd_directional(fwd_e, s.energies_ev, de, 1e-5)
    assert abs(fd - ge @ de) <= 1e-5 * abs(fd), (fd, ge @ de)
    fwd_p = lambda ph: A.loss(A.sigma_states(ph, s.energies_ev, wl.n_occ, wl.grid, wl.h, qp, om,
                                              wl.eta, wl.n_lanczos, lo, hi, wl.poly_degree), G)
    dphi = rng.standard_normal(s.phi.shape) * np.mean(np.abs(s.phi))
    fdp = A.fd_directional(fwd_p, s.phi, dphi, 1e-5)
    got = float(np.sum(go * dphi))
    assert abs(fdp - got) <= 1e-5 * abs(fdp), (fdp, got)


def test_vjp_deterministic(tiny):
    s, wl, lo, hi, om, G = tiny
    _say("vjp determinism")
    out = []
    for _ in range(2):
        with _ctx(s.phi, s.energies_ev, wl, lo, hi, block=4) as c:
            sig, ge, go = c.sigma_c_vjp(s.qp_states, om, wl.eta, wl.n_lanczos, G)
            out.append((sig, ge, go.cpu().numpy()))
    for a, b in zip(out[0], out[1]):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("n_lanczos", [7, 17])
def test_vjp_stored_iterates_match_checkpoints(tiny, n_lanczos):
    """The backward from iterates kept in the forward and the backward that
    recomputes them from checkpoints run the same kernels in the same order:
    bitwise-equal results (L = 7: a ragged last checkpoint segment; L = 17 >
    N_vc = 15: every recurrence ends early at an invariant subspace)."""
    import paper_2310_20103_amd as GW
    s, wl, lo, hi, om, G = tiny
    _say(f"vjp stored iterates vs checkpoints, L={n_lanczos}, block 4")
    out = {}
    for store in (1, 0):
        with _ctx(s.phi, s.energies_ev, wl, lo, hi, block=4) as c:
            assert c.query(GW.KEY_ADJOINT_STORED) == -1
            assert c.query(GW.KEY_ADJOINT_STORE) == 0  # default: recompute
            c.set_option(GW.KEY_ADJOINT_STORE, store)
            sig, ge, go = c.sigma_c_vjp(s.qp_states, om, wl.eta, n_lanczos, G)
            assert c.query(GW.KEY_ADJOINT_STORED) == store
            out[store] = (sig, ge, go.cpu().numpy())
    for a, b in zip(out[1], out[0]):
        assert np.all(np.isfinite(a))
        assert np.array_equal(a, b)


def test_vjp_energy_gradient_elementwise(tiny):
    s, wl, lo, hi, om, G = tiny
    qp = s.qp_states
    L = 20  # > N_vc = 15: every recurrence ends at an invariant subspace
    _say("vjp energy gradient element by element vs closed form, L", L)
    with _ctx(s.phi, s.energies_ev, wl, lo, hi) as c:
        sig, ge, _ = c.sigma_c_vjp(qp, om, wl.eta, L, G)
    sdg = A.sigma_dg_states(s.phi, s.energies_ev, wl.n_occ, wl.grid, wl.h, qp, om, wl.eta, lo,
                            hi, wl.poly_degree)
    assert np.max(np.abs(sig - sdg)) <= 1e-9 * np.max(np.abs(sdg))
    ref = A.dk_energy_gradient(s.phi, s.energies_ev, wl.n_occ, wl.grid, wl.h, qp, om, wl.eta,
                               lo, hi, wl.poly_degree, G)
    err = np.max(np.abs(ge - ref)) / np.max(np.abs(ref))
    _say(f"  max |grad| {np.max(np.abs(ref)):.3e}, rel err {err:.2e}")
    assert err <= 1e-6


def test_vjp_orbital_gradient_sampled_entries(tiny):
    s, wl, lo, hi, om, G = tiny
    qp = s.qp_states
    _say("vjp orbital gradient, 64 sampled entries vs oracle central differences")
    with _ctx(s.phi, s.energies_ev, wl, lo, hi) as c:
        _, _, go = c.sigma_c_vjp(qp, om, wl.eta, wl.n_lanczos, G)
        go = go.cpu().numpy()

    def loss_at(phi):
        return A.loss(A.sigma_states(phi, s.energies_ev, wl.n_occ, wl.grid, wl.h, qp, om,
                                     wl.eta, wl.n_lanczos, lo, hi, wl.poly_degree), G)

    rng = np.random.default_rng(8)
    step = 1e-4 * np.mean(np.abs(s.phi))
    worst = 0.0
    scale = np.max(np.abs(go))
    for a in range(wl.n_orb):
        for r in rng.choice(wl.n_r, size=8, replace=False):
            ph = s.phi.copy()
            ph[a, r] += step
            lp = loss_at(ph)
            ph[a, r] -= 2 * step
            lm = loss_at(ph)
            fd = (lp - lm) / (2 * step)
            dev = abs(fd - go[a, r])
            worst = max(worst, dev / scale)
            assert dev <= 1e-5 * scale + 1e-5 * abs(fd), (a, r, fd, go[a, r])
    _say(f"  max |dl/dphi| {scale:.3e}, worst deviation {worst:.2e} of it")


@pytest.fixture(scope="module")
def multi():
    _say("adjoint multi-tile case 5+70 orbitals, grid 12x12x16")
    wl = gi.workload("grid24_v8c32", name="adjm", seed=37, grid=(12, 12, 16), box=6.0,
                     n_occ=5, n_emp=70, n_qp_occ=1, n_qp_emp=1, n_lanczos=5, n_omega=7,
                     eta=0.3, smooth_sigma=1.0)
    s = gi.make_system(wl)
    pr = oracle.Problem(s.phi, s.energies_ev, wl.n_occ, wl.grid, wl.h)
    lo, hi = oracle.default_interval(pr, margin=0.05)
    om = np.linspace(-10, 10, wl.n_omega)
    rng = np.random.default_rng(11)
    G = rng.standard_normal((len(s.qp_states), len(om))) + 1j * rng.standard_normal(
        (len(s.qp_states), len(om)))
    return s, wl, lo, hi, om, G


def test_vjp_multi_tile(multi):
    s, wl, lo, hi, om, G = multi
    qp = s.qp_states
    _say("vjp multi-tile: directional vs gpu fd, block 64 over", len(qp) * wl.n_orb, "pairs")
    with _ctx(s.phi, s.energies_ev, wl, lo, hi, block=64) as c:
        _, ge, go = c.sigma_c_vjp(qp, om, wl.eta, wl.n_lanczos, G)
        go = go.cpu().numpy()
    assert np.all(np.isfinite(go)) and np.all(np.isfinite(ge))
    rng = np.random.default_rng(12)
    de = rng.standard_normal(wl.n_orb)
    h = 1e-5
    fd = (_gpu_loss(s.phi, s.energies_ev + h * de, wl, lo, hi, qp, om, G)
          - _gpu_loss(s.phi, s.energies_ev - h * de, wl, lo, hi, qp, om, G)) / (2 * h)
    _say(f"  energies: fd {fd:.6e}, vjp {ge @ de:.6e}")
    assert abs(fd - ge @ de) <= 1e-6 * abs(fd) + 1e-12, (fd, ge @ de)
    dphi = rng.standard_normal(s.phi.shape) * np.mean(np.abs(s.phi))
    fdp = (_gpu_loss(s.phi + h * dphi, s.energies_ev, wl, lo, hi, qp, om, G)
           - _gpu_loss(s.phi - h * dphi, s.energies_ev, wl, lo, hi, qp, om, G)) / (2 * h)
    got = float(np.sum(go * dphi))
    _say(f"  orbitals: fd {fdp:.6e}, vjp {got:.6e}")
    assert abs(fdp - got) <= 1e-6 * abs(fdp) + 1e-12, (fdp, got)

    def loss_at(phi):
        return A.loss(A.sigma_states(phi, s.energies_ev, wl.n_occ, wl.grid, wl.h, qp, om,
                                     wl.eta, wl.n_lanczos, lo, hi, wl.poly_degree), G)

    step = 1e-4 * np.mean(np.abs(s.phi))
    scale = np.max(np.abs(go))
    # occupied and empty orbitals, grid points in different tiles
    for a in (0, 4, 5, 40, 74):
        for r in rng.choice(wl.n_r, size=3, replace=False):
            ph = s.phi.copy()
            ph[a, r] += step
            lp = loss_at(ph)
            ph[a, r] -= 2 * step
            lm = loss_at(ph)
            fdr = (lp - lm) / (2 * step)
            assert abs(fdr - go[a, r]) <= 1e-5 * scale + 1e-5 * abs(fdr), (a, r, fdr, go[a, r])


def test_vjp_fp32_orbitals(tiny):
    s, wl, lo, hi, om, G = tiny
    phi32 = s.phi.astype(np.float32)
    _say("vjp with FP32 orbitals (host and device)")
    with _ctx(phi32.astype(np.float64), s.energies_ev, wl, lo, hi) as c:
        sig64, ge64, go64 = c.sigma_c_vjp(s.qp_states, om, wl.eta, wl.n_lanczos, G)
        go64 = go64.cpu().numpy()
    for src in (phi32, torch.from_numpy(phi32).cuda()):
        with _ctx(src, s.energies_ev, wl, lo, hi) as c:
            sig, ge, go = c.sigma_c_vjp(s.qp_states, om, wl.eta, wl.n_lanczos, G)
        assert go.dtype == torch.float32
        assert np.array_equal(sig, sig64)
        assert np.array_equal(ge, ge64)
        assert np.array_equal(go.cpu().numpy(), go64.astype(np.float32))


def test_vjp_range_adds_up(tiny):
    """The derivative of a partial n-sum: two ranges add up to the full VJP
    (the start vectors are independent), and the range derivative matches
    central differences of gwl_sigma_c_range."""
    s, wl, lo, hi, om, G = tiny
    qp = s.qp_states
    _say("vjp over n ranges [0, 3) + [3, 8) vs the full range")
    with _ctx(s.phi, s.energies_ev, wl, lo, hi, block=4) as c:
        sig, ge, go = c.sigma_c_vjp(qp, om, wl.eta, wl.n_lanczos, G)
        s1, ge1, go1 = c.sigma_c_vjp(qp, om, wl.eta, wl.n_lanczos, G, n_range=(0, 3))
        s2, ge2, go2 = c.sigma_c_vjp(qp, om, wl.eta, wl.n_lanczos, G, n_range=(3, 8))
        ref1 = c.sigma_c_range(qp, 0, 3, om, wl.eta, wl.n_lanczos)
    go, go1, go2 = go.cpu().numpy(), go1.cpu().numpy(), go2.cpu().numpy()
    assert np.max(np.abs(s1 + s2 - sig)) <= 1e-12 * np.max(np.abs(sig))
    assert np.max(np.abs(ge1 + ge2 - ge)) <= 1e-12 * np.max(np.abs(ge))
    assert np.max(np.abs(go1 + go2 - go)) <= 1e-12 * np.max(np.abs(go))

    def loss1(e):
        with _ctx(s.phi, e, wl, lo, hi, reorth="none") as c:
            return A.loss(c.sigma_c_range(qp, 0, 3, om, wl.eta, wl.n_lanczos), G)

    with _ctx(s.phi, s.energies_ev, wl, lo, hi, reorth="none") as c:
        ref1n = c.sigma_c_range(qp, 0, 3, om, wl.eta, wl.n_lanczos)
    assert np.max(np.abs(s1 - ref1n)) <= 1e-12 * np.max(np.abs(ref1n))
    assert np.max(np.abs(ref1 - ref1n)) <= 1e-6 * np.max(np.abs(ref1n))
    de = np.random.default_rng(13).standard_normal(wl.n_orb)
    h = 1e-5
    fd = (loss1(s.energies_ev + h * de) - loss1(s.energies_ev - h * de)) / (2 * h)
    assert abs(fd - ge1 @ de) <= 1e-6 * abs(fd) + 1e-12, (fd, ge1 @ de)


@pytest.mark.parametrize("n_lanczos,n_range", [(1, None), (7, None), (17, None), (10, (2, 7))])
def test_vjp_split_equals_one_call(tiny, n_lanczos, n_range):
    """Forward-then-backward against the one-call VJP (block 4: four blocks of
    start vectors; L = 1: one segment; L = 7, 10, 17: ragged segments; a
    partial n-sum)."""
    s, wl, lo, hi, om, G = tiny
    _say(f"vjp split vs one call, L={n_lanczos}, n_range={n_range}")
    G2 = np.conj(G[:, ::-1]) * 0.7
    with _ctx(s.phi, s.energies_ev, wl, lo, hi, block=4) as c:
        one = [c.sigma_c_vjp(s.qp_states, om, wl.eta, n_lanczos, g, n_range=n_range)
               for g in (G, G2)]
    with _ctx(s.phi, s.energies_ev, wl, lo, hi, block=4) as c:
        sig = c.sigma_c_vjp_forward(s.qp_states, om, wl.eta, n_lanczos, n_range=n_range)
        assert np.array_equal(sig, one[0][0])
        for g, (_, ge1, go1) in zip((G, G2), one):
            ge, go = c.sigma_c_vjp_backward(g)
            assert np.all(np.isfinite(ge))
            assert np.array_equal(ge, ge1)
            assert torch.equal(go, go1)


def test_vjp_backward_errors(tiny):
    import paper_2310_20103_amd as GW
    s, wl, lo, hi, om, G = tiny
    _say("vjp backward without a kept forward / after the block size changed")
    with _ctx(s.phi, s.energies_ev, wl, lo, hi) as c:
        with pytest.raises(GW.GwlError, match="no saved forward"):
            c.sigma_c_vjp_backward(G)
        c.sigma_c_vjp_forward(s.qp_states, om, wl.eta, wl.n_lanczos)
        c.set_option(GW.KEY_BLOCK, 4)
        with pytest.raises(GW.GwlError, match="changed since the saved forward"):
            c.sigma_c_vjp_backward(G)
        c.set_option(GW.KEY_BLOCK, 0)
        ge, _ = c.sigma_c_vjp_backward(G)
        assert np.all(np.isfinite(ge))
