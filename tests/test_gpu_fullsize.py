"""Parity at the headline size, in the launch configuration the benchmark
times: grid64_v128c512 (64^3 grid, 24 bohr box, 128 + 512 orbitals,
N_vc = 65536), B = 128 pair vectors per product, mixed precision (FP16
operands in both GEMMs) and the same batch in FP64.  Sampled outputs against
the oracle computed one at a time by its matrix-free FP64 route:

* C x of 128 seeded vectors, rows 0, 77 and 127: FP64 <= 1e-10 relative;
  mixed <= 1e-3 relative, and its coupling part C x - Delta^2 x <= 2e-2
  relative (the bars of the small cases: FP16 operand rounding of about
  2^-11 per factor, averaged over the grid sums, on a part that is a small
  fraction of C x);
* coupling vectors P_nm of the first QP state for n = 0, 300, 639 (FP64
  <= 1e-10);
* all 128 vectors of a second batch: the Gram matrix x_i . C x_j is
  symmetric and x . C x >= x . Delta^2 x, in FP64 (1e-12) and mixed
  (2e-3 on the coupling part; measured 1.6e-4);
* two Lanczos steps on p_7(C) for the benchmark's first batch (m = first QP
  state, n = 0..127), pairs 0 and 77: a_0, a_1, b_1 and ||P||^2 against the
  oracle's Lanczos from the same start vector: FP64 <= 1e-9 relative, mixed
  <= 1e-3 relative;
* Sigma(omega, n) of the first QP state for n = 0 and 639 at L = 5 on the
  benchmark's 2,000 frequencies (Lanczos with full reorthogonalisation, then
  the continued fraction and assembly on the GPU) against the oracle's
  matrix-free Lanczos and continued fraction: FP64 <= 1e-8 relative; the
  mixed error is reported with the same 1e-3 relative bar (these white-noise
  couplings make Sigma far smaller than 1 meV, so the absolute bar would not
  bind).
"""
import time

import numpy as np
import pytest

import gw_inputs as gi
import oracle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

ROWS = (0, 77, 127)


def _say(*a):
    print("[case]", *a, flush=True)


def relerr(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / max(np.max(np.abs(b)), 1e-300))


@pytest.fixture(scope="module")
def full():
    import paper_2310_20103_amd as G
    t = time.time()
    wl = gi.workload("grid64_v128c512")
    phi = gi.make_orbitals(wl)
    eps = gi.make_energies(wl)
    qp = gi.frontier_states(eps, wl.n_occ, wl.n_qp_occ, wl.n_qp_emp)
    _say(f"full size inputs {time.time() - t:.1f}s")
    box = tuple(n * wl.h for n in wl.grid)
    ctx = G.Context(phi, eps, wl.n_occ, wl.grid, box, precision="mixed",
                    poly_degree=wl.poly_degree, reorth="full", block=128)
    pr = oracle.Problem(phi, eps, wl.n_occ, wl.grid, wl.h, dense=False)
    yield wl, phi, eps, qp, ctx, pr
    ctx.close()


def test_poisson_full_size(full):
    """The 64^3 in-place FFT passes against the oracle's Poisson solve, FP64 and
    FP32, with an odd field count (the last complex field carries one real
    field)."""
    wl, phi, eps, qp, ctx, pr = full
    _say("full size Poisson, 7 fields")
    f = gi.random_fields(7, wl.n_r, seed=21)
    ref = oracle.poisson.poisson(f, wl.grid, wl.h)
    v64 = ctx.poisson(torch.tensor(f, device="cuda"), "fp64").cpu().numpy()
    v32 = ctx.poisson(torch.tensor(f, dtype=torch.float32, device="cuda"),
                      "mixed").double().cpu().numpy()
    _say(f"  fp64 {relerr(v64, ref):.2e}, fp32 {relerr(v32, ref):.2e}")
    assert relerr(v64, ref) <= 1e-12
    assert relerr(v32, ref) <= 2e-6


def test_apply_c_full_size(full):
    wl, phi, eps, qp, ctx, pr = full
    _say("full size C x, 128 vectors, fp64 and mixed")
    x = gi.random_pair_vectors(128, wl.n_vc, seed=12)
    xt = torch.tensor(x, device="cuda")
    got64 = ctx.apply_c(xt, "fp64").cpu().numpy()
    gotmx = ctx.apply_c(xt, "mixed").cpu().numpy()
    for r in ROWS:
        t = time.time()
        ref = pr.apply_c(x[r])
        dk = ref - pr.delta ** 2 * x[r]
        _say(f"  oracle row {r}: {time.time() - t:.1f}s; rel err fp64 {relerr(got64[r], ref):.2e}, "
             f"mixed {relerr(gotmx[r], ref):.2e}, "
             f"coupling part {relerr(gotmx[r] - pr.delta ** 2 * x[r], dk):.2e}")
        assert relerr(got64[r], ref) <= 1e-10
        assert relerr(gotmx[r], ref) <= 1e-3
        assert relerr(gotmx[r] - pr.delta ** 2 * x[r], dk) <= 2e-2


def test_apply_c_symmetry_and_bound_full_size(full):
    """Properties that hold at any size, over all 128 vectors of the batch: the
    Gram matrix x_i . C x_j is symmetric (C is), and x . C x >= x . Delta^2 x
    (the coupling term 2 Delta^1/2 K Delta^1/2 is positive semidefinite)."""
    wl, phi, eps, qp, ctx, pr = full
    _say("full size C x symmetry and lower bound, 128 vectors")
    x = gi.random_pair_vectors(128, wl.n_vc, seed=13)
    xt = torch.tensor(x, device="cuda")
    d2x = pr.delta ** 2 * x
    for prec, sym_tol in (("fp64", 1e-12), ("mixed", 2e-3)):
        cx = ctx.apply_c(xt, prec).cpu().numpy()
        gk = x @ (cx - d2x).T  # coupling part of the Gram matrix
        asym = np.max(np.abs(gk - gk.T)) / np.max(np.abs(gk))
        _say(f"  {prec}: coupling Gram asymmetry {asym:.2e}, "
             f"min diagonal {np.min(np.diag(gk)):.3e}")
        assert asym <= sym_tol
        assert np.min(np.diag(gk)) >= -sym_tol * np.max(np.abs(gk))


def test_coupling_full_size(full):
    wl, phi, eps, qp, ctx, pr = full
    m = int(qp[0])
    ns = np.array([0, 300, wl.n_orb - 1])
    _say("full size coupling vectors", m, ns)
    got = ctx.coupling(np.full_like(ns, m), ns).cpu().numpy()
    ref = pr.coupling(m, list(ns))
    _say(f"  rel err {relerr(got, ref):.2e}")
    assert relerr(got, ref) <= 1e-10


def test_lanczos_full_size(full):
    wl, phi, eps, qp, ctx, pr = full
    m = int(qp[0])
    lo, hi = ctx.interval
    _say("full size Lanczos, 128 pairs x 2 steps, mixed then fp64")
    B = 128
    amx, bmx, nmx, _ = ctx.lanczos_pairs([m] * B, list(range(B)), [2] * B)
    ctx.set_precision("fp64")
    try:
        a64, b64, n64, _ = ctx.lanczos_pairs([m] * B, list(range(B)), [2] * B)
    finally:
        ctx.set_precision("mixed")
    for i in (0, 77):
        t = time.time()
        (ra, rb, rn2), = pr.lanczos_coeffs(m, 2, lo, hi, wl.poly_degree, reorth="full",
                                            route="matfree", n_list=[i])
        _say(f"  oracle pair {i}: {time.time() - t:.1f}s")
        ref = np.concatenate([ra, rb, [rn2]])
        got64 = np.concatenate([a64[i, :2], b64[i, :1], [n64[i]]])
        gotmx = np.concatenate([amx[i, :2], bmx[i, :1], [nmx[i]]])
        _say(f"  pair {i}: max rel err fp64 {np.max(np.abs(got64 - ref) / np.abs(ref)):.2e}, "
             f"mixed {np.max(np.abs(gotmx - ref) / np.abs(ref)):.2e}")
        assert np.all(np.abs(got64 - ref) <= 1e-9 * np.abs(ref))
        assert np.all(np.abs(gotmx - ref) <= 1e-3 * np.abs(ref))


def test_sigma_full_size(full):
    from oracle import sigma as S
    wl, phi, eps, qp, ctx, pr = full
    m = int(qp[0])
    lo, hi = ctx.interval
    L = 5
    ns = [0, wl.n_orb - 1]
    om = gi.omega_grid(wl)
    _say(f"full size Sigma(omega, n), m={m}, n={ns}, L={L}, {len(om)} omega")
    got = {}
    for prec in ("fp64", "mixed"):
        ctx.set_precision(prec)
        try:
            a, b, n2, ol = ctx.lanczos_pairs([m] * len(ns), ns, [L] * len(ns))
            got[prec] = ctx.sigma_from_coeffs(ns, a, b, n2, ol, om, wl.eta)
        finally:
            ctx.set_precision("mixed")
    for i, n in enumerate(ns):
        t = time.time()
        (ra, rb, rn2), = pr.lanczos_coeffs(m, L, lo, hi, wl.poly_degree, reorth="full",
                                            route="matfree", n_list=[n])
        ref = S.sigma_n_from_tridiag(ra, rb, rn2, om / S.HARTREE_EV, pr.eps[n], pr.eta(n),
                                     wl.eta / S.HARTREE_EV) * S.HARTREE_EV
        e64, emx = relerr(got["fp64"][i], ref), relerr(got["mixed"][i], ref)
        _say(f"  n={n}: oracle {time.time() - t:.1f}s, max|Sigma| {np.max(np.abs(ref)):.3e} eV, "
             f"rel err fp64 {e64:.2e}, mixed {emx:.2e} "
             f"(abs {np.max(np.abs(got['mixed'][i] - ref)):.2e} eV)")
        assert e64 <= 1e-8
        assert emx <= 1e-3
