"""Parity at the large configuration: grid128_v512c1024 (128^3 grid, 48 bohr
box, 512 + 1,024 orbitals given in FP32, N_vc = 524,288, N_r = 2^21, so the
mixed second GEMM reads its FP16 orbitals from K panels and the FFT lines
are 128 points long), B = 128 pair vectors per product as in the large
benchmark, mixed precision and FP64 on the same context.  Against the
oracle on the FP32 orbitals widened to FP64:

* C x of 128 seeded vectors, row 0 whole (524,288 entries) against the
  oracle's matrix-free C x: FP64 <= 1e-10 relative; mixed <= 1e-3 relative,
  its coupling part C x - Delta^2 x <= 2e-2 relative;
* over all 128 vectors: the coupling part of the Gram matrix x_i . C x_j is
  symmetric and has a non-negative diagonal (FP64 1e-12, mixed 2e-3);
* the coupling vector P_nm of the first QP state for the last orbital n,
  whole, against the oracle's: FP64 <= 1e-10, mixed <= 1e-3.

The inputs take about a minute to draw and orthonormalise; the oracle
products take tens of seconds each on the host cores.
"""
import time

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


@pytest.fixture(scope="module")
def large():
    import paper_2310_20103_amd as G
    t = time.time()
    wl = gi.workload("grid128_v512c1024")
    phi32 = gi.make_orbitals(wl, dtype=np.float32, progress=_say)
    eps = gi.make_energies(wl)
    qp = gi.frontier_states(eps, wl.n_occ, wl.n_qp_occ, wl.n_qp_emp)
    _say(f"large inputs {time.time() - t:.1f}s")
    box = tuple(n * wl.h for n in wl.grid)
    t = time.time()
    # the interval only enters p_g(C), which these products do not use
    ctx = G.Context(phi32, eps, wl.n_occ, wl.grid, box, precision="mixed",
                    poly_degree=wl.poly_degree, poly_lo=0.02, poly_hi=0.8, reorth="full",
                    block=128)
    _say(f"large context {time.time() - t:.1f}s")
    pr = oracle.Problem(phi32, eps, wl.n_occ, wl.grid, wl.h, dense=False)
    del phi32
    yield wl, qp, ctx, pr
    ctx.close()


def test_large_apply_c(large):
    wl, qp, ctx, pr = large
    _say("large C x, 128 vectors, fp64 and mixed")
    x = gi.random_pair_vectors(128, wl.n_vc, seed=14)
    xt = torch.tensor(x, device="cuda")
    d2x = pr.delta ** 2 * x
    got = {}
    for prec, sym_tol in (("fp64", 1e-12), ("mixed", 2e-3)):
        cx = ctx.apply_c(xt, prec).cpu().numpy()
        gk = x @ (cx - d2x).T
        asym = np.max(np.abs(gk - gk.T)) / np.max(np.abs(gk))
        _say(f"  {prec}: coupling Gram asymmetry {asym:.2e}, "
             f"min diagonal {np.min(np.diag(gk)):.3e}")
        assert asym <= sym_tol
        assert np.min(np.diag(gk)) >= -sym_tol * np.max(np.abs(gk))
        got[prec] = cx[0]
    del xt
    t = time.time()
    ref = pr.apply_c(x[0])
    dk = ref - d2x[0]
    _say(f"  oracle row 0: {time.time() - t:.1f}s; rel err fp64 {relerr(got['fp64'], ref):.2e}, "
         f"mixed {relerr(got['mixed'], ref):.2e}, "
         f"coupling part {relerr(got['mixed'] - d2x[0], dk):.2e}")
    assert relerr(got["fp64"], ref) <= 1e-10
    assert relerr(got["mixed"], ref) <= 1e-3
    assert relerr(got["mixed"] - d2x[0], dk) <= 2e-2


def test_large_coupling(large):
    wl, qp, ctx, pr = large
    m, n = int(qp[0]), wl.n_orb - 1
    _say("large coupling vector", m, n)
    got = {}
    for prec in ("fp64", "mixed"):
        ctx.set_precision(prec)
        try:
            got[prec] = ctx.coupling(np.array([m]), np.array([n])).cpu().numpy()
        finally:
            ctx.set_precision("mixed")
    t = time.time()
    ref = pr.coupling(m, [n])
    _say(f"  oracle {time.time() - t:.1f}s; rel err fp64 {relerr(got['fp64'], ref):.2e}, "
         f"mixed {relerr(got['mixed'], ref):.2e}")
    assert relerr(got["fp64"], ref) <= 1e-10
    assert relerr(got["mixed"], ref) <= 1e-3
