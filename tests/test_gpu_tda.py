"""GPU Tamm-Dancoff path (GWL_KEY_TDA) against the oracle.

* coupling vectors are (nm|vc) (no Delta^1/2);
* Lanczos coefficients on A = Delta + K match the oracle's;
* Sigma: FP64 <= 1e-8 relative on the small and the ragged case (every
  dimension with a tail against the tiles), mixed precision <= 1e-3 eV on
  the smooth stress variant; uneven lengths with idle slots;
* switching the option back restores the full method; the adjoint refuses.
"""
import numpy as np
import pytest

import gw_inputs as gi
import oracle
from oracle import tda as T

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(*a):
    print("[case]", *a, flush=True)


def relerr(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / max(np.max(np.abs(b)), 1e-300))


class Case:
    def __init__(self, base, **kw):
        self.wl = gi.workload(base, **kw)
        self.sys = gi.make_system(self.wl)
        self.pr = oracle.Problem(self.sys.phi, self.sys.energies_ev, self.wl.n_occ,
                                 self.wl.grid, self.wl.h)


def make_ctx(case, precision="fp64", **kw):
    import paper_2310_20103_amd as G
    wl = case.wl
    lo, hi = oracle.default_interval(case.pr)
    ctx = G.Context(case.sys.phi, case.sys.energies_ev, wl.n_occ, wl.grid,
                    tuple(n * wl.h for n in wl.grid), precision=precision,
                    poly_degree=wl.poly_degree, poly_lo=lo, poly_hi=hi, **kw)
    ctx.set_tda(True)
    return ctx


@pytest.fixture(scope="module")
def small():
    _say("tda small case")
    return Case("grid24_v8c32", n_lanczos=24, n_omega=41)


@pytest.fixture(scope="module")
def ragged():
    _say("tda ragged case 12x18x8, 5+19")
    return Case("grid24_v8c32", name="ragged", seed=77, grid=(12, 18, 8), box=7.0,
                n_occ=5, n_emp=19, n_lanczos=16, n_omega=33)


def test_coupling_is_eri(small):
    _say("tda coupling")
    ctx = make_ctx(small)
    try:
        m = int(small.sys.qp_states[0])
        ns = [0, 3, 17, 39]
        got = ctx.coupling([m] * len(ns), ns).cpu().numpy()
        ref = T.eri_vectors(small.pr, m, ns)
        assert relerr(got, ref) <= 1e-11
    finally:
        ctx.close()


def test_lanczos_coefficients(small):
    _say("tda lanczos coefficients")
    ctx = make_ctx(small)
    try:
        m = int(small.sys.qp_states[1])
        ns = [2, 9, 33]
        a, b, n2, ol = ctx.lanczos_pairs([m] * len(ns), ns, [12] * len(ns))
        ref = T.lanczos_coeffs_tda(small.pr, m, 12, n_list=ns)
        for i, (ra, rb, rn2) in enumerate(ref):
            assert ol[i] == len(ra)
            assert abs(n2[i] - rn2) <= 1e-11 * rn2
            assert relerr(a[i, :len(ra)], ra) <= 1e-10
            assert relerr(b[i, :len(rb)], rb) <= 1e-9
    finally:
        ctx.close()


@pytest.mark.parametrize("which", ["small", "ragged"])
def test_sigma_fp64(request, which):
    case = request.getfixturevalue(which)
    _say("tda sigma fp64", which)
    wl = case.wl
    ctx = make_ctx(case)
    try:
        got = ctx.sigma_c(case.sys.qp_states, case.sys.omega_ev, wl.eta, wl.n_lanczos)
    finally:
        ctx.close()
    for i, m in enumerate(case.sys.qp_states):
        ref = T.sigma_tda_lanczos(case.pr, int(m), case.sys.omega_ev, wl.eta, wl.n_lanczos)
        assert relerr(got[i], ref) <= 1e-8


def test_sigma_full_length_is_exact():
    """L = N_vc reproduces the eigendecomposition of A."""
    _say("tda full length tiny 2+3")
    case = Case("grid24_v8c32", name="tiny", seed=5, grid=(8, 8, 8), box=5.0, n_occ=2,
                n_emp=3, n_lanczos=6, n_omega=21)
    ctx = make_ctx(case)
    try:
        m = int(case.sys.qp_states[0])
        got = ctx.sigma_c([m], case.sys.omega_ev, case.wl.eta, 6)[0]
    finally:
        ctx.close()
    ref = T.sigma_tda_exact(case.pr, m, case.sys.omega_ev, case.wl.eta)
    assert relerr(got, ref) <= 1e-9


def test_sigma_mixed_smooth():
    _say("tda sigma mixed smooth")
    case = Case("grid24_v8c32", name="smooth", n_lanczos=24, n_omega=41, smooth_sigma=1.0)
    wl = case.wl
    ctx = make_ctx(case, precision="mixed")
    try:
        got = ctx.sigma_c(case.sys.qp_states, case.sys.omega_ev, wl.eta, wl.n_lanczos)
    finally:
        ctx.close()
    for i, m in enumerate(case.sys.qp_states):
        ref = T.sigma_tda_lanczos(case.pr, int(m), case.sys.omega_ev, wl.eta, wl.n_lanczos)
        assert np.max(np.abs(ref)) > 0.1
        assert np.max(np.abs(got[i] - ref)) <= 1e-3


def test_uneven_lengths_and_switch_back(small):
    _say("tda uneven lengths block 2, then full method")
    import paper_2310_20103_amd as G
    ctx = make_ctx(small, block=2)
    try:
        m = int(small.sys.qp_states[0])
        ns = [1, 8, 21, 30, 5]
        lens = [3, 20, 7, 14, 1]
        a, b, n2, ol = ctx.lanczos_pairs([m] * len(ns), ns, lens)
        for i, n in enumerate(ns):
            ra, rb, rn2 = T.lanczos_coeffs_tda(small.pr, m, lens[i], n_list=[n])[0]
            assert ol[i] == lens[i]
            assert relerr(a[i, :lens[i]], ra) <= 1e-10
        with pytest.raises(G.GwlError):
            ctx.sigma_c_vjp([m], small.sys.omega_ev[:4], 0.1, 4, np.ones((1, 4)))
        ctx.set_tda(False)
        assert ctx.query(G.KEY_TDA) == 0
        lo, hi = oracle.default_interval(small.pr)
        got = ctx.sigma_c([m], small.sys.omega_ev, small.wl.eta, 8)[0]
        ref = small.pr.sigma_lanczos(m, small.sys.omega_ev, small.wl.eta, 8, lo, hi,
                                     small.wl.poly_degree)
        assert relerr(got, ref) <= 1e-8
    finally:
        ctx.close()
