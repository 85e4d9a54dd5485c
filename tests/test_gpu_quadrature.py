"""GPU Lanczos-on-C Gauss quadrature (GWL_KEY_QUADRATURE) against the oracle.

* Lanczos coefficients on C match the oracle's;
* Sigma in FP64 <= 1e-8 relative on the small and the ragged case; full
  length reproduces Eq. 7 with the exact eigenpairs of C; the mixed
  precision is refused;
* coefficients from gwl_lanczos_pairs assembled by gwl_sigma_from_coeffs
  equal gwl_sigma_c.
"""
import numpy as np
import pytest

import gw_inputs as gi
import oracle
from oracle import quadrature as Q

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
    ctx = G.Context(case.sys.phi, case.sys.energies_ev, wl.n_occ, wl.grid,
                    tuple(n * wl.h for n in wl.grid), precision=precision,
                    poly_degree=wl.poly_degree, **kw)
    ctx.set_quadrature(True)
    return ctx


@pytest.fixture(scope="module")
def small():
    _say("quadrature small case")
    return Case("grid24_v8c32", n_lanczos=28, n_omega=41)


@pytest.fixture(scope="module")
def ragged():
    _say("quadrature ragged case 12x18x8, 5+19")
    return Case("grid24_v8c32", name="ragged", seed=77, grid=(12, 18, 8), box=7.0,
                n_occ=5, n_emp=19, n_lanczos=21, n_omega=33)


def test_lanczos_on_c_coefficients(small):
    _say("quadrature coefficients")
    with make_ctx(small) as ctx:
        m = int(small.sys.qp_states[0])
        ns = [1, 12, 30]
        a, b, n2, ol = ctx.lanczos_pairs([m] * len(ns), ns, [14] * len(ns))
    ref = Q.lanczos_coeffs_c(small.pr, m, 14, n_list=ns)
    for i, (ra, rb, rn2) in enumerate(ref):
        assert ol[i] == len(ra)
        assert abs(n2[i] - rn2) <= 1e-11 * rn2
        assert relerr(a[i, :len(ra)], ra) <= 1e-9
        assert relerr(b[i, :len(rb)], rb) <= 1e-9


@pytest.mark.parametrize("which", ["small", "ragged"])
def test_sigma_fp64(request, which):
    case = request.getfixturevalue(which)
    _say("quadrature sigma fp64", which)
    wl = case.wl
    with make_ctx(case) as ctx:
        got = ctx.sigma_c(case.sys.qp_states, case.sys.omega_ev, wl.eta, wl.n_lanczos)
    for i, m in enumerate(case.sys.qp_states):
        ref = Q.sigma_quadrature(case.pr, int(m), case.sys.omega_ev, wl.eta, wl.n_lanczos)
        assert relerr(got[i], ref) <= 1e-8


def test_full_length_is_exact():
    _say("quadrature full length tiny 2+3")
    case = Case("grid24_v8c32", name="tiny", seed=5, grid=(8, 8, 8), box=5.0, n_occ=2,
                n_emp=3, n_lanczos=6, n_omega=21)
    with make_ctx(case) as ctx:
        m = int(case.sys.qp_states[0])
        got = ctx.sigma_c([m], case.sys.omega_ev, case.wl.eta, 6)[0]
    ref = case.pr.sigma_exact(m, case.sys.omega_ev, case.wl.eta)
    assert relerr(got, ref) <= 1e-9


def test_mixed_precision_refused(small):
    """The Ritz-value quadrature amplifies the mixed product's rounding (a CPU
    emulation gives 5e-3 eV at L = 28 on the smooth stress case), so the
    variant is FP64 only."""
    import paper_2310_20103_amd as G
    _say("quadrature refuses mixed precision")
    with make_ctx(small, precision="mixed") as ctx:
        with pytest.raises(G.GwlError):
            ctx.sigma_c(small.sys.qp_states[:1], small.sys.omega_ev, small.wl.eta, 8)


def test_coeffs_then_assembly(small):
    _say("quadrature coefficients + assembly")
    wl = small.wl
    m = int(small.sys.qp_states[1])
    ns = list(range(wl.n_orb))
    with make_ctx(small) as ctx:
        direct = ctx.sigma_c([m], small.sys.omega_ev, wl.eta, 10)[0]
        a, b, n2, ol = ctx.lanczos_pairs([m] * len(ns), ns, [10] * len(ns))
        per = ctx.sigma_from_coeffs(ns, a, b, n2, ol, small.sys.omega_ev, wl.eta)
    assert relerr(per.sum(axis=0), direct) <= 1e-12
