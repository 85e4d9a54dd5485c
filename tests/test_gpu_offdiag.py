"""GPU off-diagonal self-energy (gwl_sigma_c_offdiag) against the oracle.

* FP64: <= 1e-8 relative to the oracle's polarised Lanczos route (small,
  ragged and smooth cases);
* m2 = m reproduces gwl_sigma_c's diagonal element, and Sigma_mm2 = Sigma_m2m
  (both to 1e-12 relative: the runs differ only in rounding);
* mixed precision within 1 meV of the oracle on the smooth (eV-sized) case;
* the Tamm-Dancoff option: m2 = m gives the Tamm-Dancoff diagonal element.
"""
import numpy as np
import pytest

import gw_inputs as gi
import oracle
from oracle import offdiag as O

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
        self.lo, self.hi = oracle.default_interval(self.pr)
        q = [int(x) for x in self.sys.qp_states]
        self.m, self.m2 = q[0], q[-1]


def make_ctx(case, precision="fp64", **kw):
    import paper_2310_20103_amd as G
    wl = case.wl
    return G.Context(case.sys.phi, case.sys.energies_ev, wl.n_occ, wl.grid,
                     tuple(n * wl.h for n in wl.grid), precision=precision,
                     poly_degree=wl.poly_degree, poly_lo=case.lo, poly_hi=case.hi, **kw)


@pytest.fixture(scope="module")
def small():
    _say("offdiag small case")
    return Case("grid24_v8c32", n_lanczos=20, n_omega=41)


@pytest.fixture(scope="module")
def ragged():
    _say("offdiag ragged case 12x18x8, 5+19")
    return Case("grid24_v8c32", name="ragged", seed=77, grid=(12, 18, 8), box=7.0, n_occ=5,
                n_emp=19, n_lanczos=12, n_omega=33)


@pytest.fixture(scope="module")
def smooth():
    _say("offdiag smooth case")
    return Case("grid24_v8c32", name="smooth", smooth_sigma=1.0, n_lanczos=24, n_omega=41)


@pytest.mark.parametrize("which", ["small", "ragged", "smooth"])
def test_offdiag_fp64(request, which):
    case = request.getfixturevalue(which)
    wl = case.wl
    _say("offdiag fp64", which, case.m, case.m2)
    with make_ctx(case) as ctx:
        got = ctx.sigma_c_offdiag(case.m, case.m2, case.sys.omega_ev, wl.eta, wl.n_lanczos)
    ref = O.sigma_lanczos_offdiag(case.pr, case.m, case.m2, case.sys.omega_ev, wl.eta,
                                  wl.n_lanczos, case.lo, case.hi, wl.poly_degree)
    assert np.max(np.abs(ref)) > 1e-6
    assert relerr(got, ref) <= 1e-8


def test_diagonal_and_symmetry(small):
    wl = small.wl
    _say("offdiag m2 = m, symmetry")
    with make_ctx(small) as ctx:
        diag = ctx.sigma_c([small.m], small.sys.omega_ev, wl.eta, wl.n_lanczos)[0]
        same = ctx.sigma_c_offdiag(small.m, small.m, small.sys.omega_ev, wl.eta, wl.n_lanczos)
        ab = ctx.sigma_c_offdiag(small.m, small.m2, small.sys.omega_ev, wl.eta, wl.n_lanczos)
        ba = ctx.sigma_c_offdiag(small.m2, small.m, small.sys.omega_ev, wl.eta, wl.n_lanczos)
    assert relerr(same, diag) <= 1e-12
    assert relerr(ba, ab) <= 1e-12


def test_offdiag_mixed_smooth(smooth):
    wl = smooth.wl
    _say("offdiag mixed smooth")
    with make_ctx(smooth, precision="mixed") as ctx:
        got = ctx.sigma_c_offdiag(smooth.m, smooth.m2, smooth.sys.omega_ev, wl.eta,
                                  wl.n_lanczos)
    ref = O.sigma_lanczos_offdiag(smooth.pr, smooth.m, smooth.m2, smooth.sys.omega_ev, wl.eta,
                                  wl.n_lanczos, smooth.lo, smooth.hi, wl.poly_degree)
    assert np.max(np.abs(ref)) > 1e-2
    assert np.max(np.abs(got - ref)) <= 1e-3


def test_offdiag_tda_diagonal(small):
    wl = small.wl
    _say("offdiag tda m2 = m")
    with make_ctx(small) as ctx:
        ctx.set_tda(True)
        diag = ctx.sigma_c([small.m], small.sys.omega_ev, wl.eta, wl.n_lanczos)[0]
        same = ctx.sigma_c_offdiag(small.m, small.m, small.sys.omega_ev, wl.eta, wl.n_lanczos)
    assert relerr(same, diag) <= 1e-12
