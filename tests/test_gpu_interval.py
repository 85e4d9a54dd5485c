"""The Chebyshev interval [lo, hi] of p_g ~ sqrt (paragraph after Eq. 12).

* The estimated upper end (40 Lanczos steps on C, largest Ritz value plus
  its residual bound, 1 % margin) lies above the largest eigenvalue of C
  from the oracle's eigh, carries a nonzero residual term when the
  recurrence does not exhaust the space, and is not loose (< 1.1 max eig).
* A caller-given interval that misses part of the spectrum -- hi at half the
  largest eigenvalue, or lo at twice the smallest -- makes every Lanczos
  entry point on p_g(C) fail with GWL_ENUMERIC (FP64 and mixed) instead of
  returning a Sigma built on an extrapolated polynomial; the Tamm-Dancoff
  and quadrature variants use no polynomial and still run.
* The precisions the ABI names but does not build are refused with
  GWL_EUNSUPPORTED.
"""
import numpy as np
import pytest

import gw_inputs as gi
import oracle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def small():
    _say("interval: small case grid24_v8c32")
    wl = gi.workload("grid24_v8c32", n_lanczos=24, n_omega=41)
    s = gi.make_system(wl)
    pr = oracle.Problem(s.phi, s.energies_ev, wl.n_occ, wl.grid, wl.h)
    lam_min, lam_max = pr.spectral_bounds()
    return wl, s, pr, lam_min, lam_max


def _ctx(s, wl, lo=0.0, hi=0.0, **kw):
    import paper_2310_20103_amd as G
    box = tuple(n * wl.h for n in wl.grid)
    return G.Context(s.phi, s.energies_ev, wl.n_occ, wl.grid, box, poly_degree=wl.poly_degree,
                     poly_lo=lo, poly_hi=hi, **kw)


def test_estimated_upper_end(small):
    import paper_2310_20103_amd as G
    wl, s, pr, lam_min, lam_max = small
    with _ctx(s, wl) as c:
        lo, hi = c.interval
        resid = c.query(G.KEY_HI_RESIDUAL)
    _say(f"estimate: hi {hi:.6f}, lambda_max {lam_max:.6f}, residual {resid:.3e}; "
         f"lo {lo:.6f}, lambda_min {lam_min:.6f}")
    assert lo <= lam_min
    assert lam_max <= hi <= 1.1 * lam_max
    assert resid > 0.0


@pytest.mark.parametrize("bad", ["hi_half", "lo_double"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_interval_violation_is_an_error(small, bad, precision):
    import paper_2310_20103_amd as G
    wl, s, pr, lam_min, lam_max = small
    lo0, hi0 = oracle.default_interval(pr)
    lo, hi = (lo0, 0.5 * lam_max) if bad == "hi_half" else (2.0 * lam_min, hi0)
    _say("interval violation", bad, precision, f"[{lo:.4f}, {hi:.4f}]")
    m = int(s.qp_states[0])
    with _ctx(s, wl, lo, hi, precision=precision) as c:
        with pytest.raises(G.GwlError) as e:
            c.sigma_c([m], s.omega_ev, wl.eta, wl.n_lanczos)
        assert e.value.code == G.binding.GWL_ENUMERIC
        assert "interval" in str(e.value)
        with pytest.raises(G.GwlError) as e:
            c.lanczos_pairs([m] * 4, [0, 5, 9, 30], [wl.n_lanczos] * 4)
        assert e.value.code == G.binding.GWL_ENUMERIC
        with pytest.raises(G.GwlError) as e:
            c.sigma_c_offdiag(m, int(s.qp_states[1]), s.omega_ev, wl.eta, wl.n_lanczos)
        assert e.value.code == G.binding.GWL_ENUMERIC
        # the context stays usable; variants without the polynomial still run
        c.set_tda(True)
        assert np.all(np.isfinite(c.sigma_c([m], s.omega_ev, wl.eta, wl.n_lanczos)))
        c.set_tda(False)
        if precision == "fp64":
            c.set_quadrature(True)
            assert np.all(np.isfinite(c.sigma_c([m], s.omega_ev, wl.eta, wl.n_lanczos)))
            c.set_quadrature(False)


def test_interval_that_brackets_the_spectrum_passes(small):
    wl, s, pr, lam_min, lam_max = small
    lo, hi = oracle.default_interval(pr)
    _say("interval bracketing the spectrum")
    m = int(s.qp_states[0])
    with _ctx(s, wl, lo, hi) as c:
        got = c.sigma_c([m], s.omega_ev, wl.eta, wl.n_lanczos)[0]
    ref = pr.sigma_lanczos(m, s.omega_ev, wl.eta, wl.n_lanczos, lo, hi, wl.poly_degree)
    assert np.max(np.abs(got - ref)) <= 1e-8 * np.max(np.abs(ref))


def test_unbuilt_precisions_refused(small):
    import paper_2310_20103_amd as G
    wl, s, pr, lam_min, lam_max = small
    lo, hi = oracle.default_interval(pr)
    for name in ("bf16x3", "fp32"):
        _say("precision refused:", name)
        with pytest.raises(G.GwlError) as e:
            _ctx(s, wl, lo, hi, precision=name)
        assert e.value.code == G.binding.GWL_EUNSUPPORTED
        with _ctx(s, wl, lo, hi) as c:
            with pytest.raises(G.GwlError) as e:
                c.set_precision(name)
            assert e.value.code == G.binding.GWL_EUNSUPPORTED
