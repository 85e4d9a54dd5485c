"""The allocation-free entry point gwl_sigma_from_coeffs_noalloc against
gwl_sigma_from_coeffs, through the C ABI: two calls in a row (the second on a
smaller input, so the static array holds the first call's leftovers), both
bit for bit equal to the allocating entry point on the same coefficients, and
an over-size request refused with an error instead of a fault."""
import numpy as np
import pytest

import gw_inputs as gi

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print("[case]", *a, flush=True)


def _ctx(wl, s):
    import paper_2310_20103_amd as G
    box = tuple(n * wl.h for n in wl.grid)
    return G.Context(s.phi, s.energies_ev, wl.n_occ, wl.grid, box)


def test_noalloc_matches_allocating_entry_point():
    wl = gi.workload("grid24_v8c32")
    s = gi.make_system(wl)
    rng = np.random.default_rng(7)
    with _ctx(wl, s) as c:
        m = int(s.qp_states[0])
        n_all = np.arange(c.n_orb, dtype=np.int32)
        lens = rng.integers(1, 41, size=n_all.size).astype(np.int32)
        _say("noalloc: lanczos_pairs for", n_all.size, "pairs, lengths 1..40")
        a, b, n2, ol = c.lanczos_pairs(np.full(n_all.size, m), n_all, lens, ld=48)
        calls = [
            (n_all, a, b, n2, ol, s.omega_ev, wl.eta),
            (n_all[3:10], a[3:10, :20].copy(), b[3:10, :20].copy(), n2[3:10].copy(),
             np.minimum(ol[3:10], 20), np.linspace(-7.0, 9.0, 33), 0.05),
        ]
        for i, (n, aa, bb, nn2, ln, om, eta) in enumerate(calls):
            _say(f"noalloc call {i}: {len(n)} pairs, ld {aa.shape[1]}, {len(om)} frequencies")
            ref = c.sigma_from_coeffs(n, aa, bb, nn2, ln, om, eta)
            got = c.sigma_from_coeffs_noalloc(n, aa, bb, nn2, ln, om, eta)
            assert got.shape == ref.shape
            assert np.max(np.abs(ref)) > 0
            assert np.array_equal(got, ref), float(np.max(np.abs(got - ref)))


def test_noalloc_refuses_oversize_request():
    import paper_2310_20103_amd as G
    wl = gi.workload("grid24_v8c32")
    s = gi.make_system(wl)
    with _ctx(wl, s) as c:
        P, ld, nw = 40, 4000, 200  # 2.6 MB of coefficients + 40 x 200 x 16 B: fits
        n = np.arange(P, dtype=np.int32) % c.n_orb
        a = np.zeros((P, ld))
        a[:, 0] = 1.0
        b = np.zeros((P, ld))
        n2 = np.ones(P)
        ln = np.ones(P, dtype=np.int32)
        om = np.linspace(-5, 5, nw)
        _say("noalloc: fitting request of", P, "pairs, ld", ld)
        ref = c.sigma_from_coeffs(n, a, b, n2, ln, om, 0.1)
        got = c.sigma_from_coeffs_noalloc(n, a, b, n2, ln, om, 0.1)
        assert np.array_equal(got, ref)
        # 600 pairs x ld 4000 is 38 MB of coefficients: over the 32 MiB array
        P = 600
        n = np.arange(P, dtype=np.int32) % c.n_orb
        a = np.zeros((P, ld))
        b = np.zeros((P, ld))
        _say("noalloc: over-size request of", P, "pairs, ld", ld)
        with pytest.raises(G.GwlError) as e:
            c.sigma_from_coeffs_noalloc(n, a, b, np.ones(P), np.ones(P, dtype=np.int32), om, 0.1)
        assert "scratch" in str(e.value)
