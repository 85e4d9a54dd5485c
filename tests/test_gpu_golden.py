"""The GPU path against the stored oracle values of tests/golden/:
Sigma^corr of the 24^3, 8 + 32 workload in FP64 (<= 1e-8 relative, the
parity bar) and the K-means points (equal)."""
import os

import numpy as np
import pytest

import gw_inputs as gi

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_small_sigma_golden():
    import paper_2310_20103_amd as G
    with open(os.path.join(HERE, "small_sigma.txt")) as f:
        head = [next(f) for _ in range(2)]
    lo = float(head[1].split("lo = ")[1].split()[0])
    hi = float(head[1].split("hi = ")[1].split()[0])
    t = np.loadtxt(os.path.join(HERE, "small_sigma.txt"), comments="#", ndmin=2)
    wl = gi.workload("grid24_v8c32")
    s = gi.make_system(wl)
    with G.Context(s.phi, s.energies_ev, wl.n_occ, wl.grid, tuple(n * wl.h for n in wl.grid),
                   poly_lo=lo, poly_hi=hi, poly_degree=wl.poly_degree) as ctx:
        got = ctx.sigma_c([int(s.qp_states[0])], t[:, 0], wl.eta, wl.n_lanczos)[0]
    ref = t[:, 1] + 1j * t[:, 2]
    assert np.max(np.abs(got - ref)) <= 1e-8 * np.max(np.abs(ref))


def test_kmeans_golden():
    import paper_2310_20103_amd as G
    with open(os.path.join(HERE, "kmeans_small.txt")) as f:
        lines = f.read().splitlines()
    n_as = int(lines[1].split()[-1])
    ref = np.array([int(x) for x in lines[2].split()])
    wl = gi.workload("grid24_v8c32", name="smooth", smooth_sigma=1.0)
    s = gi.make_system(wl)
    init = gi.random_grid_points(40, wl.n_r, seed=23)
    with G.Context(s.phi, s.energies_ev, wl.n_occ, wl.grid,
                   tuple(n * wl.h for n in wl.grid)) as ctx:
        pts, got_n = ctx.isdf_kmeans(init, 30)
    assert got_n == n_as
    assert np.array_equal(pts, ref)
