"""Stored expected values under tests/golden/ (written by
tests/golden/make_golden.py from the oracle alone).

* single_pole.txt holds Eq. (7) for one pair and one pole; the continued-fraction
  route of Eqs. (12) and (14) with a 1 x 1 tridiagonal, and Eq. (11), must
  reproduce it (two other formulas for the same quantity);
* small_sigma.txt and kmeans_small.txt are regression values: the oracle must
  still produce them (a change of the oracle's arithmetic shows up here).
"""
import os

import numpy as np

import gw_inputs as gi
import oracle
from oracle import isdf as I
from oracle import sigma as S

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _rows(name):
    return np.loadtxt(os.path.join(HERE, name), comments="#", ndmin=2)


def test_single_pole_routes():
    t = _rows("single_pole.txt")
    for eta_n in (1.0, -1.0):
        sel = t[t[:, 0] == eta_n]
        e_n, om = sel[0, 1], sel[:, 2]
        ref = sel[:, 3] + 1j * sel[:, 4]
        cf = S.sigma_n_from_tridiag(np.array([0.5]), np.zeros(0), 0.09, om, e_n, eta_n, 0.01)
        e11 = S.sigma_n_eq11(om, e_n, eta_n, 0.01, np.array([0.09]), np.array([0.5]))
        assert np.max(np.abs(cf - ref)) <= 1e-13 * np.max(np.abs(ref))
        assert np.max(np.abs(e11 - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_small_sigma_regression():
    with open(os.path.join(HERE, "small_sigma.txt")) as f:
        head = [next(f) for _ in range(2)]
    lo = float(head[1].split("lo = ")[1].split()[0])
    hi = float(head[1].split("hi = ")[1].split()[0])
    t = _rows("small_sigma.txt")
    wl = gi.workload("grid24_v8c32")
    s = gi.make_system(wl)
    pr = oracle.Problem(s.phi, s.energies_ev, wl.n_occ, wl.grid, wl.h)
    m = int(s.qp_states[0])
    lz = pr.sigma_lanczos(m, t[:, 0], wl.eta, wl.n_lanczos, lo, hi, wl.poly_degree)
    ex = pr.sigma_exact(m, t[:, 0], wl.eta)
    ref_lz = t[:, 1] + 1j * t[:, 2]
    ref_ex = t[:, 3] + 1j * t[:, 4]
    assert np.max(np.abs(lz - ref_lz)) <= 1e-12 * np.max(np.abs(ref_lz))
    assert np.max(np.abs(ex - ref_ex)) <= 1e-12 * np.max(np.abs(ref_ex))


def test_kmeans_regression():
    with open(os.path.join(HERE, "kmeans_small.txt")) as f:
        lines = f.read().splitlines()
    n_as = int(lines[1].split()[-1])
    ref = np.array([int(x) for x in lines[2].split()])
    wl = gi.workload("grid24_v8c32", name="smooth", smooth_sigma=1.0)
    s = gi.make_system(wl)
    init = gi.random_grid_points(40, wl.n_r, seed=23)
    spacing = tuple((n * wl.h) / n for n in wl.grid)
    pts, got_n = I.kmeans_points(I.kmeans_weights(s.phi, wl.n_occ), wl.grid, spacing, init, 30)
    assert got_n == n_as
    assert np.array_equal(pts, ref)
