"""Writes the stored expected values under tests/golden/ (run from the repository
root: python tests/golden/make_golden.py).  Calls only the oracle and the seeded
input generators; nothing here comes from the GPU path.

* single_pole.txt: Eq. (7) for one pair and one pole (D = Omega, ||P|| = p):
  Sigma(w, n) = (p^2 / Omega) / (w - e_n + eta_n (Omega - i delta)), both
  occupation signs, hartree units;
* small_sigma.txt: Sigma^corr_mm(w) of the 24^3, 8 + 32 workload (seed 1000),
  QP state m = first frontier state, by the method (Lanczos on p_7(C) from
  P_nm, L = 64, Eqs. 10-14, the oracle's interval) and by Eq. (7) with the exact
  eigenpairs of C, at 11 frequencies in [-20, 20] eV, delta = 0.1 eV;
* kmeans_small.txt: weighted K-means interpolation points of the smooth variant
  of that workload (40 seeded random starting points, at most 30 updates).
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import gw_inputs as gi  # noqa: E402
import oracle  # noqa: E402
from oracle import isdf as I  # noqa: E402
from oracle import sigma as S  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def single_pole():
    om = np.linspace(-1.0, 1.0, 9)
    rows = []
    for eta_n, e_n in ((1.0, -0.4), (-1.0, 0.3)):
        v = S.sigma_n_poles(om, e_n, eta_n, 0.01, np.array([0.09]), np.array([0.5]))
        for w, x in zip(om, v):
            rows.append(f"{eta_n:+.1f} {e_n:+.3f} {w:+.6f} {x.real:+.17e} {x.imag:+.17e}")
    with open(os.path.join(HERE, "single_pole.txt"), "w") as f:
        f.write("# Eq. (7) for one pair and one pole, hartree: p^2 = 0.09, Omega = 0.5,\n"
                "# delta = 0.01; columns eta_n e_n omega Re(Sigma) Im(Sigma)\n")
        f.write("\n".join(rows) + "\n")


def small_sigma():
    wl = gi.workload("grid24_v8c32")
    s = gi.make_system(wl)
    pr = oracle.Problem(s.phi, s.energies_ev, wl.n_occ, wl.grid, wl.h)
    lo, hi = oracle.default_interval(pr)
    m = int(s.qp_states[0])
    om = np.linspace(-20.0, 20.0, 11)
    lz = pr.sigma_lanczos(m, om, wl.eta, wl.n_lanczos, lo, hi, wl.poly_degree)
    ex = pr.sigma_exact(m, om, wl.eta)
    with open(os.path.join(HERE, "small_sigma.txt"), "w") as f:
        f.write(f"# grid24_v8c32 (24^3, 12 bohr, 8 + 32 orbitals, seed 1000), m = {m}, "
                f"L = {wl.n_lanczos}, g = {wl.poly_degree}, delta = {wl.eta} eV\n"
                f"# interval lo = {lo!r} hi = {hi!r} (hartree^2)\n"
                "# columns omega_eV Re(Sigma_L) Im(Sigma_L) Re(Sigma_exact) Im(Sigma_exact), eV\n")
        for w, a, b in zip(om, lz, ex):
            f.write(f"{w:+.6f} {a.real:+.17e} {a.imag:+.17e} {b.real:+.17e} {b.imag:+.17e}\n")


def kmeans_small():
    wl = gi.workload("grid24_v8c32", name="smooth", smooth_sigma=1.0)
    s = gi.make_system(wl)
    init = gi.random_grid_points(40, wl.n_r, seed=23)
    spacing = tuple((n * wl.h) / n for n in wl.grid)
    pts, n_as = I.kmeans_points(I.kmeans_weights(s.phi, wl.n_occ), wl.grid, spacing, init, 30)
    with open(os.path.join(HERE, "kmeans_small.txt"), "w") as f:
        f.write("# weighted K-means points, grid24_v8c32 smooth variant (sigma = 1 bohr), "
                "40 starts random_grid_points(seed 23), max_iter 30\n")
        f.write(f"# assignment passes {n_as}\n")
        f.write(" ".join(str(int(p)) for p in pts) + "\n")


if __name__ == "__main__":
    single_pole()
    small_sigma()
    kmeans_small()
