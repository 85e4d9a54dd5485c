"""Seeded synthetic inputs for the Lanczos full-frequency GW self-energy path.

This module only *makes inputs*: random real orbitals on a periodic grid,
orbital energies, frequency grids, the lists of quasiparticle states and the
uneven Lanczos lengths of the batched workload.  It holds none of the method's
arithmetic (no Coulomb kernel, no pair matrix, no Lanczos, no continued
fraction), so that the CPU oracle and the GPU path can both draw from it
without sharing any computation.

Inputs stand in for the Kohn-Sham orbitals of hydrogen-passivated silicon
clusters that the paper obtains from a real-space DFT code (paper, paragraph
introducing the Casida equation and the PARSEC paragraph of the GW100
discussion).  Only sizes and ratios follow the paper's workloads (Table 1);
the orbitals are seeded Gaussian vectors made orthonormal by QR.

Recipe (all random numbers from numpy's PCG64 ``default_rng``):

* orbitals: stream ``[seed, 0]``, ``standard_normal((N_r, N_orb))`` in C
  order (row = grid point ``r = (ix*ny + iy)*nz + iz``, origin at the box
  corner), optionally low-pass filtered per column by
  ``exp(-|G|^2 sigma^2 / 2)`` (the "smooth" stress variant), then the thin
  QR factor with positive diag(R) (unique; computed by CholeskyQR2, which is
  exact to rounding for these well-conditioned Gaussian matrices), scaled by
  ``1/sqrt(dV)`` so that the grid integral of ``phi_k phi_l`` is
  ``delta_kl``.  The first ``n_occ`` columns are the occupied orbitals.
* energies: stream ``[seed, 1]``; occupied ``U[-12, -4]`` eV, then empty
  ``U[0, 12]`` eV, unsorted.
* uneven lengths and pair draws for the batched workload: stream
  ``[seed, 2]``.
* frequencies: ``linspace(w_lo, w_hi, n_omega)`` eV.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import Dict, List, Optional, Tuple

import numpy as np


@dataclass(frozen=True)
class Workload:
    """Sizes and parameters of one synthetic workload (all energies in eV)."""

    name: str
    seed: int
    grid: Tuple[int, int, int]
    box: float                 # cubic box edge, bohr
    n_occ: int                 # N_v
    n_emp: int                 # N_c
    n_qp_occ: int              # QP states taken from the top of the occupied set
    n_qp_emp: int              # ... and from the bottom of the empty set
    n_lanczos: int             # L (number of D-matvecs = number of diagonal entries)
    n_omega: int
    omega_range: Tuple[float, float] = (-20.0, 20.0)
    eta: float = 0.1           # broadening delta, eV
    poly_degree: int = 7       # g (Table 1 uses g = 7)
    smooth_sigma: float = 0.0  # > 0: low-pass filter width (bohr) before QR
    n_pairs: int = 0           # batched-pair workload: number of (m, n) vectors
    len_range: Tuple[int, int] = (0, 0)  # uneven Lanczos lengths U[lo, hi]

    @property
    def n_orb(self) -> int:
        return self.n_occ + self.n_emp

    @property
    def n_r(self) -> int:
        return int(np.prod(self.grid))

    @property
    def h(self) -> float:
        return self.box / self.grid[0]

    @property
    def dv(self) -> float:
        return self.h ** 3

    @property
    def n_vc(self) -> int:
        return self.n_occ * self.n_emp


# The workloads.  Names say what they are: grid points per edge and orbital
# counts.  Seeds are fixed per workload so every consumer sees the same data.
WORKLOADS: Dict[str, Workload] = {
    w.name: w
    for w in [
        # small case: 24^3 grid in a 12 bohr box, 8 + 32 orbitals, pair dim 256
        Workload("grid24_v8c32", 1000, (24, 24, 24), 12.0, 8, 32, 1, 1,
                 64, 200, eta=0.1),
        # headline case: 64^3 grid in a 24 bohr box, 128 + 512 orbitals,
        # pair dim 65,536, 8 QP states x 640 intermediate states
        Workload("grid64_v128c512", 1001, (64, 64, 64), 24.0, 128, 512, 4, 4,
                 200, 2000, eta=0.05),
        # batched uneven-length case on the same orbitals: 1,024 (m, n)
        # vectors with lengths drawn U[50, 300]
        Workload("grid64_v128c512_pairs1024", 1001, (64, 64, 64), 24.0, 128,
                 512, 4, 4, 300, 2000, eta=0.05, n_pairs=1024,
                 len_range=(50, 300)),
        # adjoint case: 48^3 grid (18 bohr box), 64 + 256 orbitals, pair dim 16,384
        Workload("grid48_v64c256", 1003, (48, 48, 48), 18.0, 64, 256, 1, 1,
                 120, 32, eta=0.05),
        # large dot-shaped case: 128^3 grid in a 48 bohr box, 512 + 1,024 orbitals
        Workload("grid128_v512c1024", 1004, (128, 128, 128), 48.0, 512, 1024,
                 8, 8, 300, 4000, eta=0.05),
        # scaled proxy of the headline case for oracle timing and parity:
        # 32^3 grid in a 12 bohr box, 32 + 128 orbitals, pair dim 4,096
        Workload("grid32_v32c128", 1005, (32, 32, 32), 12.0, 32, 128, 2, 2,
                 100, 400, eta=0.05),
    ]
}


def workload(base: str, **overrides) -> Workload:
    """Return a named workload, optionally with fields replaced."""
    w = WORKLOADS[base]
    return replace(w, **overrides) if overrides else w


@dataclass
class System:
    """One generated input: orbitals, energies and the quantities derived
    purely from the generator (grid spacing, QP-state list, frequencies)."""

    wl: Workload
    phi: np.ndarray            # [N_orb, N_r] float64, C order, grid-normalised
    energies_ev: np.ndarray    # [N_orb] float64, occupied first
    qp_states: np.ndarray      # [n_qp] int, orbital indices
    omega_ev: np.ndarray       # [n_omega] float64
    extras: dict = field(default_factory=dict)


def _lowpass(g: np.ndarray, grid, h: float, sigma: float) -> np.ndarray:
    """Multiply each column of ``g`` (grid-shaped) by exp(-|k|^2 sigma^2/2) in
    Fourier space.  Input shaping only; not part of the method."""
    nx, ny, nz = grid
    kx = 2 * np.pi * np.fft.fftfreq(nx, d=h)
    ky = 2 * np.pi * np.fft.fftfreq(ny, d=h)
    kz = 2 * np.pi * np.fft.fftfreq(nz, d=h)
    k2 = kx[:, None, None] ** 2 + ky[None, :, None] ** 2 + kz[None, None, :] ** 2
    filt = np.exp(-0.5 * k2 * sigma * sigma)
    out = np.empty_like(g)
    for j in range(g.shape[1]):
        f = np.fft.fftn(g[:, j].reshape(grid)) * filt
        out[:, j] = np.fft.ifftn(f).real.reshape(-1)
    return out


def make_orbitals(wl: Workload, dtype=np.float64, progress=None) -> np.ndarray:
    """Seeded orthonormal real orbitals, shape [N_orb, N_r] (float64, or
    rounded to dtype at the end).  progress(msg), if given, is called after
    each of the long steps."""
    say = progress or (lambda msg: None)
    rng = np.random.default_rng([wl.seed, 0])
    g = rng.standard_normal((wl.n_r, wl.n_orb))
    say("orbitals: random matrix drawn")
    if wl.smooth_sigma > 0:
        g = _lowpass(g, wl.grid, wl.h, wl.smooth_sigma)
    q = _thin_q(g)
    del g
    say("orbitals: orthonormalised")
    q /= np.sqrt(wl.dv)
    return q.T.astype(dtype, order="C")


def _thin_q(g: np.ndarray) -> np.ndarray:
    """Q of the thin QR factorisation g = Q R with diag(R) > 0, by two passes
    of Cholesky QR (g R^-1 with R = chol(g^T g)^T)."""
    q = g
    for _ in range(2):
        gram = q.T @ q
        r = np.linalg.cholesky(gram).T          # upper, positive diagonal
        rinv = np.linalg.inv(r)                 # small N_orb x N_orb
        q = q @ rinv
    return np.ascontiguousarray(q)


def make_energies(wl: Workload) -> np.ndarray:
    """Occupied energies U[-12,-4] eV then empty U[0,12] eV, unsorted."""
    rng = np.random.default_rng([wl.seed, 1])
    ev = rng.uniform(-12.0, -4.0, wl.n_occ)
    ec = rng.uniform(0.0, 12.0, wl.n_emp)
    return np.concatenate([ev, ec])


def frontier_states(energies_ev: np.ndarray, n_occ: int, k_occ: int,
                    k_emp: int) -> np.ndarray:
    """The k_occ highest occupied and k_emp lowest empty orbitals (indices)."""
    occ = np.argsort(energies_ev[:n_occ])[::-1][:k_occ]
    emp = n_occ + np.argsort(energies_ev[n_occ:])[:k_emp]
    return np.concatenate([occ, emp]).astype(np.int64)


def omega_grid(wl: Workload) -> np.ndarray:
    return np.linspace(wl.omega_range[0], wl.omega_range[1], wl.n_omega)


def pair_draw(wl: Workload, qp_states: np.ndarray):
    """For the batched workload: ``n_pairs`` (m, n) pairs drawn without
    replacement from qp_states x all orbitals, and uneven lengths."""
    rng = np.random.default_rng([wl.seed, 2])
    lo, hi = wl.len_range
    lengths = rng.integers(lo, hi + 1, wl.n_pairs)
    all_pairs = np.array([(m, n) for m in qp_states for n in range(wl.n_orb)],
                         dtype=np.int64)
    pick = rng.choice(len(all_pairs), size=wl.n_pairs, replace=False)
    pairs = all_pairs[pick]
    return pairs[:, 0].copy(), pairs[:, 1].copy(), lengths.astype(np.int64)


def make_system(name_or_wl, **overrides) -> System:
    """Generate the full input set of a workload."""
    if isinstance(name_or_wl, Workload):
        wl = replace(name_or_wl, **overrides) if overrides else name_or_wl
    else:
        wl = workload(name_or_wl, **overrides)
    phi = make_orbitals(wl)
    e = make_energies(wl)
    qp = frontier_states(e, wl.n_occ, wl.n_qp_occ, wl.n_qp_emp)
    sysm = System(wl=wl, phi=phi, energies_ev=e, qp_states=qp, omega_ev=omega_grid(wl))
    if wl.n_pairs > 0:
        m_idx, n_idx, lengths = pair_draw(wl, qp)
        sysm.extras.update(m_idx=m_idx, n_idx=n_idx, lengths=lengths)
    return sysm


def random_pair_vectors(n_vec: int, n_vc: int, seed: int) -> np.ndarray:
    """Seeded test vectors in pair space, [n_vec, n_vc] float64."""
    rng = np.random.default_rng([seed, 7])
    return rng.standard_normal((n_vec, n_vc))


def random_fields(n_fields: int, n_r: int, seed: int) -> np.ndarray:
    """Seeded real grid fields, [n_fields, n_r] float64."""
    rng = np.random.default_rng([seed, 8])
    return rng.standard_normal((n_fields, n_r))


def random_grid_points(n_points: int, n_r: int, seed: int) -> np.ndarray:
    """Seeded distinct grid-point indices in [0, n_r), sorted, int32 (test
    interpolation points)."""
    rng = np.random.default_rng([seed, 9])
    return np.sort(rng.choice(n_r, size=n_points, replace=False)).astype(np.int32)


__all__ = [
    "Workload", "WORKLOADS", "workload", "System", "make_system",
    "make_orbitals", "make_energies", "frontier_states", "omega_grid",
    "pair_draw", "random_pair_vectors", "random_fields", "random_grid_points",
]
