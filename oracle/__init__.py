"""Plain FP64 CPU oracle for the Lanczos full-frequency GW correlation self-energy.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or call anything in this
package.  The product path (the HIP library and its Python binding) never
imports it and shares no code with it: no kernels, helpers, tables or constant
generators.  The only common module is ``gw_inputs``, which makes the seeded
inputs and holds none of the method's arithmetic.

What it computes, in the paper's notation (Gao, Tang, Zhao, Chelikowsky,
"Efficient Full-frequency GW Calculations using a Lanczos Method"):

* ``poisson``    -- the Hartree potential of a grid density with the periodic
  kernel 4 pi / |G|^2 (G = 0 dropped); the integral (kl|nm) of Eq. (3).
* ``casida``     -- Delta, the Hartree kernel K (Eqs. 2-3), the reduced
  symmetric matrix C = Delta^2 + 2 Delta^1/2 K Delta^1/2 (Eq. 4) and the
  coupling vectors (P_nm)_vc = (nm|vc) (e_c - e_v)^1/2.
* ``chebyshev``  -- the degree-g polynomial p_g(x) ~ sqrt(x) that replaces
  D = C^1/2 (paragraph after Eq. 12), by Chebyshev interpolation.
* ``sigma``      -- Sigma_c by the sum over poles (Eq. 7 with Eq. 8), by the
  per-n form (Eqs. 10-11), by the resolvent (Eq. 12) with dense solves, and
  by the method itself: Lanczos tridiagonalisation (Eq. 13) and the Haydock
  continued fraction (Eq. 14).

Every function is a direct, unblocked evaluation of its defining formula;
library primitives (FFT, matmul, eigh, solve) serve as single steps.

Units: orbitals are grid-normalised (sum_r phi_k phi_l dV = delta_kl, bohr^-3/2),
energies are converted from eV to hartree with E_h = 27.211386245988 eV
(CODATA 2018) and results are returned in eV.

Readings of points the paper leaves open (spin factor, Coulomb kernel,
polynomial fit, continued-fraction truncation, reorthogonalisation) are listed
in the module docstrings where they apply.  Parity pins for every function
are in ``tests/test_oracle_*.py``.
"""

from . import poisson, casida, chebyshev, sigma, adjoint  # noqa: F401
from .sigma import HARTREE_EV, Problem, default_interval  # noqa: F401
