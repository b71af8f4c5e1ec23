"""CPU FP64 oracle for the exchange operator and ACE compression.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, readable restatement
of what the HIP library computes, written from the paper (arXiv 2501.03061)
with NumPy/SciPy library primitives (FFT, GEMM, Cholesky, triangular solve)
as its only building blocks.  It shares no code with the HIP path and imports
nothing from it.  Only the test suite, the smoke check and the CPU-baseline
leg of the benchmark may import it; the library never routes through it.

Modules
  exchange  -- grid frequencies, screened kernel, Vx applied to orbitals
               (Eq. 13 and the mixed-state form Eq. 10), exchange energy.
  ace       -- ACE construction and application (Eq. 14), the
               exchange-only implicit-midpoint loop (Eq. 4, 6, 7), and the
               exchange-only PT-IM step with the projector and the occupation
               matrix (Eq. 4-7).
  sigma     -- occupation-matrix diagonalisation (Eq. 11), the rotated
               orbitals Phi Q, the density with a full sigma (Sec. III-C) or
               with occupations (Eq. 12), and the latter on the twice-finer
               charge-density grid (Sec. VI).

Every function states the passage it follows and, where the paper is silent
or garbled, the reading taken.  Parity pins live in tests/test_oracle_pins.py.
"""
from .exchange import (  # noqa: F401
    signed_freq, g2_grid, kernel_hse, exchange_apply, exchange_energy_real,
    exchange_energy_gspace, exchange_apply_sigma, pair_potential,
)
from .ace import ace_build, ace_apply, ptim_exchange_loop, ptim_step, DT_50AS, ALPHA  # noqa: F401
from .sigma import sigma_eig, rotate, density_sigma, density, density_fine  # noqa: F401
