"""FP64 CPU oracle of the time-domain GRFT and the dual-scale GRFT (DS-GRFT).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, links or runs
this package; only the test-suite, the smoke check and the CPU-baseline leg of
the benchmark do.  It shares no code, tables or helpers with the HIP path:
every quantity here is recomputed from the paper's definitions in float64 and
exact integer arithmetic.

Paper: Li et al., "Efficient dual-scale generalized Radon-Fourier transform
detector family for long time coherent integration" (arXiv 2403.06788).

Modules
  grid      derived radar quantities, the integer search lattice, the exact
            trajectory numerator, range offsets and phasors (Sec. II-B,
            Sec. III-C, Sec. IV-B).
  transforms TD-GRFT (Sec. III-A-1, eq. (13)) and DS-GRFT as mGIFT followed
            by GFT (Sec. IV-A/IV-C, eqs. (44), (46), (47), (64); Alg. 1-3).
  detect    reduced maps, argmax, LRT threshold and peak parameters
            (Sec. III-C eqs. (31), (33); eq. (72); Alg. 3).
  adjoint   continuous objective |DS-GRFT|^2 over (r0, v, a) and its
            analytic gradients (not in the paper; reading documented in the
            design notes).
  brute     multi-precision direct evaluation from physical parameters
            (independent of the integer numerator formula) for tiny inputs.
  lowp      float64 model of the 8-bit float (OCP E4M3) form of the fine
            search: operand rounding, power-of-two scales, split products.
  fd        frequency-domain mGIFT (Alg. 1): range spectrum, coarse RM phase
            ramp, IFFT, pre-DFM phase; DS-GRFT on top of it.
  ktmfp     dual-scale KT-MFP (Alg. 4, P = 2): keystone transform by sinc
            interpolation over slow time, folding-factor coarse cells, GFT
            over the baseband velocities and fine accelerations.

Parity status: every function here is pinned by a CPU test (brute force,
closed forms, invariants, or a library routine); see tests/test_oracle_*.py.
"""
from .grid import Radar, Axis, Grid, make_grid  # noqa: F401
