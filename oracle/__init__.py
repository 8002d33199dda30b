"""CPU reference oracle for the multibody MFS scattering method (FP64).

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
NumPy/SciPy implementation written from the paper (Cai, Bagge, Martinsson,
"A stable and fast method for solving multibody scattering problems via the
method of fundamental solutions").  Only the test suite, the smoke check and
the benchmark's CPU-baseline leg may import it; the library path never calls
it and it imports nothing from the library.

Modules
-------
fundamental     phi_kappa, eq. (FundamentalSol)
local_s         per-body matrices A, B, D, B_hat, truncated pseudo-inverses and
                the scattering matrix S (Sec. 4, eq. scattering-matrix)
global_system   packing of equivalent points, the off-body matrix G_hat
                (eq. Gmtx-entries), the operator I + S G_hat (eq. mbody2),
                right-hand side, dense and GMRES solves, field evaluation
reconstruct     full MFS sources of each body from the solved equivalent
                sources and the field near the bodies (Sec. 4.6)

Parity status: every function is pinned by a test in ``tests/test_oracle_*``
against a closed form, a series solution, a textbook routine or brute force,
except where a docstring says "parity unpinned".
"""

from . import fundamental, local_s, global_system, reconstruct  # noqa: F401
