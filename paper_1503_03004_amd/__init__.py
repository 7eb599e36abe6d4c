"""MI355X-native sparse fixed-rank decomposition M = L + S (rank(L) = r).

FR-ADM (Alg. 1) with the FixedRankOptStep L-step (Alg. 2) and the Nystrom
variant FR-Nys (Alg. 3) of Ros et al., "Fast and Robust Fixed-Rank Matrix
Recovery", and FixedRankOptFull (Alg. 4) as a rank-r truncated SVD, as
hand-written HIP kernels for gfx950 behind the C ABI of include/sfr.h.  This package is only the Python binding of that library.
"""
from ._binding import (  # noqa: F401
    BatchSolver, Info, SFRError, Solver, lib, solve, solve_noalloc, solve_nys, status_string, tsvd,
    SFR_OK, SFR_ERR_ARG, SFR_ERR_NOMEM, SFR_ERR_DEVICE, SFR_ERR_RANK, SFR_ERR_NONFINITE,
    SFR_ERR_HANDLE, SFR_ERR_SCRATCH, SFR_ERR_BUSY, SFR_WARN_MAXITER, SFR_WARN_NOT_SPD, LIB_PATH,
)
