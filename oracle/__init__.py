"""FP64 CPU oracle of the SPPC eigensolver -- TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously correct implementation of what the GPU path computes,
written from the paper (Alg. 2; Sec. IV eqs. EP_small, first_PC, exp_seq2,
bl_diag, sm_first, sm_lin_proj, blkGS, QR, Qp; eq. rrn) in float64 with NumPy /
SciPy (LAPACK).  Only the tests, the smoke check and the benchmark's CPU
baseline leg may import it.  It shares no code with the GPU library and the
GPU library never imports it.

Pins (tests/test_oracle_pins.py, tests/test_oracle_mpnn.py) tie every function to
closed forms, brute force or library routines, with one exception:

  * sppc_stagnated -- parity unpinned.  The paper leaves the detection of the
    stagnation point open (Sec. VII); the rule (sine of the smallest new angle
    below 1e-4, or the largest residual not halved over three steps) is a
    reading.  Its inputs are pinned (the angles against the principal angles of
    scipy, the residuals through the Rayleigh-Ritz bounds), the thresholds are not.
"""
from .core import (  # noqa: F401
    Options,
    Result,
    symmetric_from_upper,
    product_from_upper,
    product_rows_from_upper,
    small_space_matrix,
    zeroth_order,
    rs_corrections,
    sppc,
    sppc_pair,
    sppc_stagnated,
    final_check,
    jacobi_correction,
    small_space_correction,
    rayleigh_ritz,
)
