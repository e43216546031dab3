"""MI355X (gfx950) implementation of the level-2 RLT dual-ascent lower bound
for the Quadratic Assignment Problem (arXiv 1510.02065).

The compute path is the HIP library libqap_rlt2.so (C ABI in
include/qap_rlt2.h); this package is its thin Python binding.
"""
from ._binding import (MAX_N, QAP_FP32_CERTIFIED, QAP_FP32_NEAREST, QAP_FP64, QapError, Rlt2,  # noqa: F401
                       bnb_solve, lap_solve, lap_solve_device, lib, LIB_PATH, local_search, objective,
                       subproblem)
