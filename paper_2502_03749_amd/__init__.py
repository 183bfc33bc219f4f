"""PINS (arXiv 2502.03749) inner-subproblem hot path for MI355X.

The solver is the HIP library ``libpins.so`` (C ABI in ``include/pins.h``);
this package is its thin Python binding.  See ``_binding`` for the calls.
"""
from ._binding import (COST_DENSE, COST_GRID, COST_POINTS, FP64, MIXED, MIXED_FAST, NOALLOC_SCRATCH_BYTES, SHIFT_IMPLICIT, SHIFT_MATERIALIZED,  # noqa
                       Context, Params, PinsError, Server, declared_functions, lib, params, probe_exp_rate, probe_texp,
                       workspace_bytes)
from ._binding import KERNEL_NAMES, LIB_PATH  # noqa
