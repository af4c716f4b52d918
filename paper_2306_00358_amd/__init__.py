"""HOTRG coarse-graining on AMD MI355X (gfx950): Python binding of libhotrg.so.

The library (include/hotrg.h) runs the higher-order TRG step of
arXiv 2306.00358 (Sec. 2) on one GPU: environment contractions and the three
coarse contractions as MFMA GEMMs, the FP64 eigendecomposition of the
environment, and FP64 log-norm accumulation.  This package only marshals
arguments; see ``_lib`` for the calls.
"""

from ._lib import (  # noqa: F401
    EXPORTS, HOTRG_BF16X3, HOTRG_FP32, HOTRG_FP64, HOTRG_GXY, HOTRG_ISING, HOTRG_ISO_ONE_SIDED,
    HOTRG_ISO_TWO_SIDED, HOTRG_POTTS, HOTRG_RAW, HOTRG_TRUNC_MULTIPLET, HOTRG_TRUNC_PLAIN, HOTRG_XY,
    HOTRG_PREC_AUTO, LIB_PATH, Context, HotrgError, State, Ticket, hotrg_coarse,
    hotrg_coarse_noalloc, hotrg_environment, hotrg_footprint, hotrg_plan, hotrg_projector, hotrg_run,
    hotrg_run_batch, hotrg_run_grouped, hotrg_thermo, lib, make_opts, model_params,
)
from .flops import step_flops, run_flops, dims_schedule  # noqa: F401
