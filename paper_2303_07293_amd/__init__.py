"""Shift-and-stack search for moving sources ("synthetic tracking",
arXiv:2303.07293) on AMD MI355X: HIP kernels for gfx950 behind a small C ABI
(include/sst.h), bound here with ctypes.

    from paper_2303_07293_amd import sst_detect, sst_stack, candidates_to_numpy
"""

from .binding import (  # noqa: F401
    CANDIDATE_DTYPE,
    EXPORTS,
    SST_BF16,
    SST_F16,
    SST_F32,
    SST_MEAN,
    SST_OP_DETECT,
    SST_OP_QUANT,
    SST_OP_REFINE,
    SST_OP_STACK,
    SST_OP_STATS,
    SST_SUM,
    SstError,
    SstBatch,
    SstPlan,
    candidates_to_numpy,
    load,
    sst_bin2x2,
    sst_coadd,
    sst_detect,
    sst_detect_noalloc,
    sst_frame_stats,
    sst_last_error,
    sst_median_subtract,
    sst_noalloc_scratch_bytes,
    sst_plan_detect,
    sst_profile_begin,
    sst_profile_end,
    sst_quantize,
    sst_refine,
    sst_set_half_search,
    sst_set_slot_keep,
    sst_set_stack_shape,
    sst_set_two_pass,
    sst_shapes,
    sst_shift_table,
    sst_stack,
    sst_workspace_bytes,
)
from .autograd import StackedSNR, stacked_snr  # noqa: F401,E402
from .tune import tune_plan, tuned_shape, tuning_times  # noqa: F401,E402
