"""Click correlators and cumulants of lossy Gaussian states on MI355X (gfx950).

The arithmetic runs in libgbs (hand-written HIP kernels behind the C ABI of
include/gbs.h); this package holds the ctypes binding with the same entry
point names, the torch.autograd.Function wrapper, and the differentiable
covariance model used to fit per-mode transmissions and squeezings.
"""
from ._binding import (  # noqa: F401
    EXPORTS, GBS_ALL_MINORS, GBS_ASYNC, GBS_CLICK, GBS_E_DEVICE, GBS_E_INVALID_ARG, GBS_E_NOT_SPD,
    GBS_E_OUT_OF_MEMORY, GBS_E_UNSUPPORTED, GBS_FP64, GBS_MAX_MODES, GBS_MAX_ORDER, GBS_MIXED,
    GBS_OK, GBS_PARITY, GBS_TIMING, GBSError, STAGE_NAMES, gbs_last_timings, LIB_PATH, gbs_autotune_batched, gbs_colex_rank,
    gbs_colex_unrank, gbs_correlators, gbs_cumulant_grad, gbs_cumulants, gbs_cumulants_batched,
    gbs_cumulants_displaced, gbs_sample, GBS_STAGE_SAMPLE, gbs_sample_cumulants, gbs_pearson,
    GBS_STAGE_ESTIMATE, gbs_cumulants_shard, gbs_cumulants_noalloc, GBS_E_SCRATCH_LIMIT,
    GBS_NOALLOC_SCRATCH_BYTES,
    gbs_last_error, gbs_num_subsets, gbs_order_offset, gbs_set_tuning, gbs_status_string,
    gbs_total_outputs, lib,
)

__all__ = [n for n in dir() if n.startswith("gbs_") or n.startswith("GBS")] + ["lib", "EXPORTS", "STAGE_NAMES"]
from .autograd import (GBSCumulants, cumulant_matching_loss, cumulants,  # noqa: E402,F401
                       interferometer_symplectic, lossy_squeezed_covariance)
