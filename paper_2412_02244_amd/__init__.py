"""Exact, index-accelerated k-means for AMD MI355X (gfx950).

The computation lives in ``libekm.so`` (hand-written HIP kernels behind the C
ABI in ``include/ekm.h``); this package only marshals torch tensors to it.
"""

from ._binding import (  # noqa: F401
    EXPORTED,
    KM_BRUTE,
    KM_ERR_HIP,
    KM_ERR_INVALID,
    KM_ERR_NOT_EXACT,
    KM_ERR_OOM,
    KM_ERR_UNSUPPORTED,
    KM_F32,
    KM_F64,
    KM_FLAG_CELL_LEAVES,
    KM_FLAG_SMALL_LISTS,
    KM_FLAG_SSE,
    KM_FLAG_TIMING,
    KM_INDEXED,
    KM_OK,
    LIB_PATH,
    PHASES,
    Context,
    Distortion,
    EKMError,
    KmConfig,
    KmIterStats,
    distortion_bwd,
    distortion_bwd_noalloc,
    distortion_fwd,
    kmeans_destroy,
    kmeans_init,
    kmeans_init_batched,
    kmeans_last_error,
    kmeans_phase_times,
    kmeans_run,
    kmeans_run_batched,
    kmeans_step,
    kmeans_step_times,
    kmeans_workspace_bytes,
    load_library,
)
