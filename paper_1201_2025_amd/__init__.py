"""paper_1201_2025_amd: DWT-reduced local hyperspectral anomaly detection on MI355X.

A thin ctypes binding over ``libhsad.so`` (C ABI in ``include/hsad.h``).  The functions
carry the C names and only marshal arguments: device pointers of torch tensors and the
current HIP stream.  Every computation runs in the library's HIP kernels.  When the
library is not built, every call raises; there is no CPU fallback.

Method: Zare Baghbidi et al., "Improvement of anomaly detection algorithms in
hyperspectral images using discrete wavelet transform", SIPIJ 2(4), 2011.
"""
from __future__ import annotations

from ._binding import (  # noqa: F401
    HSAD_EHIP, HSAD_EINVAL, HSAD_ENOMEM, HSAD_EUNSUPPORTED, HSAD_OK, HSAD_OP_DWEST,
    HSAD_OP_DWRX, HSAD_OP_LRX, HSAD_OP_LRX_DWRX, HSAD_PREC_AUTO, HSAD_PREC_FP32,
    HSAD_PREC_FP64, HSAD_PREC_GRAM_BF16, HSAD_PREC_GRAM_FP16, HsadError, WindowParams,
    hsad_detect, hsad_detect_workspace_bytes, hsad_detect_noalloc, NOALLOC_SCRATCH_BYTES, hsad_global_rx, hsad_global_rx_workspace_bytes,
    hsad_wavelet_filter, hsad_dwt_full_len, hsad_dwt_full, hsad_idwt_full, hsad_dwest, hsad_dwrx, hsad_dwt, hsad_dwt_timed, hsad_dwt_detect_fused, hsad_detect_stream_step, hsad_dwt_out_len, hsad_last_error, hsad_levels_for,
    hsad_lrx, hsad_lrx_dwrx, hsad_version, hsad_workspace_bytes, lib, lib_path,
    hsad_threshold, hsad_threshold_workspace_bytes, hsad_auc, hsad_auc_workspace_bytes,
    auc_from_counts, BatchPlan, BatchOptions, Scene, batch_default_options,
    hsad_batch_autotune, hsad_lrx_dwrx_at, hsad_mlp_dims, hsad_surrogate_features,
    hsad_mlp_norm_stats, hsad_mlp_pack, hsad_surrogate_targets, hsad_mlp_sync, hsad_mlp_infer,
    hsad_mlp_train_workspace_bytes, hsad_mlp_gradient, hsad_mlp_train_step, hsad_error_stats,
    hsad_surrogate_select, hsad_surrogate_workspace_bytes, hsad_surrogate_run, MlpModel,
    SurrogateOptions, SurrogateReport,
)
from .surrogate import Surrogate  # noqa: F401
