"""MI355X-native FX-correlator hot path (F-engine FFT + MFMA X-engine).

The compute lives in libcorr.so (HIP for gfx950, C ABI in include/corr.h);
this package is its ctypes binding.  Build with ``build.build()``.
"""
from .corr import (  # noqa: F401
    ABI_FUNCTIONS, CORR_BASELINE_MAJOR, CORR_CHAN_MAJOR, CORR_E_HIP, CORR_E_INVALID_ARG,
    CORR_E_NOMEM, CORR_E_OVERFLOW, CORR_E_STATE, CORR_E_UNSUPPORTED, CORR_FP16, CORR_FP32,
    CORR_FP8_E4M3, CORR_FULL, CORR_INT8, CORR_INT8_MAX_INTEGRATE, CORR_OK, CORR_TRI_LOWER,
    CORR_TRI_UPPER, LIB_PATH, ORDERS, LAYOUTS, PRECISIONS, SPECTRA_DTYPE, Batch, CorrError, Correlator,
    corr_copy_spectra, corr_create, corr_destroy, corr_dump_visibilities, corr_fengine,
    corr_get_counts, corr_last_error, corr_n_products, corr_params, corr_spectra_bytes,
    corr_status_string, corr_visibility_bytes, corr_xengine, lib, make_params, corr_set_tile,
    corr_autotune, corr_create_batched, corr_batch_get, corr_xengine_batched, corr_destroy_batched,
    corr_xengine_rect, corr_fengine_real8, corr_xengine_dump, corr_xengine_noalloc, corr_fx,
    corr_set_spectra_layout, corr_autotune_fx, corr_tuning,
)
