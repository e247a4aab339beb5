"""MI355X library for the algebraic two-level overlapping Schwarz preconditioner
(Al Daas, Jolivet, Rees): HIP kernels behind a C interface (include/ads.h),
with a thin ctypes binding in `paper_2201_02250_amd.ads`."""
from .ads import (  # noqa: F401
    Context, ads_setup, ads_setup_batched, ads_apply, ads_solve, ads_get_info, ads_export_maps,
    ads_export_splitting, ads_export_coarse, ads_partition_bfs, ads_destroy, ads_status_string,
    ads_last_error, options, ksp_options, SYMBOLS, LIB_PATH,
    ADS_PREC_FP64, ADS_PREC_FP32, ADS_PREC_BF16, ADS_VARIANT_DEFLATED, ADS_VARIANT_RAS,
)
