"""srm3: 3rd-order Spectral Representation Method stochastic waves on MI355X.

The generator itself is the HIP library ``libsrm3.so`` (see ``include/srm3.h``);
this package only builds it and marshals arguments to it.
"""
from .srm3 import (SRM3_ALGO_DIRECT, SRM3_ALGO_FFT2D, SRM3_ALGO_KAPPA_FFT, SRM3_ALGO_MFMA, SRM3_BATCH_AUTOTUNE, SRM3_BATCH_GRAPH,  # noqa: F401
                   SRM3_FP32, SRM3_FP64,
                   Batch, Plan, Server, Srm3Error, load, plan_from_workload, process_plan_from_workload,
                   srm3_batch_create, srm3_process_plan, srm3_wind_factors, srm3_product_factors,
                   srm3_batch_destroy, srm3_batch_info, srm3_batch_run, srm3_coefficients,
                   srm3_destroy, srm3_generate, srm3_generate_noalloc, srm3_generate_uneven, srm3_last_error,
                   srm3_algorithm_terms, srm3_mfma_shape, srm3_plan_set_mfma_shape, srm3_pair_terms, srm3_plan, srm3_plan_set_algorithm,
                   srm3_rows_per_wave, srm3_profile_enable, srm3_profile_read,
                   srm3_set_spectrum, srm3_spectrum_kaimal_davenport, srm3_transform,
                   srm3_workspace_bytes, srm3_workspace_fill)
