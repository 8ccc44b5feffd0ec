"""MI355X-native fast FCC cosine transform (Seifert, Hueper, Uhl, Sec. IV-B).

The transform runs in the HIP library ``libfccdct.so`` (built by
``paper_1807_10058_amd.build``); this package only marshals arguments to its
C ABI (``include/fcc_dct.h``).  There is no CPU fallback: importing the
binding raises if the library is missing.
"""
from .binding import (  # noqa: F401
    FCC_PREC_FP32, FCC_PREC_FP64, FCC_PREC_SPLIT_BF16, FCC_PREC_SPLIT_FP16,
    BatchedCall, FCC_LEVEL0_FP32, FCC_MAP_BALANCE, FCC_MAP_CLUSTER, FCC_MAP_F_INNER, FCC_MAP_NODES64, FCC_MAP_NODES8, FCC_MAP_ORBIT, FCC_MAP_SPLIT, FCC_MAP_XCD, FCC_MAP_XCD16, FCC_REAL_INPUT, FCC_STAGES_FP32, FCC_STAGES_FP64, FCC_TRANSPOSED, FCC_HERMITIAN_PACKED, FCC_FOLD_FFT, FCC_FOLD_BASE,
    FccError, fcc_asp_orbit_blocks, fcc_asp_tables, fcc_dct_autotune, fcc_dct_batched, fcc_dct_batched_release, fcc_dct_batched_time_launches, fcc_dct_describe_launches, fcc_dct_destroy, fcc_dct_forward, fcc_dct_packed_size,
    fcc_dct_forward_static, fcc_fold_unfold_tables,
    fcc_dct_get_tuning, fcc_dct_inverse, fcc_dct_plan, fcc_dct_plan_tuned, fcc_dct_roundtrip_residual,
    fcc_dct_time_launches, fcc_spectrum_quantise, fcc_status_string, lib_path,
)
