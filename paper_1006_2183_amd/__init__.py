"""MI355X-native local sparse product C = A (x) B over a semiring.

The computation runs in the HIP library built from ``csrc/`` (see
``include/sg_spgemm.h`` for the C ABI); this package only marshals
arguments. Importing it does not touch the GPU.
"""
from .binding import (  # noqa: F401
    DevMat,
    Plan,
    SgError,
    SEMIRINGS,
    FORMATS,
    default_tuning,
    make_tuning,
    load_library,
    spgemm,
    spgemm_grouped,
    spgemm_symbolic,
    spgemm_numeric,
    spgemm_batched,
    validate,
    build_aux,
    workspace_size,
    coo_to_sparse,
    convert,
    Mask,
    mask_set,
    chain_symbolic,
    autotune_native,
)
