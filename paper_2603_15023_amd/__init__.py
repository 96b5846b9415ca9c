"""MI355X-native PAC stochastic aggregation (SIMD-PAC-DB's hot path on gfx950).

The work runs in libpac.so (hand-written HIP kernels behind the C ABI of
include/pac.h); this package only marshals arguments.  Importing it does not
load the library; the first call does, and raises ImportError if it has not
been built (``python -m paper_2603_15023_amd.build``).
"""
from ._abi import PacError  # noqa: F401
from .api import (  # noqa: F401
    AggSpec,
    Context,
    ReleaseRequest,
    cells_tensor,
    new_state,
    pac_filter,
    pac_finalize,
    pac_finalize_batch,
    pac_group_aggregate,
    pac_group_aggregate_batch,
    pac_hash_mask,
    pac_key_index,
    pac_lift,
    pac_noised,
    pac_select_cmp,
    pac_world_values,
    stream_copy,
    stream_read,
    tune_key,
)
