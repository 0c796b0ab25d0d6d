"""Batched exact squared Mallows distances on MI355X (gfx950).

The compute lives in ``libd2.so`` (HIP kernels behind the C ABI of
include/d2.h); this package only marshals torch tensors into that ABI.
"""
from ._ffi import (D2_COST_BF16_MFMA, D2_COST_F64_DIRECT, D2_INIT_AUTO, D2_INIT_NWC,  # noqa: F401
                   D2_INIT_VOGEL, D2_INIT_LCM, D2_FLAG_EAGER, D2_SCHED_AUTO, D2_SCHED_PLAIN, D2_PAIR_BAD_POINTS, D2_PAIR_BAD_WEIGHTS, D2_PAIR_OK,
                   D2_PAIR_PIVOT_CAP, D2_PAIR_TOO_LARGE, D2_PAIR_UNLABELLED, D2_PAIR_INTERNAL, D2Error,
                   LibraryMissing)
from .api import (DeviceSet, Handle, Opts, d2_assign, d2_assign_into, d2_cost_tiles,  # noqa: F401
                  d2_emd_batch, d2_emd_batch_basis, d2_pairwise, d2_tune_pairwise, d2_workspace_bytes,
                  d2_centroid_update, d2_centroid_update_free, free_basis_buffer, constrained_d2, d2_emd_cost_batch, d2_mm_distance,
                  d2_assign_multi, d2_assign_segmented, d2_merge_level)
from .hierarchy import hierarchical_d2  # noqa: F401,E402
