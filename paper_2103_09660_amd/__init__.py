"""MI355X-native HyperNetVec refinement (arXiv 2103.09660).

The refinement hot path -- per-level projection of coarse embeddings and
smoothing sweeps over the star-expansion incidence, in FP32 or BF16 storage,
plus its reverse mode -- runs in hand-written HIP kernels for gfx950 behind
the C ABI of include/hnv.h.  This package is the thin Python binding.
"""
from .api import (  # noqa: F401
    DeviceLevel,
    Hierarchy,
    HostLevel,
    HostMap,
    Plan,
    ScorePlan,
    abi_version,
    cast,
    coarsen_features_workspace_bytes,
    coarsen_hierarchy_device,
    coarsen_hierarchy_features_device,
    coarsen_level,
    coarsen_level_device,
    coarsen_level_features_device,
    coarsen_workspace_bytes,
    last_error,
    plan_workspace_bytes,
    refine_hierarchy,
    refine_level,
    score_candidates,
    star_edgelist,
    validate_level,
)
from ._lib import HnvError  # noqa: F401
