"""Exact Density Peaks Clustering on AMD Instinct MI355X (gfx950).

The computation runs in libdpc, hand-written HIP behind the C interface of
include/libdpc.h; this package is its thin Python binding.  See
``_binding`` for the calls: ``density``, ``dependent``, ``cluster`` and
``run`` take and return device tensors.
"""
from ._binding import (  # noqa: F401
    BACKENDS,
    Batch,
    BatchPlan,
    DPCError,
    Instance,
    EXPORTED,
    INF,
    LEAF_SIZES,
    LIB_PATH,
    Plan,
    SKIP_NOISE_DEPENDENTS,
    STAGES,
    Server,
    WORK_FIELDS,
    autotune,
    autotune_dependent,
    batch_run,
    cluster,
    cluster_sweep,
    density,
    density_sweep,
    dependent_backend,
    dependent,
    last_stats,
    leaf_size,
    load,
    run,
    run_noalloc,
    NOALLOC_SCRATCH_BYTES,
    ERR_SCRATCH,
    set_dependent_backend,
    set_leaf_size,
    square_threshold,
    status_str,
    workspace_bytes,
)
