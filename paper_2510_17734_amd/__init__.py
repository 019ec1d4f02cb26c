"""MI355X-native ALS completion in the tensorized butterfly format.

The compute path is libbfc.so (HIP kernels for gfx950 behind a C ABI, see
include/bfc.h); this package is its Python binding.  Importing the package
does not load the library; the first call does, and fails loudly if it has
not been built.
"""
from .api import (  # noqa: F401
    Batch,
    BfcError,
    batch_create,
    batch_residuals,
    batch_sweep,
    Config,
    core_stats,
    profile_enable,
    profile_read,
    Problem,
    destroy,
    env_nodes,
    flatten_cores,
    get_cores,
    init_cores,
    last_error,
    num_params,
    predict_entries,
    relative_error,
    residual,
    residual_observed,
    set_cores,
    solve_counters,
    sweep,
    sweep_core,
    sync_status,
    unflatten_cores,
    use_graphs,
    set_item_size,
    autotune_item_size,
    lowrank_to_butterfly,
    adam_sweep,
    adam_reset,
    adf_sweep,
)
