"""MI355X-native t-FDP layout library.

The computation lives in ``libtfdp.so`` (hand-written HIP for gfx950, C ABI
in ``include/tfdp.h``); :mod:`paper_2303_03964_amd.tfdp` is a thin ctypes
binding with the same function names. There is no CPU fallback: every entry
point raises if the shared library is missing.
"""
from .tfdp import (  # noqa: F401
    Batch,
    Layout,
    TfdpError,
    TfdpParams,
    library_path,
    load_library,
    tfdp_batch_add,
    tfdp_batch_count,
    tfdp_batch_create,
    tfdp_batch_destroy,
    tfdp_batch_remove,
    tfdp_batch_set_graphs,
    tfdp_batch_get_tiles,
    tfdp_batch_set_tiles,
    tfdp_batch_step,
    tfdp_batch_workspace_size,
    tfdp_last_error,
    tfdp_layout_destroy,
    tfdp_layout_forces,
    tfdp_layout_get_iter,
    tfdp_layout_get_params,
    tfdp_layout_init,
    tfdp_layout_phase_times,
    tfdp_layout_set_iter,
    tfdp_layout_set_params,
    tfdp_layout_set_graphs,
    tfdp_layout_set_node_weights,
    tfdp_layout_set_overlap,
    tfdp_layout_set_profiling,
    tfdp_layout_step,
    tfdp_layout_sync_status,
    tfdp_params_default,
    tfdp_params_validate,
    tfdp_phase_count,
    tfdp_phase_name,
    tfdp_quality_sampled,
    tfdp_quality_sampled_noalloc,
    tfdp_stress_sampled,
    tfdp_stress_workspace_size,
    tfdp_workspace_size,
)
