"""libmmlttb: MinMaxLTTB time-series downsampling on AMD MI355X (gfx950).

The compute path lives in ``libmmlttb.so`` (HIP kernels behind a C ABI, see
``include/libmmlttb.h``); this package binds it with ctypes (``ops``), builds
it (``build``), and holds the seeded synthetic inputs (``synth``). Importing
the package does not load the library; the first call does, and raises if the
library is not built.
"""
from .ops import (  # noqa: F401
    batched_workspace_size,
    everynth,
    lttb,
    m4,
    m4_workspace_size,
    minmaxlttb_batched,
    segment_table,
    lttb_workspace_size,
    minmax,
    minmax_simplify,
    simplify_workspace_size,
    minmax_typed,
    minmaxlttb_typed,
    typed_workspace_size,
    minmax_xbins,
    minmaxlttb_xbins,
    xbins_workspace_size,
    minmaxlttb,
    lttb_means,
    profile_enable,
    profile_read,
    profile_samples,
    profile_reset,
    workspace_size,
    set_tuning,
    set_graph_cache,
    graph_cache_stats,
    get_tuning,
)
