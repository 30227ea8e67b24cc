"""MinMaxLTTB reference oracle -- TEST INFRASTRUCTURE ONLY.

Plain CPU statement of the method (plain C in ``mmlttb_oracle.c``, loaded
here through ctypes). Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package. The GPU library
does not import, link or call it.
"""
from .oracle import (  # noqa: F401
    OracleError,
    build,
    compile_variant,
    source_text,
    exact_sum_f32,
    exact_sum_i64,
    lib_path,
    lttb,
    lttb_means,
    m4,
    everynth,
    minmax,
    minmax_simplify,
    simplify_points,
    SIMPLIFIERS,
    minmax_typed,
    minmaxlttb_typed,
    exact_sum_f64,
    lttb_means_typed,
    minmax_xbins,
    minmaxlttb_xbins,
    minmaxlttb,
    minmaxlttb_segments,
    load_openmp,
    threads,
    XK_IMPLICIT,
    XK_INT64,
)
