"""The C-ABI library loads and exports every declared symbol (CPU only; no
compute call: only host-side argument checks and size queries, which return
before any HIP call)."""
from __future__ import annotations

import ctypes
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "libmmlttb.h")
LIB = os.path.join(ROOT, "paper_2305_00332_amd", "libmmlttb.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(mmlttb_[a-z_0-9]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2305_00332_amd import build

        build.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_four_calls():
    names = declared_functions()
    for f in ("mmlttb_minmax", "mmlttb_lttb", "mmlttb_minmaxlttb", "mmlttb_minmaxlttb_batched"):
        assert f in names


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 10
    for f in names:
        assert hasattr(lib, f), f"{f} declared in libmmlttb.h but not exported"
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (mmlttb_[a-z_0-9]+)$", out, flags=re.M))
    assert set(names) <= exported


def test_binding_lists_every_declared_symbol():
    from paper_2305_00332_amd import _lib

    assert set(declared_functions()) == set(_lib.EXPORTS)


def test_library_was_built_for_gfx950():
    data = open(LIB, "rb").read()
    assert b"amdgcn-amd-amdhsa--gfx950" in data


def _setup(lib):
    lib.mmlttb_workspace_size.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int32]
    lib.mmlttb_workspace_size.restype = ctypes.c_size_t
    lib.mmlttb_lttb_workspace_size.argtypes = [ctypes.c_int64, ctypes.c_int64]
    lib.mmlttb_lttb_workspace_size.restype = ctypes.c_size_t
    lib.mmlttb_last_error.restype = ctypes.c_char_p
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    lib.mmlttb_minmaxlttb.argtypes = [ctypes.c_int, vp, vp, i64, i64, i32, vp, vp, ctypes.c_size_t, vp]
    lib.mmlttb_lttb.argtypes = [ctypes.c_int, vp, vp, i64, i64, vp, vp, ctypes.c_size_t, vp]
    lib.mmlttb_minmax.argtypes = [ctypes.c_int, vp, vp, i64, i64, i32, vp, vp, vp, ctypes.c_size_t, vp]


def test_workspace_size_does_not_depend_on_n(lib):
    """Table 1: MinMaxLTTB keeps O(n_out) memory; the workspace never grows with n."""
    _setup(lib)
    for n_out, r_ps in [(1000, 4), (2000, 8), (4000, 4), (3, 2), (100, 3)]:
        sizes = {lib.mmlttb_workspace_size(n, n_out, r_ps) for n in (10, 10 ** 6, 10 ** 9, 10 ** 12)}
        assert len(sizes) == 1
        s = sizes.pop()
        assert 0 < s < 64 * n_out * r_ps + 128 * n_out + 8192
        lt = {lib.mmlttb_lttb_workspace_size(n, n_out) for n in (10, 10 ** 6, 10 ** 9)}
        assert len(lt) == 1


def test_invalid_arguments_rejected_on_host(lib):
    _setup(lib)
    fake = ctypes.c_void_p(0x100000)  # never dereferenced: checks run first
    ws = ctypes.c_void_p(0x200000)
    cases = [
        (0, None, fake, 0, 10, 4),        # n < 1
        (0, None, fake, 100, 2, 4),       # n_out < 3
        (0, None, fake, 100, 10, 1),      # r_ps < 2
        (0, fake, fake, 100, 10, 4),      # x given with implicit x
        (1, None, fake, 100, 10, 4),      # x missing with int64 x
        (2, None, fake, 100, 10, 4),      # bad x kind
        (0, None, None, 100, 10, 4),      # y NULL
        (0, None, ctypes.c_void_p(0x100002), 100, 10, 4),  # misaligned y
        (0, None, fake, 100, 2 ** 31, 4),  # n_out too large
        (0, None, fake, 100, 2 ** 30, 4),  # too many bins
    ]
    for xk, x, y, n, n_out, r_ps in cases:
        rc = lib.mmlttb_minmaxlttb(xk, x, y, n, n_out, r_ps, fake, ws, 1 << 30, None)
        assert rc == -1, (xk, n, n_out, r_ps)
        assert len(lib.mmlttb_last_error()) > 0
    # workspace too small
    rc = lib.mmlttb_minmaxlttb(0, None, fake, 10 ** 6, 1000, 4, fake, ws, 16, None)
    assert rc == -2
    assert b"workspace" in lib.mmlttb_last_error()
    rc = lib.mmlttb_lttb(0, None, fake, 10 ** 6, 1000, fake, ws, 16, None)
    assert rc == -2
    rc = lib.mmlttb_minmax(0, None, fake, 10 ** 6, 1000, 4, fake, None, ws, 1 << 30, None)
    assert rc == -1


def test_oracle_shares_no_code_with_gpu_path():
    """The oracle and the GPU library are independent: no source of one names the other."""
    import glob

    gpu_src = glob.glob(os.path.join(ROOT, "paper_2305_00332_amd", "**", "*.*"), recursive=True)
    for f in gpu_src:
        if f.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
            text = open(f).read()
            assert "oracle" not in text.lower() or f.endswith("synth.py"), f
    for f in glob.glob(os.path.join(ROOT, "oracle", "*")):
        if f.endswith((".py", ".c", ".h")):
            text = open(f).read()
            assert "paper_2305_00332_amd" not in text and "libmmlttb" not in text, f


def test_tuning_round_trips_including_automatic_chain(lib):
    i32p, i64p = ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int64)
    lib.mmlttb_set_tuning.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                      ctypes.c_int64]
    lib.mmlttb_get_tuning.argtypes = [i32p, i64p, i32p, i32p, i32p, i64p]

    def get():
        u, c, ch, t, bu, bc = (ctypes.c_int(), ctypes.c_int64(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int(),
                               ctypes.c_int64())
        assert lib.mmlttb_get_tuning(*(ctypes.byref(v) for v in (u, c, ch, t, bu, bc))) == 0
        return u.value, c.value, ch.value, t.value, bu.value, bc.value

    saved = get()
    assert saved[2] in (1, 2, 3) and saved[0] in (1, 2, 4, 8) and saved[3] in (2048, 4096, 8192)
    assert saved[4] in (1, 2, 4, 8) and saved[5] >= 256
    try:
        assert lib.mmlttb_set_tuning(8, 2048, 1, 8192, 2, 1000) == 0
        assert get() == (8, 2048, 1, 8192, 2, 1024)  # chunks rounded up to 256 * unroll
        assert lib.mmlttb_set_tuning(0, 0, 3, 0, 0, 0) == 0  # automatic again, the rest kept
        assert get() == (8, 2048, 3, 8192, 2, 1024)
        assert lib.mmlttb_set_tuning(0, 0, 4, 0, 0, 0) == -1
        assert lib.mmlttb_set_tuning(3, 0, 0, 0, 0, 0) == -1
        assert lib.mmlttb_set_tuning(0, 0, 0, 0, 5, 0) == -1
        assert lib.mmlttb_set_tuning(0, 0, 0, 0, 0, 100) == -1
    finally:
        assert lib.mmlttb_set_tuning(*saved) == 0
    assert get() == saved


def test_compiled_tuning_defaults_are_the_measured_best(lib):
    """Without MMLTTB_* overrides the library starts from the settings the
    committed tuning cache holds as best for MI355X (single-series stream and
    batched stream), so callers that never apply the cache run them too."""
    import json

    if any(k.startswith("MMLTTB_") and k != "MMLTTB_TUNE" for k in os.environ):
        pytest.skip("MMLTTB_* overrides are set")
    out = subprocess.run(
        [sys.executable, "-c",
         "import ctypes,sys; l=ctypes.CDLL(sys.argv[1]); P=ctypes.POINTER;"
         "l.mmlttb_get_tuning.argtypes=[P(ctypes.c_int),P(ctypes.c_int64),P(ctypes.c_int),P(ctypes.c_int),"
         "P(ctypes.c_int),P(ctypes.c_int64)];"
         "v=[ctypes.c_int(),ctypes.c_int64(),ctypes.c_int(),ctypes.c_int(),ctypes.c_int(),ctypes.c_int64()];"
         "assert l.mmlttb_get_tuning(*[ctypes.byref(a) for a in v])==0; print(*[a.value for a in v])", LIB],
        capture_output=True, text=True, check=True).stdout.split()
    unroll, chunk, chain, tile, bunroll, bchunk = map(int, out)
    cache = json.load(open(os.path.join(ROOT, "paper_2305_00332_amd", "tune_cache.json")))
    mi355x = [v for k, v in cache.items() if k.startswith("gfx950")]
    assert mi355x
    for entry in mi355x:
        assert (entry["single"]["best"]["unroll"], entry["single"]["best"]["chunk"]) == (unroll, chunk)
        b = entry["batched"]["best"]
        assert (b["unroll"], b["chunk"], b["tile"]) == (bunroll, bchunk, tile)
    assert chain == 3


def test_new_calls_reject_invalid_arguments_on_host(lib):
    _setup(lib)
    fake = ctypes.c_void_p(0x100000)
    ws = ctypes.c_void_p(0x200000)
    i64 = ctypes.c_int64
    lib.mmlttb_m4.argtypes = [ctypes.c_void_p, i64, i64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                              ctypes.c_size_t, ctypes.c_void_p]
    lib.mmlttb_everynth.argtypes = [i64, i64, ctypes.c_void_p, ctypes.c_void_p]
    xb = [ctypes.c_void_p, ctypes.c_void_p, i64, i64, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
          ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
    lib.mmlttb_minmax_xbins.argtypes = xb
    lib.mmlttb_minmaxlttb_xbins.argtypes = xb
    assert lib.mmlttb_m4(fake, 100, 3, fake, fake, ws, 1 << 20, None) == -1      # n_out < 4
    assert lib.mmlttb_m4(fake, 0, 10, fake, fake, ws, 1 << 20, None) == -1       # n < 1
    assert lib.mmlttb_m4(fake, 10 ** 6, 1000, fake, fake, ws, 16, None) == -2    # workspace
    assert lib.mmlttb_everynth(0, 10, fake, None) == -1
    assert lib.mmlttb_everynth(10, 0, fake, None) == -1
    assert lib.mmlttb_minmax_xbins(None, fake, 100, 10, 4, fake, fake, ws, 1 << 20, None) == -1   # x NULL
    assert lib.mmlttb_minmax_xbins(fake, fake, 2 ** 32 + 2, 10, 4, fake, fake, ws, 1 << 20, None) == -1
    assert lib.mmlttb_minmax_xbins(fake, fake, 100, 10, 0, fake, fake, ws, 1 << 20, None) == -1
    assert lib.mmlttb_minmaxlttb_xbins(fake, fake, 100, 10, 1, fake, fake, ws, 1 << 20, None) == -1
    assert lib.mmlttb_minmaxlttb_xbins(fake, fake, 10 ** 6, 1000, 4, fake, fake, ws, 16, None) == -2


def test_noalloc_rejects_sizes_beyond_its_array_on_host(lib):
    """The fixed-scratch call refuses a workspace larger than its array (and
    invalid n_out / r_ps) before any HIP call."""
    _setup(lib)
    i64 = ctypes.c_int64
    lib.mmlttb_minmaxlttb_noalloc.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, i64, i64,
                                              ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]
    fake = ctypes.c_void_p(0x100000)
    limit = 4 << 20
    assert "(4u << 20)" in open(HEADER).read()
    assert lib.mmlttb_workspace_size(10 ** 8, 65536, 4) > limit >= lib.mmlttb_workspace_size(10 ** 8, 16384, 4)
    assert lib.mmlttb_minmaxlttb_noalloc(0, None, fake, 10 ** 8, 65536, 4, fake, None) == -1
    assert b"fixed scratch" in lib.mmlttb_last_error()
    assert lib.mmlttb_minmaxlttb_noalloc(0, None, fake, 10 ** 8, 2, 4, fake, None) == -1   # n_out < 3
    assert lib.mmlttb_minmaxlttb_noalloc(0, None, fake, 10 ** 8, 100, 0, fake, None) == -1  # r_ps < 1


def test_profile_samples_host_checks(lib):
    """Per-launch samples: argument checks, and nothing recorded for calls the
    host rejects (no HIP call is made on this path)."""
    _setup(lib)
    i64 = ctypes.c_int64
    lib.mmlttb_profile_samples.argtypes = [ctypes.c_char_p, ctypes.POINTER(ctypes.c_float), i64, ctypes.POINTER(i64)]
    lib.mmlttb_profile_enable.argtypes = [ctypes.c_int]
    cnt = i64(-1)
    buf = (ctypes.c_float * 4)()
    assert lib.mmlttb_profile_samples(None, buf, 4, ctypes.byref(cnt)) == -1
    assert lib.mmlttb_profile_samples(b"call_minmaxlttb", buf, 4, None) == -1
    assert lib.mmlttb_profile_samples(b"call_minmaxlttb", buf, -1, ctypes.byref(cnt)) == -1
    assert lib.mmlttb_profile_samples(b"call_minmaxlttb", None, 4, ctypes.byref(cnt)) == -1
    assert lib.mmlttb_profile_reset() == 0
    assert lib.mmlttb_profile_enable(1) == 0
    try:
        fake = ctypes.c_void_p(0x100000)
        assert lib.mmlttb_minmaxlttb(0, None, fake, 10 ** 6, 1000, 1, fake, fake, 1 << 20, None) == -1  # r_ps
        assert lib.mmlttb_minmaxlttb(0, None, fake, 10 ** 6, 1000, 4, fake, fake, 16, None) == -2       # ws
        assert lib.mmlttb_profile_samples(b"call_minmaxlttb", None, 0, ctypes.byref(cnt)) == 0
        assert cnt.value == 0
        assert lib.mmlttb_profile_samples(b"no_such_kernel", buf, 4, ctypes.byref(cnt)) == 0
        assert cnt.value == 0
    finally:
        assert lib.mmlttb_profile_enable(0) == 0


def test_lttb_means_host_checks(lib):
    """The means call validates on the host before any launch."""
    _setup(lib)
    vp, i64 = ctypes.c_void_p, ctypes.c_int64
    lib.mmlttb_lttb_means.argtypes = [ctypes.c_int, vp, vp, i64, i64, vp, vp, vp]
    fake, mx, my = ctypes.c_void_p(0x100000), ctypes.c_void_p(0x200000), ctypes.c_void_p(0x300000)
    assert lib.mmlttb_lttb_means(0, None, fake, 100, 100, mx, my, None) == -1      # m <= n_out
    assert lib.mmlttb_lttb_means(0, None, fake, 100, 2, mx, my, None) == -1        # n_out < 3
    assert lib.mmlttb_lttb_means(0, None, fake, 1000, 100, None, my, None) == -1   # MX NULL
    assert lib.mmlttb_lttb_means(0, None, fake, 1000, 100, mx, ctypes.c_void_p(0x300004), None) == -1
    assert lib.mmlttb_lttb_means(1, None, fake, 1000, 100, mx, my, None) == -1     # int64 x missing
    assert lib.mmlttb_lttb_means(0, fake, fake, 1000, 100, mx, my, None) == -1     # x with implicit
