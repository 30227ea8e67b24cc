"""The tuning cache and the MMLTTB_TUNE policy the binding applies when it
loads the library (selection logic on the CPU; the applied values on the GPU)."""
from __future__ import annotations

import json
import os
import subprocess
import sys

import pytest

from paper_2305_00332_amd import autotune

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_select_maps_each_class_to_its_own_settings():
    cache = {"dev": {"single": {"best": {"unroll": 4, "chunk": 1 << 20}},
                     "batched": {"best": {"unroll": 2, "chunk": 65536, "tile": 8192}}}}
    assert autotune.select(cache, "dev", "single") == {"unroll": 4, "chunk": 1 << 20}
    assert autotune.select(cache, "dev", "batched") == {"batch_unroll": 2, "batch_chunk": 65536, "tile": 8192}
    assert autotune.select(cache, "other", "single") is None
    assert autotune.select(cache, "dev", "typed_f64") is None


def test_committed_cache_has_both_load_classes_for_mi355x():
    cache = autotune.load_cache()
    keys = [k for k in cache if k.startswith("gfx950")]
    assert keys
    for k in keys:
        for kind in autotune.LOAD_CLASSES:
            args = autotune.select(cache, k, kind)
            assert args and all(v > 0 for v in args.values())


def test_invalid_policy_is_refused():
    code = ("import os; os.environ['MMLTTB_TUNE']='sometimes';"
            "from paper_2305_00332_amd import autotune\n"
            "try:\n autotune.on_load()\nexcept ValueError as e:\n print('refused', e)")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, check=True).stdout
    assert out.startswith("refused")


@pytest.mark.gpu
def test_loaded_library_runs_the_cached_tuning():
    """A fresh process that only loads the library (MMLTTB_TUNE unset, no
    autotune call) runs the cached best settings of this device."""
    code = ("import json, torch; from paper_2305_00332_amd import _lib, ops, autotune; _lib.load();"
            "print(json.dumps({'key': autotune.device_key(), 'tuning': ops.get_tuning()._asdict(),"
            "'source': _lib.tuning_source}))")
    env = {k: v for k, v in os.environ.items() if not k.startswith("MMLTTB_")}
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True, text=True,
                         check=True).stdout.strip().splitlines()[-1]
    got = json.loads(out)
    cache = autotune.load_cache()
    if got["key"] not in cache:
        pytest.skip(f"the committed cache has no entry for {got['key']}")
    assert got["source"] == "cache: single, batched"
    for kind in autotune.LOAD_CLASSES:
        for arg, v in autotune.select(cache, got["key"], kind).items():
            assert got["tuning"][arg] == v, (kind, arg)


@pytest.mark.gpu
def test_tune_off_keeps_the_compiled_defaults():
    code = ("import json; from paper_2305_00332_amd import _lib, ops; _lib.load();"
            "print(json.dumps({'tuning': ops.get_tuning()._asdict(), 'source': _lib.tuning_source}))")
    env = {k: v for k, v in os.environ.items() if not k.startswith("MMLTTB_")}
    env["MMLTTB_TUNE"] = "off"
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True, text=True,
                         check=True).stdout.strip().splitlines()[-1]
    got = json.loads(out)
    assert got["source"] == "compiled defaults"
    assert got["tuning"] == {"unroll": 4, "chunk": 1 << 20, "chain": 3, "tile": 4096, "batch_unroll": 4,
                             "batch_chunk": 65536}
