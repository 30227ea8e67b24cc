"""Build libmmlttb.so for gfx950 with hipcc (in-tree, next to this file).

    python -m paper_2305_00332_amd.build

Flags that matter for results:
  -ffp-contract=off     no fused multiply-add: every binary64 operation of the
                        LTTB area is rounded separately, as the method defines.
  -target-feature -packed-fp32-ops
                        no packed FP32 instructions in generated code.
"""
from __future__ import annotations

import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libmmlttb.so")

SOURCES = ["minmax.hip", "lttb.hip", "lttb_tables.hip", "batched.hip", "downsamplers.hip", "xbins.hip", "typed.hip", "simplify.hip", "host.hip", "api.hip", "api_batched.hip", "noalloc.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-command-line-argument",
    "-I", INCLUDE,
    "-I", CSRC,
]


def sources():
    return [os.path.join(CSRC, s) for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    # hipcc's host pass does not know the packed-fp32 feature and says so: harmless
    noise = "is not a recognized feature for this target"
    out = "\n".join(l for l in res.stdout.splitlines() if noise not in l and l.strip())
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed ({res.returncode}):\n{out}")
    if out and verbose:
        print(out)


def build(verbose: bool = False, jobs: int | None = None) -> str:
    """Compile every HIP source into libmmlttb.so (always rebuilds): one object
    per source, compiled in parallel, then one shared-library link."""
    srcs = sources()
    jobs = jobs or min(len(srcs), max(1, min(os.cpu_count() or 1, 16)))
    with tempfile.TemporaryDirectory(prefix="mmlttb_build_") as tmpdir:
        objs = [os.path.join(tmpdir, os.path.basename(s) + ".o") for s in srcs]
        with ThreadPoolExecutor(max_workers=jobs) as pool:
            futs = [pool.submit(_run, [HIPCC, *FLAGS, "-c", "-o", o, s], verbose) for s, o in zip(srcs, objs)]
            for f in futs:
                f.result()
        tmp = LIB + ".tmp"
        _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
