"""The paper's Fig. 3 example, rebuilt as a concrete instance
(tests/golden/fig3_lttb_surface.json): in bucket B_i, LTTB keeps point (1), a
high point at the left bin edge that is not the bucket's maximum, because the
maximum (3) lies below the equisurface line through (1); MinMaxLTTB with
r_ps = 2 preselects only the bucket's minimum (2) and maximum (3) and keeps
(3) (section 3.1). Checked on the oracle and on an exact-rational LTTB."""
from __future__ import annotations

import json
import os

import numpy as np
import pytest

import oracle
from tests import pins

FIX = os.path.join(os.path.dirname(__file__), "golden", "fig3_lttb_surface.json")


def fixture():
    with open(FIX) as f:
        fx = json.load(f)
    return fx, np.array(fx["y"], dtype=np.float32)


def test_instance_has_the_figure_shape():
    fx, y = fixture()
    lo, hi = pins.lttb_buckets(len(y), fx["n_out"])[fx["bucket"]]
    seg = y[lo:hi]
    assert lo == fx["point_1"]  # (1) sits at the left bin edge
    assert lo + int(np.argmax(seg)) == fx["point_3"] != fx["point_1"]  # (3) is the bucket maximum
    assert lo + int(np.argmin(seg)) == fx["point_2"]  # (2) is the bucket minimum


def test_lttb_keeps_the_left_edge_point():
    fx, y = fixture()
    out = oracle.lttb(y, fx["n_out"])
    assert out[fx["bucket"]] == fx["previous_pick"]
    assert out[fx["bucket"] + 1] == fx["point_1"]
    # the figure's buckets, against exact rational areas (means there are exact
    # up to far-from-tie rounding; later filler buckets are outside the claim)
    exact = pins.lttb_exact(list(range(len(y))), [int(v) for v in y], fx["n_out"])
    assert list(out[: fx["bucket"] + 2]) == exact[: fx["bucket"] + 2]


def test_minmax_preselects_min_and_max_only():
    fx, y = fixture()
    P = set(oracle.minmax(y, fx["n_out"], fx["r_ps"]).tolist())
    assert fx["point_2"] in P and fx["point_3"] in P and fx["point_1"] not in P


def test_minmaxlttb_keeps_the_bucket_maximum():
    fx, y = fixture()
    out = oracle.minmaxlttb(y, fx["n_out"], fx["r_ps"])
    assert out[fx["bucket"] + 1] == fx["point_3"]
    P = pins.minmax_by_numpy(y, fx["n_out"], fx["r_ps"])
    exact_pos = pins.lttb_exact(P.tolist(), [int(v) for v in y[P]], fx["n_out"])
    k = fx["bucket"] + 2
    assert list(out[:k]) == [int(P[p]) for p in exact_pos[:k]]


@pytest.mark.gpu
def test_gpu_path_reproduces_the_figure():
    import torch

    from paper_2305_00332_amd import ops

    fx, y = fixture()
    yd = torch.from_numpy(y).cuda()
    assert int(ops.lttb(yd, fx["n_out"])[fx["bucket"] + 1]) == fx["point_1"]
    assert int(ops.minmaxlttb(yd, fx["n_out"], fx["r_ps"])[fx["bucket"] + 1]) == fx["point_3"]
