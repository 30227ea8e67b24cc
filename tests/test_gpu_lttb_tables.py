"""Whole-series LTTB with wide buckets (the transition-table form) == oracle,
element by element, and == the sequential pass. Shapes give buckets of a few
hundred to 10^5 points; the series cover hulls of a few vertices (walks,
sinusoids with spikes), hulls too large for the candidate lists (convex,
collinear and constant series: every bucket scanned in full), exact ties and
mixed signs, with implicit, irregular and epoch-nanosecond x."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
from paper_2305_00332_amd import ops, synth

pytestmark = pytest.mark.gpu

DEV = "cuda"


def _y(kind, n, seed):
    rng = np.random.default_rng(seed)
    t = np.arange(n, dtype=np.float64)
    if kind == "walk":
        return synth.to_numpy(synth.random_walk(n, seed))
    if kind == "composite":
        return synth.to_numpy(synth.composite_series(n, seed, with_x=False)[1])
    if kind == "ties":
        return synth.to_numpy(synth.ties_series(n, seed))
    if kind == "convex":  # every point on the lower hull of its bucket
        return ((t / n - 0.5) ** 2 * 1e4).astype(np.float32)
    if kind == "line":  # collinear: every point on both chains
        return (t * 0.25 - 7.0).astype(np.float32)
    if kind == "constant":
        return np.full(n, 2.5, dtype=np.float32)
    if kind == "sawtooth":  # repeated equal extremes in every bucket
        return ((t % 97) - 48).astype(np.float32)
    if kind == "spiky":  # flat noise with rare large spikes of both signs
        y = rng.standard_normal(n).astype(np.float32) * 0.01
        idx = rng.choice(n, size=max(1, n // 5000), replace=False)
        y[idx] = rng.choice([-50.0, 50.0], size=idx.size).astype(np.float32)
        return y
    raise ValueError(kind)


def _x(seed, n):
    k = seed % 3
    if k == 0:
        return None
    if k == 1:
        return synth.to_numpy(synth.irregular_x(n, seed))
    return synth.to_numpy(synth.epoch_x(n, seed))


KINDS = ["walk", "composite", "ties", "convex", "line", "constant", "sawtooth", "spiky"]


def _cases():
    rng = np.random.default_rng(77)
    out = []
    for c in range(48):
        n = int(np.exp(rng.uniform(np.log(2e4), np.log(3e6))))
        n_out = int(rng.integers(3, max(4, min(400, n // 100))))
        out.append((c, KINDS[c % len(KINDS)], n, n_out))
    return out


@pytest.mark.parametrize("case", _cases(), ids=lambda c: f"s{c[0]}-{c[1]}-n{c[2]}-o{c[3]}")
def test_wide_lttb_matches_oracle_and_sequential(case):
    seed, kind, n, n_out = case
    y = _y(kind, n, seed)
    x = _x(seed, n)
    yd = torch.from_numpy(y).to(DEV)
    xd = None if x is None else torch.from_numpy(x).to(DEV)
    got = ops.lttb(yd, n_out, x=xd).cpu().numpy()
    np.testing.assert_array_equal(got, oracle.lttb(y, n_out, x))
    old = ops.get_tuning()
    try:
        ops.set_tuning(0, 0, ops.CHAIN_SEQUENTIAL)
        seq = ops.lttb(yd, n_out, x=xd).cpu().numpy()
    finally:
        ops.set_tuning(*old)
    np.testing.assert_array_equal(got, seq)


def test_repeated_calls_reuse_the_workspace():
    n, n_out = 2_000_003, 501
    y = synth.random_walk(n, 3, device=DEV)
    ws = torch.empty(ops.lttb_workspace_size(n, n_out), dtype=torch.uint8, device=DEV)
    first = ops.lttb(y, n_out, ws=ws).clone()
    z = synth.composite_series(n, 4, with_x=False)[1].to(DEV)
    second = ops.lttb(z, n_out, ws=ws).cpu().numpy()  # tables of the first call must not leak
    np.testing.assert_array_equal(second, oracle.lttb(z.cpu().numpy(), n_out, None))
    np.testing.assert_array_equal(first.cpu().numpy(), oracle.lttb(y.cpu().numpy(), n_out, None))


@pytest.mark.parametrize("y_off", [0, 1, 2, 3])
@pytest.mark.parametrize("x_off", [0, 1])
def test_group_loads_at_every_alignment(y_off, x_off):
    """The tables and the wide means read 4-point groups from the first
    16-byte boundary of y, with x in 16-byte pairs when x shares that
    alignment and point by point otherwise: every start offset of y and x."""
    n, n_out = 300_001, 102
    rng = np.random.default_rng(77 + 4 * x_off + y_off)
    y_np = (np.cumsum(rng.standard_normal(n)) + 5 * rng.standard_normal(n)).astype(np.float32)
    x_np = np.cumsum(rng.integers(1, 2000, n)).astype(np.int64)
    ybuf = torch.empty(n + y_off, dtype=torch.float32, device="cuda")
    ybuf[y_off:] = torch.from_numpy(y_np).to("cuda")
    xbuf = torch.empty(n + x_off, dtype=torch.int64, device="cuda")
    xbuf[x_off:] = torch.from_numpy(x_np).to("cuda")
    got = ops.lttb(ybuf[y_off:], n_out, x=xbuf[x_off:]).cpu().numpy()
    np.testing.assert_array_equal(got, oracle.lttb(y_np, n_out, x_np))
    got_i = ops.lttb(ybuf[y_off:], n_out).cpu().numpy()
    np.testing.assert_array_equal(got_i, oracle.lttb(y_np, n_out))


@pytest.mark.parametrize("per_bucket", [65, 100, 257, 8187, 8192, 8196, 8451])
@pytest.mark.parametrize("y_off", [0, 3])
@pytest.mark.parametrize("kind", ["walk", "composite", "spiky"])
def test_slab_rows_around_32_chunks(per_bucket, y_off, kind):
    """Buckets of at most 32 chunks of 256 points keep a slab per 64-point row
    in both passes, longer buckets a slab per chunk: buckets of a few rows and
    just below, at and above 8192 points, at two alignments of y, equal the
    oracle and the sequential pass."""
    n_out = 40
    n = (n_out - 2) * per_bucket + 2
    y_np = _y(kind, n, per_bucket + y_off)
    x_np = _x(per_bucket, n)
    ybuf = torch.empty(n + y_off, dtype=torch.float32, device=DEV)
    ybuf[y_off:] = torch.from_numpy(y_np).to(DEV)
    xd = None if x_np is None else torch.from_numpy(x_np).to(DEV)
    got = ops.lttb(ybuf[y_off:], n_out, x=xd).cpu().numpy()
    np.testing.assert_array_equal(got, oracle.lttb(y_np, n_out, x_np))
    old = ops.get_tuning()
    try:
        ops.set_tuning(0, 0, ops.CHAIN_SEQUENTIAL)
        seq = ops.lttb(ybuf[y_off:], n_out, x=xd).cpu().numpy()
    finally:
        ops.set_tuning(*old)
    np.testing.assert_array_equal(got, seq)
