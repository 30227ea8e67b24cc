"""Seeded synthetic inputs for the downsampling path.

This module holds only input generation: it computes nothing of the method.
Both the GPU path's tests and the oracle's tests draw their inputs here, so
the two sides see the same bytes. Generation runs in torch on the requested
device (CPU for small host-side cases, the GPU for the large workloads, whose
bytes are copied back to the host when the oracle needs them). Values are
built in float64 and cast once to float32.

Workload recipes (sizes follow the paper's setting: one long in-memory series
downsampled to a chart-sized n_out, section 3.2; many series of uneven length;
a resident pool queried by sub-range):
  random_walk        y = cumsum(N(0, sigma^2)), x implicit
  composite_series   random walk + 3 sinusoids (periods 1e3/1e5/1e7 samples,
                     amplitude 10) + N(0, 0.5^2) noise + 0.01% spikes of +-50,
                     x int64 timestamps with gaps 1 + floor(Exp(999.5)) ns
  batch_lengths      log-uniform integer lengths
  edge cases         ties, signed zeros, subnormals, extreme magnitudes,
                     epoch-nanosecond timestamps
  other types        float64 random walk, int32 counts (int_series), float64
                     timestamps in seconds (float_x), bursty int64 timestamps
                     with outages (bursty_x)
"""
from __future__ import annotations

import math

import numpy as np
import torch

_CHUNK = 1 << 26  # elements per generation chunk (bounds temporaries)


def _gen(seed: int, device) -> torch.Generator:
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    return g


def random_walk(n: int, seed: int, sigma: float = 1.0, device="cpu", start: float = 0.0,
                dtype=torch.float32) -> torch.Tensor:
    """Random walk with Gaussian increments (accumulated in float64), stored
    as dtype (float32 or float64)."""
    g = _gen(seed, device)
    out = torch.empty(n, dtype=dtype, device=device)
    carry = torch.tensor(start, dtype=torch.float64, device=device)
    for lo in range(0, n, _CHUNK):
        hi = min(n, lo + _CHUNK)
        inc = torch.randn(hi - lo, generator=g, dtype=torch.float64, device=device)
        if sigma != 1.0:
            inc.mul_(sigma)
        walk = torch.cumsum(inc, 0).add_(carry)
        carry = walk[-1].clone()
        out[lo:hi] = walk.to(dtype)
        del inc, walk
    return out


def int_series(n: int, seed: int, device="cpu", scale: float = 1e6) -> torch.Tensor:
    """int32 sensor counts: a float64 random walk of step sigma scale/1e3,
    rounded and clipped to the int32 range (long flat runs of equal values
    when scale is small)."""
    w = random_walk(n, seed, sigma=scale / 1e3, device=device, dtype=torch.float64)
    return torch.clamp(torch.round(w), -2 ** 31, 2 ** 31 - 1).to(torch.int32)


def float_x(n: int, seed: int, device="cpu", start: float = 1.7e9) -> torch.Tensor:
    """Strictly increasing float64 timestamps in seconds: start + cumulative
    gaps 1e-6 * (1 + Exp(999.5)), not integers."""
    g = _gen(seed + 11_000_003, device)
    out = torch.empty(n, dtype=torch.float64, device=device)
    carry = float(start)
    for lo in range(0, n, _CHUNK):
        hi = min(n, lo + _CHUNK)
        u = torch.rand(hi - lo, generator=g, dtype=torch.float64, device=device)
        gaps = (1.0 - torch.log1p(-u) * 999.5) * 1e-6
        if lo == 0:
            gaps[0] = 0.0
        xs = torch.cumsum(gaps, 0) + carry
        carry = float(xs[-1].item())
        out[lo:hi] = xs
    return out


def irregular_x(n: int, seed: int, mean_gap: float = 1000.0, start: int = 0, device="cpu") -> torch.Tensor:
    """Strictly increasing int64 timestamps: x_0 = start, gap = 1 + floor(Exp(mean_gap - 0.5))."""
    g = _gen(seed, device)
    out = torch.empty(n, dtype=torch.int64, device=device)
    carry = int(start)
    for lo in range(0, n, _CHUNK):
        hi = min(n, lo + _CHUNK)
        u = torch.rand(hi - lo, generator=g, dtype=torch.float64, device=device)
        gaps = torch.floor(-torch.log1p(-u) * (mean_gap - 0.5)).to(torch.int64) + 1
        if lo == 0:
            gaps[0] = 0
        xs = torch.cumsum(gaps, 0) + carry
        carry = int(xs[-1].item())
        out[lo:hi] = xs
        del u, gaps, xs
    return out


def composite_series(n: int, seed: int, device="cpu", with_x: bool = True, x_start: int = 0,
                     periods=(1e3, 1e5, 1e7), amplitude: float = 10.0, noise_sigma: float = 0.5,
                     spike_frac: float = 1e-4, spike_height: float = 50.0):
    """Random walk + sinusoids + Gaussian noise + sparse spikes; int64 irregular x.

    Returns (x, y) with x an int64 tensor (or None when with_x is False)."""
    gp = _gen(seed + 1_000_003, "cpu")
    phases = (torch.rand(len(periods), generator=gp, dtype=torch.float64) * (2 * math.pi)).tolist()
    y = torch.empty(n, dtype=torch.float32, device=device)
    gw = _gen(seed, device)  # walk increments
    gn = _gen(seed + 4_000_003, device)  # observation noise
    carry = torch.tensor(0.0, dtype=torch.float64, device=device)
    for lo in range(0, n, _CHUNK):
        hi = min(n, lo + _CHUNK)
        inc = torch.randn(hi - lo, generator=gw, dtype=torch.float64, device=device)
        walk = torch.cumsum(inc, 0).add_(carry)
        carry = walk[-1].clone()
        i = torch.arange(lo, hi, dtype=torch.float64, device=device)
        for p, ph in zip(periods, phases):
            walk.add_(torch.sin(i * (2 * math.pi / p) + ph) * amplitude)
        walk.add_(torch.randn(hi - lo, generator=gn, dtype=torch.float64, device=device) * noise_sigma)
        y[lo:hi] = walk.to(torch.float32)
        del inc, walk, i
    n_spikes = int(round(n * spike_frac))
    if n_spikes > 0:
        gs = _gen(seed + 2_000_003, "cpu")
        pos = torch.randperm(n, generator=gs)[:n_spikes] if n <= (1 << 27) else \
            torch.unique(torch.randint(0, n, (n_spikes * 2,), generator=gs))[:n_spikes]
        sign = torch.randint(0, 2, (pos.numel(),), generator=gs).to(torch.float64) * 2 - 1
        pos = pos.to(device)
        y[pos] = (y[pos].to(torch.float64) + sign.to(device) * spike_height).to(torch.float32)
    x = irregular_x(n, seed + 3_000_003, start=x_start, device=device) if with_x else None
    return x, y


def batch_lengths(count: int, lo: float, hi: float, seed: int) -> np.ndarray:
    """Integer lengths, log-uniform in [lo, hi] (host numpy, int64)."""
    rng = np.random.default_rng(seed)
    u = rng.uniform(math.log(lo), math.log(hi), size=count)
    return np.floor(np.exp(u)).astype(np.int64)


def choice(values, count: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.choice(np.asarray(values), size=count)


def batch_series(lengths, seed: int, device="cpu", with_x: bool = True, noise_sigma: float = 0.5,
                 sinusoids: bool = False, periods=(1e3, 1e5, 1e7), amplitude: float = 10.0):
    """Series of the given lengths stored back to back: y = random walk + N(0, 0.5^2)
    noise (one walk across the whole buffer, so each series is a walk segment),
    optionally + sinusoids of the given periods (in samples of the buffer),
    x = one strictly increasing irregular int64 timeline (each series a slice).
    Returns (x, y, offsets)."""
    lengths = np.asarray(lengths, dtype=np.int64)
    offsets = np.concatenate([[0], np.cumsum(lengths)[:-1]]).astype(np.int64)
    total = int(lengths.sum())
    y = random_walk(total, seed, device=device)
    g = _gen(seed + 5_000_011, device)
    for lo in range(0, total, _CHUNK):
        hi = min(total, lo + _CHUNK)
        v = y[lo:hi].to(torch.float64) + torch.randn(hi - lo, generator=g, dtype=torch.float64,
                                                      device=device) * noise_sigma
        if sinusoids:
            i = torch.arange(lo, hi, dtype=torch.float64, device=device)
            for p, ph in zip(periods, (0.3, 1.7, 4.1)):
                v.add_(torch.sin(i * (2 * math.pi / p) + ph) * amplitude)
            del i
        y[lo:hi] = v.to(torch.float32)
        del v
    x = irregular_x(total, seed + 6_000_011, device=device) if with_x else None
    return x, y, offsets


# ---------------------------------------------------------------- edge cases

def ties_series(n: int, seed: int, levels: int = 5, device="cpu") -> torch.Tensor:
    """Few distinct values (many exact ties), with -0.0 and +0.0 both present."""
    g = _gen(seed, device)
    v = torch.randint(-(levels // 2), levels - levels // 2, (n,), generator=g, device=device).to(torch.float32)
    flip = torch.rand(n, generator=g, device=device) < 0.5
    v = torch.where((v == 0) & flip, torch.tensor(-0.0, device=device), v)
    return v


def subnormal_series(n: int, seed: int, device="cpu") -> torch.Tensor:
    """Subnormal float32 values (plus some zeros of both signs)."""
    g = _gen(seed, device)
    k = torch.randint(-40, 41, (n,), generator=g, device=device).to(torch.float32)
    v = k * torch.tensor(1.401298464324817e-45, dtype=torch.float32)  # multiples of 2^-149
    zeros = torch.rand(n, generator=g, device=device) < 0.1
    v = torch.where(zeros, torch.tensor(-0.0, device=device), v)
    return v


def extreme_series(n: int, seed: int, device="cpu") -> torch.Tensor:
    """Magnitudes from 2^-149 up to near FLT_MAX, random signs."""
    g = _gen(seed, device)
    e = torch.randint(-149, 128, (n,), generator=g, device=device).to(torch.float64)
    m = 1.0 + torch.rand(n, generator=g, dtype=torch.float64, device=device) * 0.99
    s = torch.randint(0, 2, (n,), generator=g, device=device).to(torch.float64) * 2 - 1
    v = (s * m * torch.pow(torch.tensor(2.0, dtype=torch.float64, device=device), e)).to(torch.float32)
    return v


def bursty_x(n: int, seed: int, mean_gap: float = 1000.0, outage_frac: float = 1e-3,
             outage_len=(1e6, 1e9), start: int = 0, device="cpu") -> torch.Tensor:
    """Strictly increasing int64 timestamps with outages: gaps as irregular_x,
    plus, at a fraction outage_frac of the points, a jump drawn log-uniformly
    from outage_len (sensor downtime; leaves runs of empty x-width bins)."""
    base = irregular_x(n, seed, mean_gap=mean_gap, start=0, device=device)
    g = _gen(seed + 7_000_003, device)
    out = torch.empty(n, dtype=torch.int64, device=device)
    carry = 0
    lo_l, hi_l = math.log(outage_len[0]), math.log(outage_len[1])
    for lo in range(0, n, _CHUNK):
        hi = min(n, lo + _CHUNK)
        u = torch.rand(hi - lo, generator=g, dtype=torch.float64, device=device)
        v = torch.rand(hi - lo, generator=g, dtype=torch.float64, device=device)
        jump = torch.where(u < outage_frac, torch.exp(lo_l + v * (hi_l - lo_l)).floor(), torch.zeros_like(v))
        if lo == 0:
            jump[0] = 0
        js = torch.cumsum(jump.to(torch.int64), 0) + carry
        carry = int(js[-1].item())
        out[lo:hi] = base[lo:hi] + js + int(start)
    return out


def epoch_x(n: int, seed: int, device="cpu") -> torch.Tensor:
    """Nanosecond epoch timestamps (~1.7e18, above 2^53, so not exact in binary64)."""
    return irregular_x(n, seed, mean_gap=1000.0, start=1_700_000_000_123_456_789, device=device)


def to_numpy(t):
    return None if t is None else t.detach().cpu().numpy()
