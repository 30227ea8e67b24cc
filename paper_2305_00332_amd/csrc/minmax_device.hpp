// Device bodies of the MinMax stream, shared by the single-series and the
// batched kernels.
#pragma once

#include "device_common.hpp"

namespace mmlttb {

// Bin key pair. High 32 bits: order key of the value (f32_order_key, so
// -0.0 == +0.0); low 32 bits: offset of the index inside its bin (min key) or
// its complement (max key). atomicMin / atomicMax on these keys then keep the
// smallest / largest value and, among equal values, the lowest index.
__device__ inline unsigned long long pack_min_key(float v, int64_t off)
{
    return ((unsigned long long)f32_order_key(v) << 32) | (unsigned long long)(uint32_t)off;
}

__device__ inline unsigned long long pack_max_key(float v, int64_t off)
{
    return ((unsigned long long)f32_order_key(v) << 32) | (unsigned long long)(0xffffffffu - (uint32_t)off);
}

// Puts one work item's key pair into its bin. A bin that is a single work
// item (`whole`) has no other contributor, so a plain store gives what an
// atomic merge into identity keys would, and the keys need no initialisation;
// otherwise the item merges with atomicMin / atomicMax into keys that start
// at the identities (~0 for the min key, 0 for the max key).
__device__ inline void put_bin_keys(unsigned long long *keys, int64_t b, bool whole, unsigned long long kmin,
                                    unsigned long long kmax)
{
    if (whole) {
        keys[2 * b] = kmin;
        keys[2 * b + 1] = kmax;
    } else {
        atomicMin(&keys[2 * b], kmin);
        atomicMax(&keys[2 * b + 1], kmax);
    }
}

__device__ inline int64_t min_key_offset(unsigned long long k) { return (int64_t)(uint32_t)(k & 0xffffffffull); }

// The value a key holds (inverse of f32_order_key; -0.0 comes back as +0.0,
// which no sum or area can tell apart).
__device__ inline float key_value(unsigned long long k)
{
    const uint32_t o = (uint32_t)(k >> 32);
    return __uint_as_float((o & 0x80000000u) ? (o ^ 0x80000000u) : ~o);
}

__device__ inline int64_t max_key_offset(unsigned long long k)
{
    return (int64_t)(0xffffffffu - (uint32_t)(k & 0xffffffffull));
}

// Reduce y[lo, hi) (hi > lo) with one full wave. Returns, uniform across the
// wave, the minimum and maximum values and the lowest index of each.
template <int U>
__device__ inline void wave_reduce_range(const float *__restrict__ y, int64_t lo, int64_t hi, int lane, float &o_min,
                                         int64_t &o_imin, float &o_max, int64_t &o_imax)
{
    const float kNaN = __int_as_float(0x7fc00000);
    // Head: points before the first 16-byte aligned address; tail: after the
    // last full float4. At most 3 each, handled by lanes 0-2 and 4-6.
    const uint64_t addr = (uint64_t)(uintptr_t)(y + lo);
    int64_t head = (int64_t)(((16u - (unsigned)(addr & 15u)) & 15u) >> 2);
    head = head < hi - lo ? head : hi - lo;
    const int64_t body = lo + head;
    const int64_t nvec = (hi - body) >> 2;
    const int64_t body_end = body + (nvec << 2);
    const f32x4 *__restrict__ v4 = reinterpret_cast<const f32x4 *>(y + body);

    float sv = kNaN; // NaN: identity of fminf/fmaxf
    int64_t sidx = INT64_MAX;
    if (lane < head) {
        sidx = lo + lane;
        sv = y[sidx];
    } else if (lane >= 4 && lane < 4 + (hi - body_end)) {
        sidx = body_end + (lane - 4);
        sv = y[sidx];
    }

    constexpr int64_t kPerBatch = (int64_t)kWave * U; // float4 per batch
    const int64_t nfull = nvec / kPerBatch;
    float mn = __int_as_float(0x7f800000), mx = -__int_as_float(0x7f800000);
    int64_t bmn = -1, bmx = -1;
    for (int64_t t = 0; t < nfull; ++t) {
        f32x4 d[U];
        const f32x4 *p = v4 + t * kPerBatch + lane;
#pragma unroll
        for (int u = 0; u < U; ++u)
            d[u] = __builtin_nontemporal_load(p + u * kWave);
        float a = fminf(fminf(d[0].x, d[0].y), fminf(d[0].z, d[0].w));
        float b = fmaxf(fmaxf(d[0].x, d[0].y), fmaxf(d[0].z, d[0].w));
#pragma unroll
        for (int u = 1; u < U; ++u) {
            a = fminf(a, fminf(fminf(d[u].x, d[u].y), fminf(d[u].z, d[u].w)));
            b = fmaxf(b, fmaxf(fmaxf(d[u].x, d[u].y), fmaxf(d[u].z, d[u].w)));
        }
        if (a < mn) {
            mn = a;
            bmn = t;
        }
        if (b > mx) {
            mx = b;
            bmx = t;
        }
    }
    if (nfull * kPerBatch < nvec) { // last, partial batch
        const int64_t t = nfull;
        float a = kNaN, b = kNaN;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            int64_t q = t * kPerBatch + u * kWave + lane;
            if (q < nvec) {
                f32x4 d = v4[q];
                a = fminf(a, fminf(fminf(d.x, d.y), fminf(d.z, d.w)));
                b = fmaxf(b, fmaxf(fmaxf(d.x, d.y), fmaxf(d.z, d.w)));
            }
        }
        if (a < mn) {
            mn = a;
            bmn = t;
        }
        if (b > mx) {
            mx = b;
            bmx = t;
        }
    }

    const float wmin = wave_min_f32(fminf(mn, sv));
    const float wmax = wave_max_f32(fmaxf(mx, sv));

    // Lowest index holding each extreme: the lane's scalar point, and the
    // first match inside the lane's winning batch (batches of one lane are
    // visited in increasing index order, so the first batch that reached the
    // value holds the lane's lowest such index).
    int64_t cmin = (sv == wmin) ? sidx : INT64_MAX;
    int64_t cmax = (sv == wmax) ? sidx : INT64_MAX;
    if (bmn >= 0 && mn == wmin) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            int64_t q = bmn * kPerBatch + u * kWave + lane;
            if (q < nvec) {
                f32x4 d = v4[q];
                int64_t i = body + 4 * q;
                int64_t c = (d.x == wmin) ? i : (d.y == wmin) ? i + 1 : (d.z == wmin) ? i + 2 : (d.w == wmin) ? i + 3 : INT64_MAX;
                cmin = c < cmin ? c : cmin;
            }
        }
    }
    if (bmx >= 0 && mx == wmax) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            int64_t q = bmx * kPerBatch + u * kWave + lane;
            if (q < nvec) {
                f32x4 d = v4[q];
                int64_t i = body + 4 * q;
                int64_t c = (d.x == wmax) ? i : (d.y == wmax) ? i + 1 : (d.z == wmax) ? i + 2 : (d.w == wmax) ? i + 3 : INT64_MAX;
                cmax = c < cmax ? c : cmax;
            }
        }
    }
    o_min = wmin;
    o_max = wmax;
    o_imin = wave_min_i64(cmin);
    o_imax = wave_min_i64(cmax);
}

// Bin holding interior position p (1 <= p < 1 + bins.len): the last b with
// 1 + split_lo(bins, b) <= p. A binary64 estimate, corrected exactly.
__device__ inline int64_t bin_of(const Split &bins, int64_t p)
{
    const int64_t r = p - 1;
    int64_t b = (int64_t)((double)r * ((double)bins.parts / (double)bins.len));
    b = b < 0 ? 0 : (b >= bins.parts ? bins.parts - 1 : b);
    while (b > 0 && split_lo(bins, b) > r)
        --b;
    while (b + 1 < bins.parts && split_lo(bins, b + 1) <= r)
        ++b;
    return b;
}

// Per-lane running extremes of one bin part, positions relative to the
// stream's first point (-1: none yet). Points arrive in increasing position
// per lane, so strict comparisons keep the lowest position of each extreme.
struct PartAcc {
    float vmin, vmax;
    int32_t imin, imax;
    __device__ void reset()
    {
        vmin = __int_as_float(0x7f800000);
        vmax = -__int_as_float(0x7f800000);
        imin = imax = -1;
    }
    __device__ void add(float v, int32_t i)
    {
        if (v < vmin) {
            vmin = v;
            imin = i;
        }
        if (v > vmax) {
            vmax = v;
            imax = i;
        }
    }
    __device__ void add_if(float v, int32_t i, bool in)
    {
        const float kInf = __int_as_float(0x7f800000);
        const float a = in ? v : kInf, b = in ? v : -kInf;
        if (a < vmin) {
            vmin = a;
            imin = i;
        }
        if (b > vmax) {
            vmax = b;
            imax = i;
        }
    }
};

// MinMax keys of every bin part of y[lo, hi) (1 <= lo < hi <= 1 + bins.len,
// hi - lo < 2^31) with one full wave, merged into keys[2b], keys[2b + 1] by
// atomicMin / atomicMax (up to 64 parts per vector atomic), so parts of one
// bin streamed by different waves combine in any order. Reads stay in flight across bin ends: the body is
// read in batches of U float4 per lane, the next batch requested before the
// current one is reduced; a batch cut by bin ends is reduced part by part.
// Each finished part is reduced across the wave (packed keys) and merged. A
// part whose values never compare below +inf (or above -inf) reports its
// first position, so every key that a part touches decodes into its bin.
template <int U>
__device__ inline void wave_stream_bins(const float *__restrict__ y, int64_t lo, int64_t hi, const Split &bins,
                                        unsigned long long *__restrict__ keys, int lane)
{
    const float kInf = __int_as_float(0x7f800000);
    int64_t b = bin_of(bins, lo);
    SplitWalker w;
    w.init(bins, b);
    int64_t blo = 1 + w.lo, bend = 1 + w.next_lo(bins), part_lo = lo;
    PartAcc acc;
    acc.reset();
    // Finished parts wait in lane `held` (one part per lane) and go out as one
    // vector atomic per 64 parts: an atomic ahead of a load in the queue would
    // hold up the wait for that load.
    unsigned long long hold_min = 0, hold_max = 0;
    int64_t hold_bin = 0;
    int held = 0;
    auto release = [&]() {
        if (lane < held) {
            atomicMin(&keys[2 * hold_bin], hold_min);
            atomicMax(&keys[2 * hold_bin + 1], hold_max);
        }
        held = 0;
    };
    auto merge_part = [&]() {
        unsigned long long kmin = acc.imin >= 0 ? pack_min_key(acc.vmin, lo + acc.imin - blo) : ~0ull;
        unsigned long long kmax = acc.imax >= 0 ? pack_max_key(acc.vmax, lo + acc.imax - blo) : 0ull;
        wave_minmax_u64(kmin, kmax);
        if (kmin == ~0ull)
            kmin = pack_min_key(kInf, part_lo - blo);
        if (kmax == 0ull)
            kmax = pack_max_key(-kInf, part_lo - blo);
        if (lane == held) {
            hold_min = kmin;
            hold_max = kmax;
            hold_bin = b;
        }
        if (++held == kWave)
            release();
    };
    auto close_bin = [&]() { // bend reached: merge the part, move to the next bin
        merge_part();
        acc.reset();
        w.advance(bins);
        ++b;
        blo = bend;
        bend = 1 + w.next_lo(bins);
        part_lo = blo;
    };
    // One point per lane (pos < 0: none) covering positions [r0, r1).
    auto scalar_span = [&](int64_t r0, int64_t r1, float v, int64_t pos) {
        int64_t c = r0;
        while (c < r1) {
            const int64_t e = r1 < bend ? r1 : bend;
            if (pos >= c && pos < e)
                acc.add(v, (int32_t)(pos - lo));
            c = e;
            if (c == bend)
                close_bin();
        }
    };

    // 16-byte aligned body [body, body_end); head [lo, body) and tail
    // [body_end, hi) hold at most 3 points each, one per lane.
    const uint64_t addr = (uint64_t)(uintptr_t)(y + lo);
    int64_t head = (int64_t)(((16u - (unsigned)(addr & 15u)) & 15u) >> 2);
    head = head < hi - lo ? head : hi - lo;
    const int64_t body = lo + head;
    const int64_t nvec = (hi - body) >> 2;
    const int64_t body_end = body + 4 * nvec;
    {
        const int64_t pos = lane < head ? lo + lane : -1;
        scalar_span(lo, body, pos >= 0 ? y[pos] : 0.0f, pos);
    }

    const f32x4 *__restrict__ v4 = reinterpret_cast<const f32x4 *>(y + body);
    constexpr int64_t kVec = (int64_t)kWave * U; // float4 per batch
    const int64_t nfull = nvec / kVec; // full batches; a partial one may follow
    auto load = [&](f32x4(&d)[U], int64_t t) {
#pragma unroll
        for (int u = 0; u < U; ++u)
            d[u] = __builtin_nontemporal_load(v4 + t * kVec + (int64_t)u * kWave + lane);
    };
    // The points of slab u (one float4 per lane, 4 * kWave positions from
    // s0) that lie in positions [c, e), for a slab a bin end cuts. Points
    // outside enter as +inf to the minimum and -inf to the maximum, which
    // never replace a running extreme: selects, no branch.
    auto slab_part = [&](const f32x4 &v, int32_t r, int64_t c, int64_t e) {
        const int32_t rc = (int32_t)(c - lo), re = (int32_t)(e - lo);
        acc.add_if(v.x, r, r >= rc && r < re);
        acc.add_if(v.y, r + 1, r + 1 >= rc && r + 1 < re);
        acc.add_if(v.z, r + 2, r + 2 >= rc && r + 2 < re);
        acc.add_if(v.w, r + 3, r + 3 >= rc && r + 3 < re);
    };
    // A batch inside one bin (the common case) is reduced without a branch.
    // Otherwise slab by slab: whole slabs before the bin end go in directly,
    // only the slab holding it is split. Loops and atomics come after the
    // slab reads they depend on, so each batch's registers are waited for
    // alone while the next batch stays in flight.
    auto reduce = [&](const f32x4(&d)[U], int64_t t) {
        const int64_t base = body + 4 * t * kVec;
        const int64_t bhi = (base + 4 * kVec < body_end) ? base + 4 * kVec : body_end;
        const int32_t rel = (int32_t)(base - lo) + 4 * lane; // the lane's first point, relative to lo
        if (bhi == base + 4 * kVec && bhi < bend) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                acc.add(d[u].x, rel + u * 4 * kWave);
                acc.add(d[u].y, rel + u * 4 * kWave + 1);
                acc.add(d[u].z, rel + u * 4 * kWave + 2);
                acc.add(d[u].w, rel + u * 4 * kWave + 3);
            }
            return;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t s0 = base + (int64_t)u * 4 * kWave;
            const int64_t s1 = (s0 + 4 * kWave < bhi) ? s0 + 4 * kWave : bhi;
            const int32_t r = rel + u * 4 * kWave;
            if (s0 >= s1)
                continue; // past the end of a partial batch
            if (s1 == s0 + 4 * kWave && s1 < bend) {
                acc.add(d[u].x, r);
                acc.add(d[u].y, r + 1);
                acc.add(d[u].z, r + 2);
                acc.add(d[u].w, r + 3);
                continue;
            }
            int64_t e = s1 < bend ? s1 : bend;
            slab_part(d[u], r, s0, e);
            if (e == bend)
                close_bin();
            for (int64_t c = e; c < s1; c = e) { // bins shorter than a slab
                e = s1 < bend ? s1 : bend;
                slab_part(d[u], r, c, e);
                if (e == bend)
                    close_bin();
            }
        }
    };
    // Two register sets in turn over the full batches: the next batch is in
    // flight while one is reduced. Loads and reductions pair up on every
    // path, so each reduction waits for its own batch only.
    f32x4 da[U], db[U];
    int64_t t = 0;
    if (nfull > 0)
        load(da, 0);
    for (; t + 1 < nfull; t += 2) { // batch t is in da
        load(db, t + 1);
        reduce(da, t);
        load(da, t + 2 < nfull ? t + 2 : nfull - 1); // the last one again at the end: never reduced
        reduce(db, t + 1);
    }
    if (t < nfull)
        reduce(da, t);
    if (nfull * kVec < nvec) { // partial last batch: missing float4 are never read
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t q = nfull * kVec + (int64_t)u * kWave + lane;
            db[u] = q < nvec ? __builtin_nontemporal_load(v4 + q) : f32x4{0.0f, 0.0f, 0.0f, 0.0f};
        }
        reduce(db, nfull);
    }
    {
        const int64_t pos = lane < hi - body_end ? body_end + lane : -1;
        scalar_span(body_end, hi, pos >= 0 ? y[pos] : 0.0f, pos);
    }
    if (part_lo < hi) // the stream ends inside a bin: merge that part
        merge_part();
    release();
}

// Block-wide exclusive scan of small non-negative counts (blockDim 1024).
__device__ inline int block_exclusive_scan(int c, int *wave_tot, int &total)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
    const int nw = blockDim.x / kWave;
    int incl = c;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        int o = __shfl_up(incl, off);
        incl += (lane >= off) ? o : 0;
    }
    if (lane == kWave - 1)
        wave_tot[wid] = incl;
    __syncthreads();
    if (threadIdx.x == 0) {
        int run = 0;
        for (int w = 0; w < nw; ++w) {
            int t = wave_tot[w];
            wave_tot[w] = run;
            run += t;
        }
        wave_tot[nw] = run;
    }
    __syncthreads();
    total = wave_tot[nw];
    int r = wave_tot[wid] + incl - c;
    __syncthreads(); // wave_tot may be reused by the caller's next round
    return r;
}

// One bin's kept points from its key pair: the lowest index of the minimum and
// of the maximum (offsets inside the bin), in index order; 1 when they
// coincide, else 2. A key offset past its bin (keys no part ever reached, or
// values that never compare, such as NaN) decodes to the bin's first point, so
// every index stays inside its bin.
__device__ inline int decode_bin(unsigned long long kmin, unsigned long long kmax, int64_t blo, int64_t len,
                                 int64_t &i0, int64_t &i1, float &v0, float &v1)
{
    int64_t omin = min_key_offset(kmin), omax = max_key_offset(kmax);
    omin = omin < len ? omin : 0;
    omax = omax < len ? omax : 0;
    const int64_t imin = 1 + blo + omin, imax = 1 + blo + omax;
    const float vmin = key_value(kmin), vmax = key_value(kmax);
    const bool lo_min = imin < imax;
    i0 = lo_min ? imin : imax;
    i1 = lo_min ? imax : imin;
    v0 = lo_min ? vmin : vmax;
    v1 = lo_min ? vmax : vmin;
    return (imin == imax) ? 1 : 2;
}

// Points of bin b alone (as decode_bin counts them).
__device__ inline int bin_kept(const unsigned long long *__restrict__ keys, const Split &bins, int64_t b)
{
    const int64_t blo = split_lo(bins, b), len = split_lo(bins, b + 1) - blo;
    int64_t i0, i1;
    float v0, v1;
    return decode_bin(keys[2 * b], keys[2 * b + 1], blo, len, i0, i1, v0, v1);
}

// Decode the keys of bins [b0, b1) into P from slot `first` on (section 3:
// the per-bin extrema; the first and last points are the caller's). Bins are
// disjoint and in index order, so emitting each bin's pair in index order
// yields P sorted. Called by a whole workgroup (blockDim a multiple of 64, at
// most 1024). A round covers kCompactBins slabs of blockDim consecutive bins,
// bin base + u*blockDim + tid for thread tid: the keys of all slabs are
// decoded and scanned slab by slab, then the x gathers of all of them are in
// flight together. Optionally writes XP (raw x, gathered, or the index for
// implicit x) and YP (decoded from the keys, so y is not read again).
// Returns the slot after the last one written (the same in every thread).
// wave_tot: 17 ints of LDS.
constexpr int kCompactBins = 4;
__device__ inline int64_t compact_bin_range(const unsigned long long *__restrict__ keys, const Split &bins, int64_t b0,
                                            int64_t b1, int64_t first, const int64_t *__restrict__ x,
                                            int64_t *__restrict__ P, int64_t *__restrict__ XP,
                                            float *__restrict__ YP, int *wave_tot)
{
    const int tid = threadIdx.x;
    int64_t running = first;
    for (int64_t base = b0; base < b1; base += (int64_t)blockDim.x * kCompactBins) {
        int64_t i0[kCompactBins], i1[kCompactBins], off[kCompactBins];
        float v0[kCompactBins], v1[kCompactBins];
        int cnt[kCompactBins];
        unsigned long long kmin[kCompactBins], kmax[kCompactBins];
#pragma unroll
        for (int u = 0; u < kCompactBins; ++u) {
            const int64_t b = base + (int64_t)u * blockDim.x + tid;
            if (b < b1) {
                kmin[u] = keys[2 * b];
                kmax[u] = keys[2 * b + 1];
            }
        }
#pragma unroll
        for (int u = 0; u < kCompactBins; ++u) {
            const int64_t b = base + (int64_t)u * blockDim.x + tid;
            cnt[u] = 0;
            i0[u] = i1[u] = 0;
            v0[u] = v1[u] = 0.0f;
            if (b < b1) {
                const int64_t blo = split_lo(bins, b), len = split_lo(bins, b + 1) - blo;
                cnt[u] = decode_bin(kmin[u], kmax[u], blo, len, i0[u], i1[u], v0[u], v1[u]);
            }
            int total;
            off[u] = running + block_exclusive_scan(cnt[u], wave_tot, total);
            running += total;
        }
        int64_t xs0[kCompactBins], xs1[kCompactBins];
        if (XP) {
#pragma unroll
            for (int u = 0; u < kCompactBins; ++u) { // gathers first, all in flight
                xs0[u] = (x && cnt[u] >= 1) ? x[i0[u]] : i0[u];
                xs1[u] = (x && cnt[u] == 2) ? x[i1[u]] : i1[u];
            }
        }
#pragma unroll
        for (int u = 0; u < kCompactBins; ++u) {
            if (cnt[u] >= 1) {
                P[off[u]] = i0[u];
                if (XP) {
                    XP[off[u]] = xs0[u];
                    YP[off[u]] = v0[u];
                }
            }
            if (cnt[u] == 2) {
                P[off[u] + 1] = i1[u];
                if (XP) {
                    XP[off[u] + 1] = xs1[u];
                    YP[off[u] + 1] = v1[u];
                }
            }
        }
    }
    return running;
}

// The first point (slot 0) or the last point of the series into P (and XP,
// YP): one thread.
__device__ inline void put_end_point(int64_t slot, int64_t i, const int64_t *__restrict__ x,
                                     const float *__restrict__ y, int64_t *__restrict__ P, int64_t *__restrict__ XP,
                                     float *__restrict__ YP)
{
    P[slot] = i;
    if (XP) {
        XP[slot] = x ? x[i] : i;
        YP[slot] = y[i];
    }
}

// The whole preselection P = {0} + every bin's kept points + {n-1} by one
// workgroup, and its size into *m_out.
__device__ inline void compact_keys(const unsigned long long *__restrict__ keys, const Split &bins, int64_t n,
                                    const int64_t *__restrict__ x, const float *__restrict__ y,
                                    int64_t *__restrict__ P, int64_t *__restrict__ XP, float *__restrict__ YP,
                                    int64_t *__restrict__ m_out, int *wave_tot)
{
    if (threadIdx.x == 0)
        put_end_point(0, 0, x, y, P, XP, YP);
    const int64_t running = compact_bin_range(keys, bins, 0, bins.parts, 1, x, P, XP, YP, wave_tot);
    if (threadIdx.x == 0) {
        put_end_point(running, n - 1, x, y, P, XP, YP);
        *m_out = running + 1;
    }
}


} // namespace mmlttb
