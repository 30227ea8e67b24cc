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

// Decode the bin keys into the sorted distinct preselection P (section 3: the
// first and last points join the per-bin extrema). Bins are disjoint and in
// index order, so emitting each bin's pair in index order yields P sorted.
// Called by a whole workgroup of 1024 threads. Optionally writes XP (raw x,
// gathered, or the index for implicit x) and YP (decoded from the keys, so y
// is not read again) at the same time. wave_tot: 17 ints of LDS.
__device__ inline void compact_keys(const unsigned long long *__restrict__ keys, const Split &bins, int64_t n,
                                    const int64_t *__restrict__ x, const float *__restrict__ y,
                                    int64_t *__restrict__ P, int64_t *__restrict__ XP, float *__restrict__ YP,
                                    int64_t *__restrict__ m_out, int *wave_tot)
{
    const int tid = threadIdx.x;
    int64_t running = 1;
    if (tid == 0) {
        P[0] = 0;
        if (XP) {
            XP[0] = x ? x[0] : 0;
            YP[0] = y[0];
        }
    }
    const int64_t nb = bins.parts;
    for (int64_t base = 0; base < nb; base += blockDim.x) {
        const int64_t b = base + tid;
        int c = 0;
        int64_t i0 = 0, i1 = 0;
        float v0 = 0.0f, v1 = 0.0f;
        if (b < nb) {
            const int64_t blo = 1 + split_lo(bins, b);
            const unsigned long long kmin = keys[2 * b], kmax = keys[2 * b + 1];
            const int64_t imin = blo + min_key_offset(kmin);
            const int64_t imax = blo + max_key_offset(kmax);
            const bool lo_min = imin < imax;
            i0 = lo_min ? imin : imax;
            i1 = lo_min ? imax : imin;
            v0 = key_value(lo_min ? kmin : kmax);
            v1 = key_value(lo_min ? kmax : kmin);
            c = (imin == imax) ? 1 : 2;
        }
        int total;
        const int64_t off = running + block_exclusive_scan(c, wave_tot, total);
        if (c >= 1) {
            P[off] = i0;
            if (XP) {
                XP[off] = x ? x[i0] : i0;
                YP[off] = v0;
            }
        }
        if (c == 2) {
            P[off + 1] = i1;
            if (XP) {
                XP[off + 1] = x ? x[i1] : i1;
                YP[off + 1] = v1;
            }
        }
        running += total;
    }
    if (tid == 0) {
        P[running] = n - 1;
        if (XP) {
            XP[running] = x ? x[n - 1] : n - 1;
            YP[running] = y[n - 1];
        }
        *m_out = running + 1;
    }
}


} // namespace mmlttb
