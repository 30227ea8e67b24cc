// Device bodies of the LTTB means and of the segmented chain, shared by the
// single-series and the batched kernels.
#pragma once

#include "device_common.hpp"
#include "kernels.hpp"

namespace mmlttb {

// Positions of the bucket whose mean bucket k uses: bucket k+1, or the last
// point alone for the last interior bucket.
__device__ inline void next_bucket_range(const Split &bk, int64_t m, int64_t k, int64_t &g0, int64_t &g1)
{
    if (k < bk.parts - 1) {
        g0 = 1 + split_lo(bk, k + 1);
        g1 = 1 + split_lo(bk, k + 2);
    } else {
        g0 = m - 1;
        g1 = m;
    }
}

// Next-bucket mean of bucket k by one thread: exact sums of X and Y, each
// rounded once to binary64, then one binary64 division by the count.
// XP == NULL means x = position.
__device__ inline void bucket_mean_one(const int64_t *__restrict__ XP, const float *__restrict__ YP, const Split &bk,
                                       int64_t m, int64_t k, double &mx, double &my)
{
    int64_t g0, g1;
    next_bucket_range(bk, m, k, g0, g1);
    I64ExactSum sx;
    F32ExactSum sy;
    sx.clear();
    sy.clear();
    for (int64_t i = g0; i < g1; ++i) {
        sx.add(XP ? XP[i] : i);
        sy.add(YP[i]);
    }
    const double c = (double)(g1 - g0);
    mx = sx.round() / c;
    my = sy.round() / c;
}

// Phase 1 of the segmented chain for chain segment s (buckets
// [s*kSegLen, min(B, (s+1)*kSegLen))), one wave of kSegStarts lanes.
// A segment's walk depends only on its start point, which lies in the bucket
// just before the segment (point 0 for the first segment). Lane l walks the
// segment from start candidate l, with the segment's points and means staged
// in LDS (`lds`: 2*stage_cap + 2*kSegLen doubles), and records each pick's
// offset inside its bucket in path[(s*kSegStarts + l)*kSegLen + t] and the
// last one in finals[s*kSegStarts + l]. Every walk evaluates the same binary64
// area on the same operands as the sequential pass, so the walk from the true
// start repeats the sequential picks exactly.
template <class XT, class YT>
__device__ inline void seg_walk(const XT *__restrict__ XP, const YT *__restrict__ YP, const Split &bk,
                                const double *__restrict__ MX, const double *__restrict__ MY, int64_t s,
                                int stage_cap, double *lds, uint8_t *__restrict__ path,
                                uint8_t *__restrict__ finals)
{
    const int lane = threadIdx.x;
    const int64_t B = bk.parts;
    const int64_t k0 = s * kSegLen, k1 = (k0 + kSegLen < B) ? k0 + kSegLen : B;
    const int64_t p0 = 1 + split_lo(bk, k0), p1 = 1 + split_lo(bk, k1);
    double *sx = lds, *sy = lds + stage_cap, *smx = lds + 2 * stage_cap, *smy = smx + kSegLen;
    for (int64_t p = p0 + lane; p < p1; p += kSegStarts) {
        sx[p - p0] = (double)(XP ? XP[p] : p);
        sy[p - p0] = (double)YP[p];
    }
    for (int64_t k = k0 + lane; k < k1; k += kSegStarts) {
        smx[k - k0] = MX[k];
        smy[k - k0] = MY[k];
    }
    __syncthreads();

    int64_t apos = 0;
    if (s > 0) {
        const int64_t sa = 1 + split_lo(bk, k0 - 1);
        const int64_t ca = p0 - sa; // points of the bucket before the segment (<= kSegStarts)
        apos = sa + (lane < ca ? lane : ca - 1);
    }
    double ax = (double)(XP ? XP[apos] : apos);
    double ay = (double)YP[apos];
    SplitWalker w;
    w.init(bk, k0);
    uint8_t *mypath = path + ((size_t)s * kSegStarts + lane) * kSegLen;
    int bo = 0;
    for (int64_t k = k0; k < k1; ++k) {
        const int64_t s0 = 1 + w.lo, s1 = 1 + w.next_lo(bk);
        w.advance(bk);
        const double mx = smx[k - k0], my = smy[k - k0];
        // the bucket's first point stands unless an area beats -1 (areas are
        // >= 0, or NaN when binary64 means overflow: NaN never wins)
        double best = -1.0, bx = sx[s0 - p0], by = sy[s0 - p0];
        bo = 0;
        for (int64_t j = s0; j < s1; ++j) {
            const double xj = sx[j - p0], yj = sy[j - p0];
            const double ar = lttb_area2(ax, ay, xj, yj, mx, my);
            if (ar > best) { // strict: lowest position wins ties
                best = ar;
                bo = (int)(j - s0);
                bx = xj;
                by = yj;
            }
        }
        ax = bx;
        ay = by;
        mypath[k - k0] = (uint8_t)bo;
    }
    finals[(size_t)s * kSegStarts + lane] = (uint8_t)bo;
}

// Phase 2: follow the true start through the segments. The start of segment
// t+1 is the last pick of segment t walked from its own start: one LDS lookup
// per segment, by thread 0, with the finals staged in LDS windows of
// kChaseWindow segments by the whole workgroup. Runs in a later kernel than
// the walks, so their finals are visible without any fence. The starts go to
// `start` (global) and are visible to the whole workgroup on return.
__device__ inline void seg_link(const uint8_t *finals, uint8_t *start, int64_t S, uint8_t *F)
{
    const int tid = threadIdx.x;
    int cur = 0;
    if (tid == 0)
        start[0] = 0;
    for (int64_t w0 = 0; w0 < S - 1; w0 += kChaseWindow) {
        const int64_t w1 = (w0 + kChaseWindow < S - 1) ? w0 + kChaseWindow : S - 1;
        const int64_t words = (w1 - w0) * kSegStarts / 4;
        const uint32_t *src = reinterpret_cast<const uint32_t *>(finals + w0 * kSegStarts);
        for (int64_t q = tid; q < words; q += blockDim.x)
            reinterpret_cast<uint32_t *>(F)[q] = src[q];
        __syncthreads();
        if (tid == 0) {
            for (int64_t t = w0; t < w1; ++t) {
                cur = F[(t - w0) * kSegStarts + cur];
                start[t + 1] = (uint8_t)cur;
            }
        }
        __syncthreads();
    }
    __threadfence_block();
    __syncthreads();
}

// Phase 3 for one bucket: position of the pick of bucket k.
__device__ inline int64_t seg_pick(const uint8_t *__restrict__ path, const uint8_t *__restrict__ start, const Split &bk,
                                   int64_t k)
{
    const int64_t s = k / kSegLen;
    const int l = start[s];
    const int off = path[((size_t)s * kSegStarts + l) * kSegLen + (k - s * kSegLen)];
    return 1 + split_lo(bk, k) + off;
}

} // namespace mmlttb
