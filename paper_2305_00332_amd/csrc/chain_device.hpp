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
//
// Buckets of at most kFastMean points take a short form that gives the same
// two binary64 values, with the loads of up to kFastLoad points issued
// together:
//  - X: every |x| at most 2^48, so the int64 sum of at most 16 stays within
//    2^52 and converts to binary64 exactly;
//  - Y: a float32 is mant * 2^(s - 149) with mant < 2^24 and s = max(E, 1) - 1
//    (E: biased exponent). If the nonzero values span s_min..s_max with
//    (s_max - s_min) + 24 + bits(count) <= 53, every partial sum is a multiple
//    of 2^(s_min - 149) below 2^(s_min - 149 + 53) in magnitude, so the
//    binary64 additions are exact and the sum needs no rounding.
// Otherwise (more points, a larger |x|, or Y values too far apart in scale)
// the exact accumulators run.
constexpr int kFastMean = 16;
constexpr int kFastLoad = 8;

__device__ inline void bucket_mean_exact(const int64_t *__restrict__ XP, const float *__restrict__ YP, int64_t g0,
                                         int64_t g1, double &mx, double &my)
{
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

// Folds one point into the short form's state.
struct FastMeanAcc {
    int64_t sx = 0;
    double sy = 0.0;
    int smin = 255, smax = -1;
    bool x_small = true;
    __device__ void add(int64_t x, float y)
    {
        sx = (int64_t)((uint64_t)sx + (uint64_t)x); // wraps, never overflows; used only when every |x| <= 2^48
        x_small = x_small && (uint64_t)x + (1ull << 48) < (1ull << 49);
        sy += (double)y;
        const uint32_t bits = __float_as_uint(y);
        const int e = (int)((bits >> 23) & 0xffu);
        const int sc = e ? e - 1 : 0;
        const bool nz = (bits & 0x7fffffffu) != 0u;
        smin = (nz && sc < smin) ? sc : smin;
        smax = (nz && sc > smax) ? sc : smax;
    }
};

__device__ inline void bucket_mean_one(const int64_t *__restrict__ XP, const float *__restrict__ YP, const Split &bk,
                                       int64_t m, int64_t k, double &mx, double &my)
{
    int64_t g0, g1;
    next_bucket_range(bk, m, k, g0, g1);
    const int cnt = (int)(g1 - g0 < kFastMean + 1 ? g1 - g0 : kFastMean + 1);
    if (cnt > kFastMean) {
        bucket_mean_exact(XP, YP, g0, g1, mx, my);
        return;
    }
    int64_t xs[kFastLoad];
    float ys[kFastLoad];
#pragma unroll
    for (int u = 0; u < kFastLoad; ++u) {
        if (u < cnt) {
            xs[u] = XP ? XP[g0 + u] : g0 + u;
            ys[u] = YP[g0 + u];
        }
    }
    FastMeanAcc a;
#pragma unroll
    for (int u = 0; u < kFastLoad; ++u)
        if (u < cnt)
            a.add(xs[u], ys[u]);
    for (int u = kFastLoad; u < cnt; ++u)
        a.add(XP ? XP[g0 + u] : g0 + u, YP[g0 + u]);
    const int cbits = 32 - __clz(cnt);
    if (!a.x_small || (a.smax >= 0 && (a.smax - a.smin) + 24 + cbits > 53)) {
        bucket_mean_exact(XP, YP, g0, g1, mx, my);
        return;
    }
    const double c = (double)cnt;
    mx = (double)a.sx / c;
    my = a.sy / c;
}

// Block-wide exact mean: every thread of a workgroup of 256 holds partial
// exact sums of x and y over its points; thread 0 writes the sums, each
// rounded once to binary64, divided by `count`. Ends with a barrier.
struct BlockMeanLds {
    int64_t limb[4][9];
    int64_t xlo[4], xhi[4];
};

__device__ inline void block_store_mean(I64ExactSum &sx, F32ExactSum &sy, int64_t count, BlockMeanLds &sm,
                                        double *mx, double *my)
{
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    sy.normalize();
    // wave sums: normalized limbs are < 2^32 (limb 8 small), 64 of them fit
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
#pragma unroll
        for (int q = 0; q < 9; ++q)
            sy.limb[q] += __shfl_xor(sy.limb[q], off);
        int64_t lo64 = (int64_t)(uint64_t)sx.s, hi64 = (int64_t)(sx.s >> 64);
        int64_t olo = __shfl_xor(lo64, off), ohi = __shfl_xor(hi64, off);
        sx.s += (__int128)(((unsigned __int128)(uint64_t)ohi << 64) | (uint64_t)olo);
    }
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < 9; ++q)
            sm.limb[wid][q] = sy.limb[q];
        sm.xlo[wid] = (int64_t)(uint64_t)sx.s;
        sm.xhi[wid] = (int64_t)(sx.s >> 64);
    }
    __syncthreads();
    if (tid == 0) {
        F32ExactSum ty;
        ty.clear();
        I64ExactSum tx;
        tx.clear();
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
#pragma unroll
            for (int q = 0; q < 9; ++q)
                ty.limb[q] += sm.limb[w][q];
            tx.s += (__int128)(((unsigned __int128)(uint64_t)sm.xhi[w] << 64) | (uint64_t)sm.xlo[w]);
        }
        const double c = (double)count;
        *mx = tx.round() / c;
        *my = ty.round() / c;
    }
    __syncthreads();
}

// Phase 1 of the segmented chain for chain segment s (buckets
// [s*kSegLen, min(B, (s+1)*kSegLen))), one wave of kSegStarts lanes.
// A segment's walk depends only on its start point, which lies in the bucket
// just before the segment (point 0 for the first segment). The pick in bucket
// k depends only on the pick in bucket k-1, so the wave first tabulates, for
// every point of the segment's buckets but the last, its pick in the next
// bucket (one lane per point, all in parallel), and for every start its pick
// in the segment's first bucket; lane l then follows the table from start l.
// Each table entry evaluates the same binary64 area on the same operands as
// the sequential pass, so the walk from the true start repeats its picks
// exactly. Points, means, bucket starts and tables live in LDS
// (seg_walk_lds_bytes(stage_cap)). Lane l records each pick's offset inside
// its bucket in path[(s*kSegStarts + l)*kSegLen + t] and the last one in
// finals[s*kSegStarts + l].
template <class XT, class YT>
__device__ inline void seg_walk(const XT *__restrict__ XP, const YT *__restrict__ YP, const Split &bk,
                                const double *__restrict__ MX, const double *__restrict__ MY, int64_t s,
                                int stage_cap, unsigned char *lds, uint8_t *__restrict__ path,
                                uint8_t *__restrict__ finals, int lane, bool active = true)
{
    // A wave with `active` false walks nothing but meets the same two
    // workgroup barriers, so several waves of one workgroup can walk
    // segments side by side in rounds.
    const int64_t B = bk.parts;
    const int64_t k0 = s * kSegLen, k1 = (k0 + kSegLen < B) ? k0 + kSegLen : B;
    const int nk = (int)(k1 - k0);
    SplitWalker w;
    w.init(bk, k0);
    const int64_t p0 = 1 + w.lo;
    double *sx = reinterpret_cast<double *>(lds), *sy = sx + stage_cap, *smx = sy + stage_cap, *smy = smx + kSegLen;
    int32_t *sb = reinterpret_cast<int32_t *>(smy + kSegLen); // bucket starts relative to p0, nk + 1 of them
    uint8_t *T = reinterpret_cast<uint8_t *>(sb + kSegLen + 1); // point -> offset of its pick in the next bucket
    double ax0 = 0.0, ay0 = 0.0;
    if (active) {
        const int64_t p1 = 1 + split_lo(bk, k1);
        for (int64_t p = p0 + lane; p < p1; p += kSegStarts) {
            sx[p - p0] = (double)(XP ? XP[p] : p);
            sy[p - p0] = (double)YP[p];
        }
        for (int64_t k = k0 + lane; k < k1; k += kSegStarts) {
            smx[k - k0] = MX[k];
            smy[k - k0] = MY[k];
        }
        for (int i = lane; i <= nk; i += kSegStarts) // bucket starts, one per lane
            sb[i] = (int32_t)(1 + split_lo(bk, k0 + i) - p0);
        // start l: the l-th point of bucket k0 - 1 (the last one for lanes
        // past its end), whose size is q, plus one when the step into k0 carried
        int64_t apos = 0;
        if (s > 0) {
            const int64_t ca = bk.q + (w.rem < bk.r ? 1 : 0);
            apos = p0 - ca + (lane < ca ? lane : ca - 1);
        }
        ax0 = (double)(XP ? XP[apos] : apos);
        ay0 = (double)YP[apos];
    }
    __syncthreads();

    // the bucket's first point stands unless an area beats -1 (areas are >= 0,
    // or NaN when binary64 means overflow: NaN never wins); strict > keeps
    // the lowest position on ties
    auto pick = [&](double ax, double ay, int i) {
        const int j0 = sb[i], j1 = sb[i + 1];
        const double mx = smx[i], my = smy[i];
        double best = -1.0;
        int bo = 0;
        for (int j = j0; j < j1; ++j) {
            const double ar = lttb_area2(ax, ay, sx[j], sy[j], mx, my);
            if (ar > best) {
                best = ar;
                bo = j - j0;
            }
        }
        return bo;
    };
    int first = 0;
    if (active) {
        first = pick(ax0, ay0, 0);
        const int tab_end = sb[nk - 1]; // points of buckets 0 .. nk-2
        for (int r = lane; r < tab_end; r += kSegStarts) {
            int lo = 0, hi = nk - 1; // bucket of r: the last i with sb[i] <= r
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (sb[mid] <= r)
                    lo = mid;
                else
                    hi = mid;
            }
            T[r] = (uint8_t)pick(sx[r], sy[r], lo + 1);
        }
    }
    __syncthreads();
    if (!active)
        return;

    uint32_t words[kSegLen / 4];
#pragma unroll
    for (int q = 0; q < kSegLen / 4; ++q)
        words[q] = 0;
    int o = first;
    words[0] = (uint32_t)o;
#pragma unroll
    for (int i = 1; i < kSegLen; ++i) {
        if (i < nk) {
            o = T[sb[i - 1] + o];
            words[i / 4] |= (uint32_t)o << (8 * (i % 4));
        }
    }
    uint4 *dst = reinterpret_cast<uint4 *>(path + ((size_t)s * kSegStarts + lane) * kSegLen);
    dst[0] = make_uint4(words[0], words[1], words[2], words[3]);
    dst[1] = make_uint4(words[4], words[5], words[6], words[7]);
    finals[(size_t)s * kSegStarts + lane] = (uint8_t)o;
}

// Phase 2: follow the true start through the segments. The start of segment
// t+1 is the last pick of segment t walked from its own start: one LDS lookup
// per segment, by thread 0, with the finals staged in LDS windows of
// kChaseWindow segments by the whole workgroup. Runs after the walks, in a
// later kernel or after a workgroup barrier that follows them. The starts go to
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

typedef long long i64x2 __attribute__((ext_vector_type(2)));

// f(p, x, y) with the raw x (int64; the position when X is NULL) and y of
// every p in [s, e), spread over a workgroup of nthreads
// threads, each of which sees its points in increasing p. The body comes in
// groups of 4 points at a 16-byte boundary of Y: one 16-byte load of y and
// two 16-byte (or, when X is not aligned with Y, four 8-byte) loads of x per
// group, kDepth groups per thread in flight. The up to 3 points before the
// boundary go to threads 0-2 first, the up to 3 after the last group to
// threads 0-2 last.
template <int kDepth, bool kHasX, class F>
__device__ inline void scan_groups_x(const int64_t *__restrict__ X, const float *__restrict__ Y, int64_t s,
                                     int64_t e, int tid, int nthreads, F &&f)
{
    const uint64_t ya = (uint64_t)(uintptr_t)(Y + s);
    int64_t a0 = s + (int64_t)(((16u - (unsigned)(ya & 15u)) & 15u) >> 2);
    a0 = a0 < e ? a0 : e;
    if (s + tid < a0)
        f(s + tid, kHasX ? X[s + tid] : s + tid, Y[s + tid]);
    const int64_t nq = (e - a0) >> 2;
    const f32x4 *__restrict__ Y4 = reinterpret_cast<const f32x4 *>(Y + a0);
    const bool x16 = kHasX && ((((uint64_t)(uintptr_t)(X + a0)) & 15u) == 0);
    auto load_x = [&](int64_t q, int64_t (&xv)[4]) {
        const int64_t p0 = a0 + 4 * q;
        if (!kHasX) {
#pragma unroll
            for (int i = 0; i < 4; ++i)
                xv[i] = p0 + i;
        } else if (x16) {
            const i64x2 *__restrict__ X2 = reinterpret_cast<const i64x2 *>(X + p0);
            const i64x2 lo = X2[0], hi = X2[1];
            xv[0] = lo.x;
            xv[1] = lo.y;
            xv[2] = hi.x;
            xv[3] = hi.y;
        } else {
#pragma unroll
            for (int i = 0; i < 4; ++i)
                xv[i] = X[p0 + i];
        }
    };
    int64_t q = tid;
    for (; q + (int64_t)(kDepth - 1) * nthreads < nq; q += (int64_t)kDepth * nthreads) {
        f32x4 yv[kDepth];
        int64_t xv[kDepth][4];
#pragma unroll
        for (int u = 0; u < kDepth; ++u) {
            yv[u] = Y4[q + (int64_t)u * nthreads];
            load_x(q + (int64_t)u * nthreads, xv[u]);
        }
#pragma unroll
        for (int u = 0; u < kDepth; ++u) {
            const int64_t p0 = a0 + 4 * (q + (int64_t)u * nthreads);
            f(p0, xv[u][0], yv[u].x);
            f(p0 + 1, xv[u][1], yv[u].y);
            f(p0 + 2, xv[u][2], yv[u].z);
            f(p0 + 3, xv[u][3], yv[u].w);
        }
    }
    for (; q < nq; q += nthreads) {
        const f32x4 yv = Y4[q];
        int64_t xv[4];
        load_x(q, xv);
        const int64_t p0 = a0 + 4 * q;
        f(p0, xv[0], yv.x);
        f(p0 + 1, xv[1], yv.y);
        f(p0 + 2, xv[2], yv.z);
        f(p0 + 3, xv[3], yv.w);
    }
    const int64_t t0 = a0 + 4 * nq;
    if (t0 + tid < e)
        f(t0 + tid, kHasX ? X[t0 + tid] : t0 + tid, Y[t0 + tid]);
}

// Points [s, e) in chunks of 64 groups of 4 (256 points at a 16-byte
// boundary of Y), one chunk per wave at a time (wave w takes chunks w, w+4, ...
// of a workgroup of 256), three chunks of loads in flight per wave
// (nontemporal: each point is read once). For each group a lane holds,
// fg(p0, xl, xh, y4) with p0 its first point and xl, xh the raw x of its
// points 0-1 and 2-3 (the positions when kHasX is false); after each chunk,
// fc(c) on every lane of the wave (uniform). The up to 3 points before the
// first group and after the last are left to the caller: returns a0 (the
// first group's first point) and sets *t0 (the point after the last group).
template <bool kHasX, class FG, class FC>
__device__ __forceinline__ int64_t scan_chunks(const int64_t *__restrict__ X, const float *__restrict__ Y, int64_t s,
                                               int64_t e, int64_t *t0, FG &&fg, FC &&fc)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const uint64_t ya = (uint64_t)(uintptr_t)(Y + s);
    int64_t a0 = s + (int64_t)(((16u - (unsigned)(ya & 15u)) & 15u) >> 2);
    a0 = a0 < e ? a0 : e;
    const int64_t nq = (e - a0) >> 2;
    *t0 = a0 + 4 * nq;
    const f32x4 *__restrict__ Y4 = reinterpret_cast<const f32x4 *>(Y + a0);
    const bool x16 = kHasX && ((((uint64_t)(uintptr_t)(X + a0)) & 15u) == 0);
    const f32x4 zy = {0.0f, 0.0f, 0.0f, 0.0f};
    const i64x2 zx = {0, 0};
    auto ly = [&](int64_t q) { return q < nq ? __builtin_nontemporal_load(Y4 + q) : zy; };
    auto lx = [&](int64_t q, int half) -> i64x2 {
        const int64_t p = a0 + 4 * q + 2 * half;
        if (q >= nq)
            return zx;
        if (!kHasX)
            return i64x2{p, p + 1};
        if (x16)
            return __builtin_nontemporal_load(reinterpret_cast<const i64x2 *>(X + p));
        return i64x2{__builtin_nontemporal_load(X + p), __builtin_nontemporal_load(X + p + 1)};
    };
    int64_t base = 64 * (int64_t)wid;
    f32x4 y0 = ly(base + lane), y1 = ly(base + 256 + lane);
    i64x2 a0l = lx(base + lane, 0), a0h = lx(base + lane, 1);
    i64x2 a1l = lx(base + 256 + lane, 0), a1h = lx(base + 256 + lane, 1);
    for (; base < nq; base += 256) {
        const int64_t q2 = base + 512 + lane;
        const f32x4 y2 = ly(q2);
        const i64x2 a2l = lx(q2, 0), a2h = lx(q2, 1);
        if (base + lane < nq)
            fg(a0 + 4 * (base + lane), a0l, a0h, y0);
        fc(base >> 6);
        y0 = y1;
        a0l = a1l;
        a0h = a1h;
        y1 = y2;
        a1l = a2l;
        a1h = a2h;
    }
    return a0;
}

template <int kDepth = 2, class F>
__device__ inline void scan_groups(const int64_t *__restrict__ X, const float *__restrict__ Y, int64_t s, int64_t e,
                                   int tid, int nthreads, F &&f)
{
    if (X)
        scan_groups_x<kDepth, true>(X, Y, s, e, tid, nthreads, f);
    else
        scan_groups_x<kDepth, false>(X, Y, s, e, tid, nthreads, f);
}

} // namespace mmlttb
