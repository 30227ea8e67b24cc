// Whole-series LTTB (section 2.2.1 LTTB; Fig. 3) for wide buckets, by
// transition tables instead of B dependent bucket scans.
//
// The pick in bucket k depends only on the pick a in bucket k-1: it is the
// point j of bucket k with the largest |(Xa - MX)(Yj - Ya) - (Xa - Xj)(MY - Ya)|
// (binary64, lowest position on ties). That value is the absolute value of a
// linear function of (Xj, Yj), so in exact arithmetic its maximum over the
// bucket lies on the bucket's convex hull, whatever a and the mean are.
//
//   k_lttb_hull    one wave per bucket k < B-1: the candidate picks of bucket
//                  k, the vertices of its upper and lower hull plus points
//                  close to a hull edge (a relative tolerance far above
//                  rounding), at most kCandMax of them, or none (count -1)
//                  when the hull is larger.
//   k_lttb_tables  for every candidate a of bucket k-1 (point 0 for k = 0):
//                  the pick in bucket k, evaluated over every point of bucket
//                  k with the exact definition above, and the slot of that
//                  pick among bucket k's candidates (-1 if it is not one).
//   k_lttb_table_walk  one workgroup follows the tables from point 0. Where a
//                  pick is not a candidate of its bucket (a rounding near-tie
//                  off the hull, or a bucket without candidates), the next
//                  bucket is scanned in full for that pick instead.
//
// Candidates only decide which work is tabulated: every pick the walk emits is
// either a table entry (the exact argmax for its exact predecessor) or a full
// scan, so the result equals the sequential pass whatever the hulls hold.
#include "chain_device.hpp"
#include "device_common.hpp"
#include "kernels.hpp"

namespace mmlttb {

// Chunk-hull vertices each lane keeps per chain (upper, lower).
constexpr int kHullLane = 24;
// A point stays on a chain unless it lies inside by more than this fraction
// of the terms of the orientation test (float coordinates relative to the
// bucket's first point): near-collinear points remain candidates.
constexpr float kHullTol = 1e-4f;
// Candidates per table workgroup.
constexpr int kTabGroup = 8;
// Buckets of tables staged in LDS per window of the walk.
constexpr int kWalkWindow = 32;

__device__ inline double xval(const int64_t *__restrict__ X, int64_t p) { return X ? (double)X[p] : (double)p; }

// Orientation test of the monotone chain: true when b lies clearly inside
// (below the segment a-p for the upper chain, above it for the lower one).
__device__ inline bool hull_pop(float ax, float ay, float bx, float by, float px, float py, bool upper)
{
    const float t1 = (bx - ax) * (py - ay), t2 = (by - ay) * (px - ax);
    const float cr = t1 - t2, tol = kHullTol * (fabsf(t1) + fabsf(t2));
    return upper ? cr > tol : cr < -tol;
}

// One wave per bucket k in [0, B - 1). Phase 1: lane l builds both chains of
// its contiguous chunk of the bucket (LDS, kHullLane points each, indexed
// [i * kWave + lane]). Phase 2: lane 0 (upper) and lane 1 (lower) run the
// chain again over the chunk chains in lane order, which is position order.
// Lane 0 then merges both into cand[k * kCandMax ..] (offsets inside the
// bucket, increasing) and writes their count, or -1 on any overflow.
__global__ __launch_bounds__(kWave) void k_lttb_hull(const int64_t *__restrict__ X, const float *__restrict__ Y,
                                                     int64_t n, int64_t B, int32_t *__restrict__ cand_cnt,
                                                     int32_t *__restrict__ cand)
{
    __shared__ float hx[2][kHullLane * kWave], hy[2][kHullLane * kWave];
    __shared__ int32_t hi[2][kHullLane * kWave];
    __shared__ int32_t hn[2][kWave];
    __shared__ float mx_[2][kCandMax], my_[2][kCandMax];
    __shared__ int32_t mi[2][kCandMax];
    __shared__ int32_t mn[2];
    __shared__ int32_t ovf;
    const int lane = threadIdx.x;
    const int64_t k = blockIdx.x;
    const Split bk = make_split(n - 2, B);
    const int64_t s = 1 + split_lo(bk, k), e = 1 + split_lo(bk, k + 1);
    const double x0 = xval(X, s);
    const float y0 = Y[s];
    if (lane == 0)
        ovf = 0;
    __syncthreads();

    const int64_t c = (e - s + kWave - 1) / kWave;
    const int64_t p0 = s + lane * c < e ? s + lane * c : e;
    const int64_t p1 = p0 + c < e ? p0 + c : e;
    int cnt[2] = {0, 0};
    bool bad = false;
    constexpr int kRun = 16; // points read ahead per lane
    for (int64_t q = p0; q < p1; q += kRun) {
        float px[kRun], py[kRun];
#pragma unroll
        for (int u = 0; u < kRun; ++u) {
            const int64_t p = q + u < p1 ? q + u : p1 - 1;
            px[u] = (float)(xval(X, p) - x0);
            py[u] = Y[p] - y0;
        }
#pragma unroll
        for (int u = 0; u < kRun; ++u) {
            if (q + u >= p1)
                break;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                int m = cnt[h];
                while (m >= 2 && hull_pop(hx[h][(m - 2) * kWave + lane], hy[h][(m - 2) * kWave + lane],
                                          hx[h][(m - 1) * kWave + lane], hy[h][(m - 1) * kWave + lane], px[u], py[u],
                                          h == 0))
                    --m;
                if (m < kHullLane) {
                    hx[h][m * kWave + lane] = px[u];
                    hy[h][m * kWave + lane] = py[u];
                    hi[h][m * kWave + lane] = (int32_t)(q + u - s);
                    ++m;
                } else {
                    bad = true;
                }
                cnt[h] = m;
            }
        }
    }
    hn[0][lane] = cnt[0];
    hn[1][lane] = cnt[1];
    if (bad)
        ovf = 1;
    __syncthreads();

    if (lane < 2) {
        const int h = lane;
        int m = 0;
        for (int l = 0; l < kWave; ++l) {
            for (int i = 0; i < hn[h][l]; ++i) {
                const float px = hx[h][i * kWave + l], py = hy[h][i * kWave + l];
                while (m >= 2 && hull_pop(mx_[h][m - 2], my_[h][m - 2], mx_[h][m - 1], my_[h][m - 1], px, py, h == 0))
                    --m;
                if (m < kCandMax) {
                    mx_[h][m] = px;
                    my_[h][m] = py;
                    mi[h][m] = hi[h][i * kWave + l];
                    ++m;
                } else {
                    ovf = 1;
                }
            }
        }
        mn[h] = m;
    }
    __syncthreads();

    if (lane == 0) {
        int32_t *out = cand + k * (int64_t)kCandMax;
        int a = 0, b = 0, m = 0;
        bool full = ovf != 0;
        while (!full && (a < mn[0] || b < mn[1])) {
            int32_t v;
            if (b >= mn[1] || (a < mn[0] && mi[0][a] <= mi[1][b])) {
                v = mi[0][a++];
                if (b < mn[1] && mi[1][b] == v)
                    ++b;
            } else {
                v = mi[1][b++];
            }
            if (m < kCandMax)
                out[m++] = v;
            else
                full = true;
        }
        cand_cnt[k] = full ? -1 : m;
    }
}

// Workgroup (k, g): candidates g*kTabGroup .. of bucket k-1 (point 0 alone
// for k = 0) against every point of bucket k. Each thread scans its points in
// increasing position with a strict comparison; the workgroup then keeps the
// largest area and the lowest position among equal ones; no area above -1
// (every one NaN) leaves the bucket's first point, as in the sequential pass.
__global__ __launch_bounds__(256) void k_lttb_tables(const int64_t *__restrict__ X, const float *__restrict__ Y,
                                                     int64_t n, int64_t B, const double *__restrict__ MX,
                                                     const double *__restrict__ MY,
                                                     const int32_t *__restrict__ cand_cnt,
                                                     const int32_t *__restrict__ cand, int2 *__restrict__ tab)
{
    __shared__ double s_best[4][kTabGroup];
    __shared__ int64_t s_idx[4][kTabGroup];
    constexpr int kGroups = kCandMax / kTabGroup;
    const int64_t k = blockIdx.x / kGroups;
    const int g = blockIdx.x % kGroups;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
    const int ncand = k == 0 ? 1 : cand_cnt[k - 1];
    const int c0 = g * kTabGroup;
    if (c0 >= ncand) // also no candidates at all (-1)
        return;
    const int nc = ncand - c0 < kTabGroup ? ncand - c0 : kTabGroup;
    const Split bk = make_split(n - 2, B);
    const int64_t s = 1 + split_lo(bk, k), e = 1 + split_lo(bk, k + 1);
    const int64_t sp = k == 0 ? 0 : 1 + split_lo(bk, k - 1);
    const double mx = MX[k], my = MY[k];
    double xa[kTabGroup], ya[kTabGroup], best[kTabGroup];
    int64_t bi[kTabGroup];
#pragma unroll
    for (int c = 0; c < kTabGroup; ++c) {
        const int64_t a = k == 0 ? 0 : sp + cand[(k - 1) * (int64_t)kCandMax + c0 + (c < nc ? c : 0)];
        xa[c] = xval(X, a);
        ya[c] = (double)Y[a];
        best[c] = -1.0;
        bi[c] = INT64_MAX;
    }
    for (int64_t j = s + tid; j < e; j += blockDim.x) {
        const double xj = xval(X, j), yj = (double)Y[j];
#pragma unroll
        for (int c = 0; c < kTabGroup; ++c) {
            const double ar = lttb_area2(xa[c], ya[c], xj, yj, mx, my);
            if (ar > best[c]) {
                best[c] = ar;
                bi[c] = j;
            }
        }
    }
#pragma unroll
    for (int c = 0; c < kTabGroup; ++c) {
        const double wb = wave_max_f64(best[c]);
        const int64_t wi = wave_min_i64(best[c] == wb ? bi[c] : INT64_MAX);
        if (lane == 0) {
            s_best[wid][c] = wb;
            s_idx[wid][c] = wi;
        }
    }
    __syncthreads();
    if (tid < nc) {
        double b = -1.0;
        int64_t p = INT64_MAX;
        for (int w = 0; w < 4; ++w) {
            const double a = s_best[w][tid];
            const int64_t i = s_idx[w][tid];
            if (a > b || (a == b && i < p)) {
                b = a;
                p = i;
            }
        }
        if (!(b > -1.0)) // no numeric area: the bucket's first point
            p = s;
        const int32_t off = (int32_t)(p - s);
        int32_t next = -1;
        const int nk = k + 1 < B ? cand_cnt[k] : -1;
        if (nk > 0) {
            const int32_t *ck = cand + k * (int64_t)kCandMax;
            int lo = 0, hi = nk;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (ck[mid] < off)
                    lo = mid + 1;
                else
                    hi = mid;
            }
            next = (lo < nk && ck[lo] == off) ? lo : -1;
        }
        tab[k * (int64_t)kCandMax + c0 + tid] = make_int2(off, next);
    }
}

// One workgroup of 1024 threads. Thread 0 follows the tables through LDS
// windows of kWalkWindow buckets; where the slot is -1 the whole workgroup
// scans that bucket for the pick of the known predecessor.
__global__ __launch_bounds__(1024) void k_lttb_table_walk(const int64_t *__restrict__ X, const float *__restrict__ Y,
                                                          int64_t n, int64_t B, const double *__restrict__ MX,
                                                          const double *__restrict__ MY,
                                                          const int32_t *__restrict__ cand_cnt,
                                                          const int32_t *__restrict__ cand,
                                                          const int2 *__restrict__ tab, int64_t *__restrict__ out)
{
    __shared__ int2 sT[kWalkWindow * kCandMax];
    __shared__ double s_area[16];
    __shared__ int64_t s_idx[16];
    __shared__ int64_t s_k, s_a;
    __shared__ int32_t s_slot;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
    const int nw = blockDim.x / kWave;
    const Split bk = make_split(n - 2, B);
    int64_t k = 0, a = 0; // next bucket to pick in, previous pick (a position)
    int32_t slot = 0;     // a's slot among the candidates of bucket k-1 (point 0 for k = 0)
    while (k < B) {
        if (slot >= 0) {
            const int64_t k1 = k + kWalkWindow < B ? k + kWalkWindow : B;
            const int64_t words = (k1 - k) * kCandMax;
            for (int64_t q = tid; q < words; q += blockDim.x)
                sT[q] = tab[k * kCandMax + q];
            __syncthreads();
            if (tid == 0) {
                SplitWalker w;
                w.init(bk, k);
                int64_t kk = k;
                int32_t sl = slot;
                while (kk < k1 && sl >= 0) {
                    const int2 t = sT[(kk - k) * kCandMax + sl];
                    a = 1 + w.lo + t.x;
                    out[kk + 1] = a;
                    sl = t.y;
                    w.advance(bk);
                    ++kk;
                }
                s_k = kk;
                s_a = a;
                s_slot = sl;
            }
            __syncthreads();
            k = s_k;
            a = s_a;
            slot = s_slot;
            __syncthreads();
            continue;
        }
        // slot -1: scan bucket k for the pick of a
        const int64_t s0 = 1 + split_lo(bk, k), s1 = 1 + split_lo(bk, k + 1);
        const double ax = xval(X, a), ay = (double)Y[a], mx = MX[k], my = MY[k];
        double best = -1.0;
        int64_t bj = INT64_MAX;
        for (int64_t j = s0 + tid; j < s1; j += blockDim.x) {
            const double ar = lttb_area2(ax, ay, xval(X, j), (double)Y[j], mx, my);
            if (ar > best) {
                best = ar;
                bj = j;
            }
        }
        const double wb = wave_max_f64(best);
        const int64_t wsel = wave_min_i64(best == wb ? bj : INT64_MAX);
        if (lane == 0) {
            s_area[wid] = wb;
            s_idx[wid] = wsel;
        }
        __syncthreads();
        if (tid == 0) {
            double ba = -1.0;
            int64_t bi = INT64_MAX;
            for (int q = 0; q < nw; ++q) {
                if (s_area[q] > ba || (s_area[q] == ba && s_idx[q] < bi)) {
                    ba = s_area[q];
                    bi = s_idx[q];
                }
            }
            if (!(ba > -1.0))
                bi = s0;
            out[k + 1] = bi;
            int32_t sl = -1;
            const int nk = k + 1 < B ? cand_cnt[k] : -1;
            const int32_t *ck = cand + k * (int64_t)kCandMax;
            for (int i = 0; i < nk; ++i)
                if (ck[i] == (int32_t)(bi - s0))
                    sl = i;
            s_a = bi;
            s_slot = sl;
        }
        __syncthreads();
        a = s_a;
        slot = s_slot;
        ++k;
        __syncthreads();
    }
    if (tid == 0) {
        out[0] = 0;
        out[B + 1] = n - 1;
    }
}

hipError_t launch_lttb_hull(const int64_t *X, const float *Y, int64_t n, int64_t B, int32_t *cand_cnt, int32_t *cand,
                            hipStream_t s)
{
    if (B < 2)
        return hipSuccess;
    hipLaunchKernelGGL(k_lttb_hull, dim3((unsigned)(B - 1)), dim3(kWave), 0, s, X, Y, n, B, cand_cnt, cand);
    return hipGetLastError();
}

hipError_t launch_lttb_tables(const int64_t *X, const float *Y, int64_t n, int64_t B, const double *MX,
                              const double *MY, const int32_t *cand_cnt, const int32_t *cand, int2 *tab,
                              hipStream_t s)
{
    hipLaunchKernelGGL(k_lttb_tables, dim3((unsigned)(B * (kCandMax / kTabGroup))), dim3(256), 0, s, X, Y, n, B, MX,
                       MY, cand_cnt, cand, tab);
    return hipGetLastError();
}

hipError_t launch_lttb_table_walk(const int64_t *X, const float *Y, int64_t n, int64_t B, const double *MX,
                                  const double *MY, const int32_t *cand_cnt, const int32_t *cand, const int2 *tab,
                                  int64_t *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_lttb_table_walk, dim3(1), dim3(1024), 0, s, X, Y, n, B, MX, MY, cand_cnt, cand, tab, out);
    return hipGetLastError();
}

} // namespace mmlttb
