// Whole-series LTTB (section 2.2.1 LTTB; Fig. 3) for wide buckets, by
// transition tables instead of B dependent bucket scans.
//
// The pick in bucket k depends only on the pick a in bucket k-1: it is the
// point j of bucket k with the largest |(Xa - MX)(Yj - Ya) - (Xa - Xj)(MY - Ya)|
// (binary64, lowest position on ties). That value is the absolute value of a
// linear function of (Xj, Yj), so in exact arithmetic its maximum over the
// bucket lies on the bucket's convex hull, whatever a and the mean are.
//
//   k_lttb_hull    one workgroup per bucket k < B-1: the candidate picks of
//                  bucket k, the hull vertices (plus points close to a hull
//                  edge) at which a line with the slope of some line from a
//                  possible predecessor to the next-bucket mean touches the
//                  hull; at most kCandMax, or none (count -1) when the search
//                  overflows.
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

// Candidate search for bucket b (one workgroup of kHullThreads):
//  - the range [g0, g1] of slopes of the lines from the points that can
//    precede b's pick (bucket b-1, or point 0 for b = 0) to b's next-bucket
//    mean M_b, from the corners of the predecessors' bounding box, widened by
//    a margin: the pick is the point farthest from such a line, where a line
//    of that slope touches the bucket's hull (upper or lower chain);
//  - the points where lines of kSlopes slopes spread over [g0, g1] touch the
//    bucket from above and from below: every upper-hull vertex that a slope
//    between two neighbouring ones touches lies on or above the line through
//    their two tangent points (the chain is concave), every lower one on or
//    below the corresponding lower line;
//  - survivors: the points on the outer side of any of those lines, or within
//    a relative kSideTol of it, sorted by position (at most kSurvMax);
//  - the upper and lower monotone chains of the survivors (binary64, points
//    within a relative kChainTol of an edge kept);
//  - the chain vertices whose range of tangent slopes meets [g0, g1]: the
//    candidates.
// Every threshold only widens the candidate set; it stays an aid, never a
// part of the result.
constexpr int kHullThreads = 256;
constexpr int kSlopes = 6;     // slopes whose tangent points bound the survivors
constexpr int kSurvMax = 512; // survivors kept per bucket
constexpr int kChainMax = 128; // vertices per chain
constexpr double kSideTol = 1e-9;
constexpr double kChainTol = 1e-9;
// Candidates per table pass, and workgroups per bucket (each takes every
// kTabWGs-th group of candidates).
constexpr int kTabGroup = 4;
constexpr int kTabWGs = 2;
// The walk stages the first kWalkSlots entries of kWalkWindow buckets in LDS
// (entries past them, rare, are read from global memory).
constexpr int kWalkWindow = 128;
constexpr int kWalkSlots = 16;
constexpr int kWalkSeg = 16; // buckets per segment followed by one thread

__device__ inline double xval(const int64_t *__restrict__ X, int64_t p) { return X ? (double)X[p] : (double)p; }

// f(p, x, y) for p = first, first + step, ... < end, in increasing p, with the
// loads of kDepth points issued together (a scan with one load per step
// waits a full memory latency per step).
template <int kDepth, bool kHasX, class F>
__device__ inline void scan_points_x(const int64_t *__restrict__ X, const float *__restrict__ Y, int64_t first,
                                     int64_t end, int64_t step, F &&f)
{
    int64_t p = first;
    for (; p + (kDepth - 1) * step < end; p += kDepth * step) {
        double xs[kDepth];
        float ys[kDepth];
#pragma unroll
        for (int u = 0; u < kDepth; ++u) {
            xs[u] = kHasX ? (double)X[p + u * step] : (double)(p + u * step);
            ys[u] = Y[p + u * step];
        }
#pragma unroll
        for (int u = 0; u < kDepth; ++u)
            f(p + u * step, xs[u], (double)ys[u]);
    }
    for (; p < end; p += step)
        f(p, kHasX ? (double)X[p] : (double)p, (double)Y[p]);
}

template <int kDepth = 8, class F>
__device__ inline void scan_points(const int64_t *__restrict__ X, const float *__restrict__ Y, int64_t first,
                                   int64_t end, int64_t step, F &&f)
{
    if (X)
        scan_points_x<kDepth, true>(X, Y, first, end, step, f);
    else
        scan_points_x<kDepth, false>(X, Y, first, end, step, f);
}

// Orientation test of the monotone chain: true when b lies inside (below the
// segment a-p for the upper chain, above it for the lower one) by more than
// the tolerance.
__device__ inline bool chain_pop(double ax, double ay, double bx, double by, double px, double py, bool upper)
{
    const double t1 = (bx - ax) * (py - ay), t2 = (by - ay) * (px - ax);
    const double cr = t1 - t2, tol = kChainTol * (fabs(t1) + fabs(t2));
    return upper ? cr > tol : cr < -tol;
}

__global__ __launch_bounds__(kHullThreads) void k_lttb_hull(const int64_t *__restrict__ X, const float *__restrict__ Y,
                                                            int64_t n, int64_t B, const double *__restrict__ MX,
                                                            const double *__restrict__ MY,
                                                            const float2 *__restrict__ YR,
                                                            int32_t *__restrict__ cand_cnt, int32_t *__restrict__ cand)
{
    __shared__ double sx[kSurvMax], sy[kSurvMax], tx[kSurvMax], ty[kSurvMax];
    __shared__ int32_t si[kSurvMax], ti[kSurvMax];
    __shared__ double cxs[2][kChainMax], cys[2][kChainMax];
    __shared__ int32_t ci[2][kChainMax], ckeep[2][kChainMax];
    __shared__ int32_t cn[2], nsurv, ovf;
    __shared__ double tv[kHullThreads / kWave][2 * kSlopes], tpx[2 * kSlopes], tpy[2 * kSlopes];
    __shared__ int32_t to[kHullThreads / kWave][2 * kSlopes];
    const int tid = threadIdx.x;
    const int64_t b = blockIdx.x;
    const Split bk = make_split(n - 2, B);
    const int64_t s = 1 + split_lo(bk, b), e = 1 + split_lo(bk, b + 1);
    const int64_t ps = b == 0 ? 0 : 1 + split_lo(bk, b - 1), pe = b == 0 ? 1 : s;
    if (tid == 0) {
        nsurv = 0;
        ovf = 0;
    }
    const double inf = __longlong_as_double(0x7ff0000000000000ll);

    // slope range from the predecessors' bounding box (M_b lies right of it)
    const float2 pr = b == 0 ? make_float2(Y[0], Y[0]) : YR[b - 1];
    const double plo = (double)pr.x, phi = (double)pr.y;
    const double mxb = MX[b], myb = MY[b];
    const double dx0 = mxb - xval(X, ps), dx1 = mxb - xval(X, pe - 1); // both > 0
    const double c0 = (myb - phi) / dx0, c1 = (myb - phi) / dx1, c2 = (myb - plo) / dx0, c3 = (myb - plo) / dx1;
    double g0 = fmin(fmin(c0, c1), fmin(c2, c3)), g1 = fmax(fmax(c0, c1), fmax(c2, c3));
    const double pad = 1e-6 * (g1 - g0) + 1e-9 * (fabs(g0) + fabs(g1)) + 1e-300;
    g0 -= pad;
    g1 += pad;
    const bool wide = !(g1 - g0 < inf); // a slope the box cannot bound: keep every chain vertex

    // the bucket's y span sets the spacing of kSlopes slopes across [g0, g1]
    // (even in angle in the bucket's own scale)
    const double ylo = (double)YR[b].x, yhi = (double)YR[b].y;
    const double x0 = xval(X, s);
    double r = (xval(X, e - 1) - x0) / (yhi - ylo);
    r = (r > 0.0 && r < inf) ? r : 1.0;
    double gs[kSlopes];
    {
        const double t0 = atan(g0 * r), t1 = atan(g1 * r);
#pragma unroll
        for (int i = 0; i < kSlopes; ++i)
            gs[i] = i == 0 ? g0 : (i == kSlopes - 1 ? g1 : tan(t0 + (t1 - t0) * i / (kSlopes - 1)) / r);
    }

    // tangent points of those slopes, from above and from below
    double fmax_[kSlopes], fmin_[kSlopes];
    int32_t omax[kSlopes], omin[kSlopes];
#pragma unroll
    for (int i = 0; i < kSlopes; ++i) {
        fmax_[i] = -inf;
        fmin_[i] = inf;
        omax[i] = omin[i] = 0;
    }
    scan_points<4>(X, Y, s + tid, e, kHullThreads, [&](int64_t p, double xr, double y) {
        const double x = xr - x0;
        const int32_t o = (int32_t)(p - s);
#pragma unroll
        for (int i = 0; i < kSlopes; ++i) {
            const double f = y - gs[i] * x;
            if (f > fmax_[i]) {
                fmax_[i] = f;
                omax[i] = o;
            }
            if (f < fmin_[i]) {
                fmin_[i] = f;
                omin[i] = o;
            }
        }
    });
    {
        const int lane = tid & (kWave - 1), wid = tid / kWave;
#pragma unroll
        for (int i = 0; i < kSlopes; ++i) {
            const double vmax = wave_max_f64(fmax_[i]), vmin = -wave_max_f64(-fmin_[i]);
            const int64_t cmax = wave_min_i64(fmax_[i] == vmax ? omax[i] : INT64_MAX);
            const int64_t cmin = wave_min_i64(fmin_[i] == vmin ? omin[i] : INT64_MAX);
            if (lane == 0) {
                tv[wid][i] = vmax;
                tv[wid][kSlopes + i] = -vmin;
                to[wid][i] = (int32_t)cmax;
                to[wid][kSlopes + i] = (int32_t)cmin;
            }
        }
        __syncthreads();
        if (tid < 2 * kSlopes) { // tangent point tid: upper for tid < kSlopes, lower after
            double bv = tv[0][tid];
            int32_t bo = to[0][tid];
            for (int q = 1; q < kHullThreads / kWave; ++q) {
                if (tv[q][tid] > bv || (tv[q][tid] == bv && to[q][tid] < bo)) {
                    bv = tv[q][tid];
                    bo = to[q][tid];
                }
            }
            bo = (bo >= 0 && bo < e - s) ? bo : 0; // some thread holds the extreme: never past the bucket
            tpx[tid] = xval(X, s + bo) - x0;
            tpy[tid] = (double)Y[s + bo];
        }
        __syncthreads();
    }

    // survivors (appended in any order, then sorted by position): points on
    // the outer side of a chord between tangent points of neighbouring slopes.
    // Such a point also lies outside the chord between the outermost tangent
    // points (the arc between them is concave), which is tested first.
    auto side = [&](int i0, int i1, int gi, double sgn, double x, double y) {
        // > 0 outside the line through tangent points i0, i1 (slopes gs[gi], gs[gi + 1])
        const double ax = tpx[i0], ay = tpy[i0];
        double ex = tpx[i1] - ax, ey = tpy[i1] - ay;
        if (ex < 0.0) { // orient left to right
            ex = -ex;
            ey = -ey;
        }
        if (ex == 0.0 && ey == 0.0) { // one tangent point: the line of a slope between through it
            const double g = 0.5 * (gs[gi] + gs[gi + 1]);
            const double d = (y - ay) - g * (x - ax);
            return sgn * d >= -kSideTol * (fabs(y - ay) + fabs(g * (x - ax)));
        }
        const double t1 = ex * (y - ay), t2 = ey * (x - ax);
        return sgn * (t1 - t2) >= -kSideTol * (fabs(t1) + fabs(t2));
    };
    scan_points<4>(X, Y, s + tid, e, kHullThreads, [&](int64_t p, double xr, double y) {
        const double x = xr - x0;
        const bool up = side(0, kSlopes - 1, 0, 1.0, x, y), dn = side(kSlopes, 2 * kSlopes - 1, 0, -1.0, x, y);
        bool keep = wide;
        if (!keep && (up || dn)) {
            for (int i = 0; i + 1 < kSlopes; ++i)
                keep = keep || (up && side(i, i + 1, i, 1.0, x, y)) ||
                       (dn && side(kSlopes + i, kSlopes + i + 1, i, -1.0, x, y));
        }
        if (keep) {
            const int q = atomicAdd(&nsurv, 1);
            if (q < kSurvMax) {
                sx[q] = x;
                sy[q] = y;
                si[q] = (int32_t)(p - s);
            }
        }
    });
    __syncthreads();
    const int total = nsurv;
    const int ns = total < kSurvMax ? total : kSurvMax;
    for (int q = tid; q < ns; q += kHullThreads) { // rank sort by position (distinct)
        const int32_t me = si[q];
        int r = 0;
        for (int j = 0; j < ns; ++j)
            r += si[j] < me ? 1 : 0;
        tx[r] = sx[q];
        ty[r] = sy[q];
        ti[r] = me;
    }
    __syncthreads();

    // chains: thread 0 the upper, thread 1 the lower; then the slope filter
    if (tid < 2 && total <= kSurvMax) {
        const bool upper = tid == 0;
        int m = 0;
        for (int q = 0; q < ns; ++q) {
            const double x = tx[q], y = ty[q];
            while (m >= 2 && chain_pop(cxs[tid][m - 2], cys[tid][m - 2], cxs[tid][m - 1], cys[tid][m - 1], x, y, upper))
                --m;
            if (m < kChainMax) {
                cxs[tid][m] = x;
                cys[tid][m] = y;
                ci[tid][m] = ti[q];
                ++m;
            } else {
                ovf = 1;
            }
        }
        cn[tid] = m;
        // upper vertex i is touched by the slopes between its right and left
        // edge slopes, lower vertex i by those between its left and right ones
        for (int i = 0; i < m; ++i) {
            double left = upper ? inf : -inf, right = upper ? -inf : inf;
            if (i > 0 && cxs[tid][i] > cxs[tid][i - 1])
                left = (cys[tid][i] - cys[tid][i - 1]) / (cxs[tid][i] - cxs[tid][i - 1]);
            if (i + 1 < m && cxs[tid][i + 1] > cxs[tid][i])
                right = (cys[tid][i + 1] - cys[tid][i]) / (cxs[tid][i + 1] - cxs[tid][i]);
            const double lo = fmin(left, right), hi = fmax(left, right);
            ckeep[tid][i] = (wide || (hi >= g0 && lo <= g1)) ? 1 : 0;
        }
    }
    __syncthreads();

    if (tid == 0) {
        int32_t *out = cand + b * (int64_t)kCandMax;
        int a = 0, c = 0, m = 0;
        bool full = ovf != 0 || total > kSurvMax;
        auto next = [&](int h, int &i) { // next kept vertex of chain h at or after i
            while (i < cn[h] && !ckeep[h][i])
                ++i;
        };
        if (!full) {
            next(0, a);
            next(1, c);
        }
        while (!full && (a < cn[0] || c < cn[1])) {
            int32_t v;
            if (c >= cn[1] || (a < cn[0] && ci[0][a] <= ci[1][c])) {
                v = ci[0][a++];
                if (c < cn[1] && ci[1][c] == v)
                    ++c;
            } else {
                v = ci[1][c++];
            }
            if (m < kCandMax)
                out[m++] = v;
            else
                full = true;
            next(0, a);
            next(1, c);
        }
        cand_cnt[b] = full ? -1 : m;
    }
}

// Table entries c0 .. c0 + kTabGroup - 1 of bucket k (candidates of bucket
// k-1, or point 0 alone for k = 0) against every point [s, e) of bucket k.
// Each thread scans its points in increasing position with a strict
// comparison; the workgroup then keeps the largest area and the lowest
// position among equal ones; no area above -1 (every one NaN) leaves the
// bucket's first point, as in the sequential pass.
__device__ inline void table_group(const int64_t *__restrict__ X, const float *__restrict__ Y, int64_t k, int64_t B,
                                   int64_t s, int64_t e, int64_t sp, int c0, int nc, double mx, double my,
                                   const int32_t *__restrict__ cand_cnt, const int32_t *__restrict__ cand,
                                   int2 *__restrict__ tab, double (*s_best)[kTabGroup], int32_t (*s_idx)[kTabGroup])
{
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
    double xa[kTabGroup], ya[kTabGroup], best[kTabGroup];
    int32_t bi[kTabGroup];
#pragma unroll
    for (int c = 0; c < kTabGroup; ++c) {
        const int64_t a = k == 0 ? 0 : sp + cand[(k - 1) * (int64_t)kCandMax + c0 + (c < nc ? c : 0)];
        xa[c] = xval(X, a);
        ya[c] = (double)Y[a];
        best[c] = -1.0;
        bi[c] = 0x7fffffff;
    }
    scan_groups<2>(X, Y, s, e, tid, (int)blockDim.x, [&](int64_t p, int64_t xraw, float yraw) {
        const double xj = (double)xraw, yj = (double)yraw;
#pragma unroll
        for (int c = 0; c < kTabGroup; ++c) {
            const double ar = lttb_area2(xa[c], ya[c], xj, yj, mx, my);
            if (ar > best[c]) { // strict, positions increasing per thread: the lowest wins ties
                best[c] = ar;
                bi[c] = (int32_t)(p - s);
            }
        }
    });
#pragma unroll
    for (int c = 0; c < kTabGroup; ++c) {
        const double wb = wave_max_f64(best[c]);
        const int64_t wi = wave_min_i64(best[c] == wb ? bi[c] : 0x7fffffff);
        if (lane == 0) {
            s_best[wid][c] = wb;
            s_idx[wid][c] = (int32_t)wi;
        }
    }
    __syncthreads();
    if (tid < nc) {
        double bb = -1.0;
        int32_t off = 0x7fffffff;
        for (int w = 0; w < (int)(blockDim.x / kWave); ++w) {
            const double a = s_best[w][tid];
            const int32_t i = s_idx[w][tid];
            if (a > bb || (a == bb && i < off)) {
                bb = a;
                off = i;
            }
        }
        if (!(bb > -1.0)) // no numeric area: the bucket's first point
            off = 0;
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
    __syncthreads(); // s_best and s_idx are reused by the next group
}

// Workgroup (k, g) of kTableThreads: the candidate groups g, g + kTabWGs, ...
// of bucket k.
constexpr int kTableThreads = 256;
__global__ __launch_bounds__(kTableThreads) void k_lttb_tables(const int64_t *__restrict__ X,
                                                               const float *__restrict__ Y, int64_t n, int64_t B,
                                                               const double *__restrict__ MX,
                                                               const double *__restrict__ MY,
                                                               const int32_t *__restrict__ cand_cnt,
                                                               const int32_t *__restrict__ cand, int2 *__restrict__ tab)
{
    __shared__ double s_best[kTableThreads / kWave][kTabGroup];
    __shared__ int32_t s_idx[kTableThreads / kWave][kTabGroup];
    const int64_t k = blockIdx.x / kTabWGs;
    const int g = blockIdx.x % kTabWGs;
    const int ncand = k == 0 ? 1 : cand_cnt[k - 1];
    if (g * kTabGroup >= ncand) // also no candidates at all (-1)
        return;
    const Split bk = make_split(n - 2, B);
    const int64_t s = 1 + split_lo(bk, k), e = 1 + split_lo(bk, k + 1);
    const int64_t sp = k == 0 ? 0 : 1 + split_lo(bk, k - 1);
    const double mx = MX[k], my = MY[k];
    for (int c0 = g * kTabGroup; c0 < ncand; c0 += kTabWGs * kTabGroup) {
        const int nc = ncand - c0 < kTabGroup ? ncand - c0 : kTabGroup;
        table_group(X, Y, k, B, s, e, sp, c0, nc, mx, my, cand_cnt, cand, tab, s_best, s_idx);
    }
}

// One workgroup of 1024 threads. Windows of kWalkWindow buckets: their first
// kWalkSlots table entries are staged in LDS, every segment of kWalkSeg
// buckets is followed from every entry slot at once (one thread each), thread
// 0 links the segments from the true entry slot, and the picks of the window
// are written in parallel. The window ends early where a slot is -1 (the
// predecessor is not a candidate: the whole workgroup then scans that bucket
// for its pick) or past the staged entries (one step from global memory).
__global__ __launch_bounds__(1024) void k_lttb_table_walk(const int64_t *__restrict__ X, const float *__restrict__ Y,
                                                          int64_t n, int64_t B, const double *__restrict__ MX,
                                                          const double *__restrict__ MY,
                                                          const int32_t *__restrict__ cand_cnt,
                                                          const int32_t *__restrict__ cand,
                                                          const int2 *__restrict__ tab, int64_t *__restrict__ out)
{
    constexpr int kSegs = kWalkWindow / kWalkSeg;
    __shared__ int2 sT[kWalkWindow * kWalkSlots];
    __shared__ uint8_t spath[kSegs][kWalkSlots][kWalkSeg]; // slot used at each bucket of the segment
    __shared__ int32_t sdone[kSegs][kWalkSlots], sexit[kSegs][kWalkSlots], sent[kSegs];
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
        if (slot >= 0 && slot < kWalkSlots) {
            const int64_t k1 = k + kWalkWindow < B ? k + kWalkWindow : B;
            const int W = (int)(k1 - k), nseg = (W + kWalkSeg - 1) / kWalkSeg;
            for (int q = tid; q < W * kWalkSlots; q += blockDim.x)
                sT[q] = tab[(k + q / kWalkSlots) * kCandMax + q % kWalkSlots];
            __syncthreads();
            if (tid < nseg * kWalkSlots) { // segment g from entry slot e
                const int g = tid / kWalkSlots, e = tid % kWalkSlots;
                const int len = W - g * kWalkSeg < kWalkSeg ? W - g * kWalkSeg : kWalkSeg;
                int sl = e, i = 0;
                for (; i < len && sl >= 0 && sl < kWalkSlots; ++i) {
                    spath[g][e][i] = (uint8_t)sl;
                    sl = sT[(g * kWalkSeg + i) * kWalkSlots + sl].y;
                }
                sdone[g][e] = i; // steps taken from the tables
                sexit[g][e] = sl; // the slot after them
            }
            __syncthreads();
            if (tid == 0) {
                int cur = slot;
                int64_t stop = k1;
                for (int g = 0; g < nseg; ++g) {
                    sent[g] = cur;
                    const int len = W - g * kWalkSeg < kWalkSeg ? W - g * kWalkSeg : kWalkSeg;
                    const int done = sdone[g][cur];
                    cur = sexit[g][cur];
                    if (done < len) {
                        stop = k + g * kWalkSeg + done;
                        break;
                    }
                    if (cur < 0 || cur >= kWalkSlots) { // the next segment cannot start from the tables
                        stop = k + (int64_t)g * kWalkSeg + len; // <= k1: the last segment may be short
                        break;
                    }
                }
                s_k = stop;
                s_slot = cur;
            }
            __syncthreads();
            const int64_t stop = s_k; // k < stop <= k1 <= B
            for (int t = tid; t < (int)(stop - k); t += blockDim.x) { // the picks of buckets k .. stop-1
                const int g = t / kWalkSeg, i = t % kWalkSeg;
                const int sl = spath[g][sent[g]][i];
                const int64_t pick = 1 + split_lo(bk, k + t) + sT[t * kWalkSlots + sl].x;
                out[k + t + 1] = pick;
                if (k + t + 1 == stop)
                    s_a = pick;
            }
            __syncthreads();
            k = stop;
            a = s_a;
            slot = s_slot;
            __syncthreads();
            continue;
        }
        if (slot >= kWalkSlots) { // an entry past the staged ones: one step from global memory
            const int2 t = tab[k * kCandMax + slot];
            a = 1 + split_lo(bk, k) + t.x;
            if (tid == 0)
                out[k + 1] = a;
            slot = t.y;
            ++k;
            continue;
        }
        // slot -1: scan bucket k for the pick of a
        const int64_t s0 = 1 + split_lo(bk, k), s1 = 1 + split_lo(bk, k + 1);
        const double ax = xval(X, a), ay = (double)Y[a], mx = MX[k], my = MY[k];
        double best = -1.0;
        int64_t bj = INT64_MAX;
        scan_points(X, Y, s0 + tid, s1, blockDim.x, [&](int64_t j, double xj, double yj) {
            const double ar = lttb_area2(ax, ay, xj, yj, mx, my);
            if (ar > best) {
                best = ar;
                bj = j;
            }
        });
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

hipError_t launch_lttb_hull(const int64_t *X, const float *Y, int64_t n, int64_t B, const double *MX, const double *MY,
                            const float2 *YR, int32_t *cand_cnt, int32_t *cand, hipStream_t s)
{
    if (B < 2)
        return hipSuccess;
    hipLaunchKernelGGL(k_lttb_hull, dim3((unsigned)(B - 1)), dim3(kHullThreads), 0, s, X, Y, n, B, MX, MY, YR,
                       cand_cnt, cand);
    return hipGetLastError();
}

hipError_t launch_lttb_tables(const int64_t *X, const float *Y, int64_t n, int64_t B, const double *MX,
                              const double *MY, const int32_t *cand_cnt, const int32_t *cand, int2 *tab,
                              hipStream_t s)
{
    hipLaunchKernelGGL(k_lttb_tables, dim3((unsigned)(B * kTabWGs)), dim3(kTableThreads), 0, s, X, Y, n, B, MX,
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
