// Whole-series LTTB (section 2.2.1 LTTB; Fig. 3) for wide buckets, by
// transition tables instead of B dependent bucket scans, in two passes over
// the points.
//
// The pick in bucket k depends only on the pick a in bucket k-1: it is the
// point j of bucket k with the largest |(Xa - MX)(Yj - Ya) - (Xa - Xj)(MY - Ya)|
// (binary64, lowest position on ties). Written with s = (MY - Ya) / (MX - Xa),
// the slope from a to the next-bucket mean, that value is
// |Xa - MX| * |Ls(j) - Ls(a)| with Ls(p) = Yp - s * Xp: the bucket's largest
// and smallest Ls decide it, and both lie on the bucket's convex hull.
//
//   k_lttb_scan    one workgroup per bucket, one read of its points: the
//                  exact sums of the next-bucket mean, the bucket's y range,
//                  and for each of kSlabs slabs of consecutive points its
//                  highest and its lowest point (wave reductions merged in
//                  LDS); any points of the bucket would serve, these only make
//                  the next pass cheap.
//   k_lttb_hull    one workgroup per bucket: the slopes s of its possible
//                  predecessors (the bucket before, by its bounding box) lie
//                  in [g0, g1]; an upper arc through the slab highs and a
//                  lower one through the slab lows, from the hull's touching
//                  point for one end slope to that of the other, continued by
//                  lines of those slopes. A point that lies, by more than
//                  2 delta, below the upper arc (and its end lines) and above
//                  the lower one can be neither the largest nor the smallest
//                  Ls for any s in [g0, g1]. A slab whose highest point lies
//                  that far below the upper arc's least value over the slab's
//                  x range, and its lowest that far above the lower arc's
//                  greatest, holds no other point either and is not read
//                  again; the points of the other slabs (the few near the
//                  arcs) that fail the test (survivors) go through two
//                  monotone chains that drop only points more than 2 delta
//                  inside a segment between two points; what stays are the
//                  candidates. Every test adds a bound of its own rounding
//                  error (a float32 test first, binary64 where it cannot
//                  decide), so "more than 2 delta" is exact; delta = 2^-30
//                  times the bucket's y span.
//   k_lttb_tables  for every candidate a of bucket k-1 (point 0 for k = 0):
//                  the largest area over bucket k's candidates. A point that
//                  is not a candidate has, in exact arithmetic, an area at
//                  least 2 delta |Xa - MX| below the largest one, and every
//                  binary64 area is within E = 2^-49 (|Xa - MX| max|Yj - Ya| +
//                  max|Xa - Xj| |MY - Ya|) of the exact one; when s lies in
//                  [lo, hi] and delta |Xa - MX| > E the candidates' pick is the
//                  pick over the whole bucket, ties included. Otherwise the
//                  entry scans the bucket in full.
//   k_lttb_table_walk  one workgroup follows the tables from point 0. Where a
//                  pick is not a candidate of its bucket (a bucket whose
//                  candidates overflowed), the next bucket is scanned in full
//                  for that pick instead.
//
// Every pick the walk emits is thus either a certified table entry, a full
// scan or a table entry computed by a full scan: the result equals the
// sequential pass whatever the candidates hold.
#include "chain_device.hpp"
#include "device_common.hpp"
#include "kernels.hpp"

namespace mmlttb {

constexpr int kHullThreads = 256;
constexpr int kSurvMax = 128;  // survivors kept per bucket
constexpr int kChainMax = 64; // vertices per chain
// Slabs per bucket in the first pass: runs of 256 points (one wave's group
// of 16-byte loads), merged evenly when a bucket holds more.
constexpr int kSlabs = kSlabsHost;
// Bound on the relative rounding error of the few binary64 operations behind
// each test and area (at most 4 roundings: 4 * 2^-53 / (1 - 4 * 2^-53) < 2^-49).
constexpr double kErr = 0x1p-49;
// Candidates per full-scan group of the table pass.
constexpr int kTabGroup = 4;
// The walk stages, for the first kWalkSlots entries of up to kWalkWindow
// buckets, the slot each leads to (entries past them, rare, are read from
// global memory); segments of kWalkSeg buckets are followed from every entry
// slot, then groups of kWalkGroup segments.
constexpr int kWalkWindow = 2048;
constexpr int kWalkSlots = 16;
constexpr int kWalkSeg = 16;
constexpr int kWalkGroup = 16;
constexpr uint8_t kWalkOut = 0xff; // a slot outside [0, kWalkSlots)

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

// ------------------------------------------------------------------ pass 1

// Packed keys of a point at offset o of its bucket (o < 2^32): the largest
// key is the highest y (lowest offset on ties), the smallest the lowest y.
__device__ inline unsigned long long high_key(float y, uint32_t o)
{
    return ((unsigned long long)f32_order_key(y) << 32) | (0xffffffffu - o);
}
__device__ inline unsigned long long low_key(float y, uint32_t o)
{
    return ((unsigned long long)f32_order_key(y) << 32) | o;
}

// Per-lane sum of float32 values in binary64, exact while the nonzero values
// span few enough binades: a float32 is mant * 2^(sc - 149) with mant < 2^24
// and sc = max(E, 1) - 1 (E its biased exponent); if the nonzero values have
// sc in [smin, smax], every partial sum of cnt of them is a multiple of
// 2^(smin - 149) below cnt * 2^(smax - 149 + 24), so it needs no rounding when
// (smax - smin) + 24 + bits(cnt) <= 53.
struct LaneF64Sum {
    double acc = 0.0;
    float amax = 0.0f, amin = __int_as_float(0x7f800000); // largest |y|, smallest nonzero |y|
    int cnt = 0;
    __device__ void add(float y)
    {
        acc += (double)y;
        const float a = fabsf(y);
        amax = fmaxf(amax, a);
        amin = fminf(amin, a > 0.0f ? a : amin);
        ++cnt;
    }
    // sc = max(E, 1) - 1 grows with |y|, so the largest and the smallest
    // nonzero |y| give the span of sc over the nonzero values
    __device__ bool exact() const
    {
        if (!(amax > 0.0f))
            return amax == 0.0f; // every value zero (NaN: not exact)
        auto sc = [](float a) {
            const int e = (int)((__float_as_uint(a) >> 23) & 0xffu);
            return e ? e - 1 : 0;
        };
        return (sc(amax) - sc(amin)) + 24 + (32 - __clz(cnt | 1)) <= 53;
    }
};

__device__ inline float f32_from_order_key(uint32_t k)
{
    return __uint_as_float((k & 0x80000000u) ? (k & 0x7fffffffu) : ~k);
}

// Workgroup k < B-1 reads bucket k+1 (whose points make bucket k's mean);
// workgroup B-1 sets the last bucket's mean (the last point) and reads bucket
// 0. Each records the slab highs and lows of the bucket it reads (keys; 0 and
// ~0 for an empty slab) and its y range (from them).
template <bool kHasX>
__device__ inline void lttb_scan_body(const int64_t *__restrict__ X, const float *__restrict__ Y, int64_t n, int64_t B,
                                      double *__restrict__ MX, double *__restrict__ MY, float2 *__restrict__ YR,
                                      unsigned long long *__restrict__ slab_hi, unsigned long long *__restrict__ slab_lo)
{
    __shared__ BlockMeanLds sm;
    __shared__ unsigned long long s_up[kSlabs], s_dn[kSlabs];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const float kInf = __int_as_float(0x7f800000);
    const Split bk = make_split(n - 2, B);
    const int64_t k = blockIdx.x;
    const bool last = k == B - 1;
    const int64_t b = last ? 0 : k + 1;
    const int64_t s = 1 + split_lo(bk, b), e = 1 + split_lo(bk, b + 1);
    for (int i = tid; i < kSlabs; i += blockDim.x) {
        s_up[i] = 0ull;
        s_dn[i] = ~0ull;
    }
    __syncthreads();
    I64ExactSum sx;
    F32ExactSum sy;
    LaneF64Sum fy;
    sx.clear();
    sy.clear();
    // groups of 4 points at a 16-byte boundary of Y, a chunk of 64 groups per
    // wave at a time; the up to 3 points before the first group join slab 0,
    // the up to 3 after the last the last slab
    const uint64_t ya = (uint64_t)(uintptr_t)(Y + s);
    int64_t a0 = s + (int64_t)(((16u - (unsigned)(ya & 15u)) & 15u) >> 2);
    a0 = a0 < e ? a0 : e;
    const int64_t nq = (e - a0) >> 2, nchunks = (nq + 63) >> 6;
    // slabs: a chunk each, merged evenly when there are more than kSlabs;
    // with at most kSlabs / 4 chunks, a 64-point row (16 lanes) of a chunk each
    const bool fine = nchunks * 4 <= kSlabs;
    auto slab_of = [&](int64_t c) { return (int)(nchunks <= kSlabs ? c : (c * kSlabs) / nchunks); };
    float vmax = -kInf, vmin = kInf;
    uint32_t omax = 0, omin = 0;
    auto take = [&](int64_t p, int64_t x, float y) {
        sx.add(x);
        fy.add(y);
        const uint32_t o = (uint32_t)(p - s);
        if (y > vmax) { // strict: the lowest offset of the lane keeps a tie
            vmax = y;
            omax = o;
        }
        if (y < vmin) {
            vmin = y;
            omin = o;
        }
    };
    // this lane's high and low as keys into slab sl, then a fresh start
    auto flush = [&](bool wave, int sl) {
        unsigned long long ku = vmax > -kInf ? high_key(vmax, omax) : 0ull;
        unsigned long long kd = vmin < kInf ? low_key(vmin, omin) : ~0ull;
        if (wave)
            wave_minmax_u64(kd, ku);
        if (!wave || lane == 0) {
            atomicMax(&s_up[sl], ku);
            atomicMin(&s_dn[sl], kd);
        }
        vmax = -kInf;
        vmin = kInf;
    };
    int64_t t0;
    scan_chunks<kHasX>(
        X, Y, s, e, &t0,
        [&](int64_t p0, i64x2 xl, i64x2 xh, f32x4 yv) {
            take(p0, xl.x, yv.x);
            take(p0 + 1, xl.y, yv.y);
            take(p0 + 2, xh.x, yv.z);
            take(p0 + 3, xh.y, yv.w);
        },
        [&](int64_t c) {
            if (!fine) {
                flush(true, slab_of(c));
                return;
            }
            unsigned long long ku = vmax > -kInf ? high_key(vmax, omax) : 0ull;
            unsigned long long kd = vmin < kInf ? low_key(vmin, omin) : ~0ull;
            group_minmax(16, kd, ku); // each 16-lane row: one slab
            if ((lane & 15) == 0) {
                atomicMax(&s_up[4 * c + (lane >> 4)], ku);
                atomicMin(&s_dn[4 * c + (lane >> 4)], kd);
            }
            vmax = -kInf;
            vmin = kInf;
        });
    if (fy.exact()) {
        sy.add_exact_f64(fy.acc);
    } else { // values too far apart in scale: this lane's groups again, exactly
        const f32x4 *__restrict__ Y4 = reinterpret_cast<const f32x4 *>(Y + a0);
        for (int64_t q = 64 * (int64_t)wid + lane; q < nq; q += 256) {
            const f32x4 yv = Y4[q];
            sy.add(yv.x);
            sy.add(yv.y);
            sy.add(yv.z);
            sy.add(yv.w);
        }
    }
    const bool head = tid < 3 && s + tid < a0, tail = tid >= 64 && tid < 67 && t0 + (tid - 64) < e;
    if (head || tail) { // edge points: threads 0-2 before the groups, 64-66 after them
        const int64_t p = head ? s + tid : t0 + (tid - 64);
        const float y = Y[p];
        sx.add(kHasX ? X[p] : p);
        sy.add(y);
        const uint32_t o = (uint32_t)(p - s);
        if (y > vmax) {
            vmax = y;
            omax = o;
        }
        if (y < vmin) {
            vmin = y;
            omin = o;
        }
        flush(false, head || nchunks == 0 ? 0 : (fine ? (int)((nq - 1) >> 4) : slab_of(nchunks - 1)));
    }
    __syncthreads();
    for (int i = tid; i < kSlabs; i += blockDim.x) {
        slab_hi[b * kSlabs + i] = s_up[i];
        slab_lo[b * kSlabs + i] = s_dn[i];
    }
    if (wid == 0) { // the y range from the slabs (wave 0)
        unsigned long long hmax = 0ull, lmin = ~0ull;
        for (int i = lane; i < kSlabs; i += 64) {
            hmax = s_up[i] > hmax ? s_up[i] : hmax;
            lmin = s_dn[i] < lmin ? s_dn[i] : lmin;
        }
        wave_minmax_u64(lmin, hmax);
        if (lane == 0)
            YR[b] = make_float2(lmin == ~0ull ? kInf : f32_from_order_key((uint32_t)(lmin >> 32)),
                                hmax == 0ull ? -kInf : f32_from_order_key((uint32_t)(hmax >> 32)));
    }
    if (!last) {
        block_store_mean(sx, sy, e - s, sm, &MX[k], &MY[k]);
    } else if (tid == 0) { // the last bucket's mean is the last point
        MX[k] = (double)(kHasX ? X[n - 1] : n - 1);
        MY[k] = (double)Y[n - 1];
    }
}

__global__ __launch_bounds__(256) void k_lttb_scan(const int64_t *__restrict__ X, const float *__restrict__ Y, int64_t n,
                                                   int64_t B, double *__restrict__ MX, double *__restrict__ MY,
                                                   float2 *__restrict__ YR, unsigned long long *__restrict__ slab_hi,
                                                   unsigned long long *__restrict__ slab_lo)
{
    if (X)
        lttb_scan_body<true>(X, Y, n, B, MX, MY, YR, slab_hi, slab_lo);
    else
        lttb_scan_body<false>(X, Y, n, B, MX, MY, YR, slab_hi, slab_lo);
}

// ------------------------------------------------------------------ pass 2

// One side's arc: vertices (x relative to the bucket's first point, y) in
// increasing x, the float32 slopes of its edges, and the slopes of the lines
// that stand for it left of its first and right of its last vertex.
constexpr int kArcSlopes = 12; // touching points that make an arc
constexpr int kScanU = 8;     // points in flight per thread in the survivor scan
struct Arc {
    double x[kArcSlopes], y[kArcSlopes];
    float xf[kArcSlopes], yf[kArcSlopes], sf[kArcSlopes];
    double gl, gr;
    float glf, grf;
    int n;
};

// Vertical depth of (x, y) inside the line through vertex i with slope g
// (float32 pre-test, then binary64): true when it is certainly more than
// 2 delta below (sign = +1) or above (sign = -1) that line.
__device__ __forceinline__ bool line_inside(const Arc &A, int i, double g, float gf, double sign, double delta,
                                            float d2f, double x, double y, float xf, float yf)
{
    const float dxf = xf - A.xf[i], u = yf - A.yf[i], t = gf * dxf, df = u - t;
    const float tol = 0x1p-18f * (fabsf(u) + fabsf(t) + fabsf(df) + fabsf(gf) * (fabsf(xf) + fabsf(A.xf[i]) + fabsf(dxf)));
    if ((float)sign * df < -(tol + d2f))
        return true;
    const double dy = y - A.y[i], dt = g * (x - A.x[i]);
    const double d = sign * (dy - dt);
    return d + kErr * (fabs(dy) + fabs(dt)) < -2.0 * delta;
}

// The same for the chord between vertices i and i+1.
__device__ __forceinline__ bool chord_inside(const Arc &A, int i, double sign, double delta, float d2f, double x,
                                             double y, float xf, float yf)
{
    const float dxf = xf - A.xf[i], u = yf - A.yf[i], t = A.sf[i] * dxf, df = u - t;
    const float tol =
        0x1p-18f * (fabsf(u) + fabsf(t) + fabsf(df) + fabsf(A.sf[i]) * (fabsf(xf) + fabsf(A.xf[i]) + fabsf(dxf)));
    if ((float)sign * df < -(tol + d2f))
        return true;
    const double ex = A.x[i + 1] - A.x[i], ey = A.y[i + 1] - A.y[i];
    const double t1 = ex * (y - A.y[i]), t2 = ey * (x - A.x[i]);
    const double cr = sign * (t1 - t2);
    return cr + kErr * (fabs(t1) + fabs(t2)) < -2.0 * delta * ex;
}

// Whether (x, y) is certainly inside the arc (and its end lines) by more
// than 2 delta; `it` follows the chord under x for points of increasing x.
__device__ __forceinline__ bool arc_inside(const Arc &A, double sign, double delta, float d2f, double x, double y,
                                           float xf, float yf, int &it)
{
    if (A.n < 1)
        return false;
    if (x < A.x[0])
        return line_inside(A, 0, A.gl, A.glf, sign, delta, d2f, x, y, xf, yf);
    if (x > A.x[A.n - 1])
        return line_inside(A, A.n - 1, A.gr, A.grf, sign, delta, d2f, x, y, xf, yf);
    if (A.n < 2)
        return false; // the vertex itself
    while (it + 2 < A.n && A.x[it + 1] <= x)
        ++it;
    return chord_inside(A, it, sign, delta, d2f, x, y, xf, yf);
}

// The arc's value at x (its end lines outside [x[0], x[n-1]]) and a bound of
// the rounding of that value's binary64 evaluation.
__device__ inline double arc_value(const Arc &A, double x, double &err)
{
    if (x <= A.x[0]) {
        const double t = A.gl * (x - A.x[0]);
        err = 0x1p-50 * (fabs(A.y[0]) + fabs(t));
        return x == A.x[0] ? A.y[0] : A.y[0] + t;
    }
    if (x >= A.x[A.n - 1]) {
        const double t = A.gr * (x - A.x[A.n - 1]);
        err = 0x1p-50 * (fabs(A.y[A.n - 1]) + fabs(t));
        return x == A.x[A.n - 1] ? A.y[A.n - 1] : A.y[A.n - 1] + t;
    }
    int i = 0; // here x[0] < x < x[n-1], so n >= 2
    while (i + 2 < A.n && A.x[i + 1] <= x)
        ++i;
    const double dy = A.y[i + 1] - A.y[i], t = dy * ((x - A.x[i]) / (A.x[i + 1] - A.x[i]));
    err = 0x1p-50 * (fabs(A.y[i]) + 2.0 * fabs(dy));
    return A.y[i] + t;
}

// Monotone-chain step: b (between a and p) lies more than 2 delta inside the
// segment a-p (below it for the upper chain, sign = +1; above for the lower).
__device__ inline bool chain_drop(double ax, double ay, double bx, double by, double px, double py, double sign,
                                  double delta)
{
    const double t1 = (px - ax) * (by - ay), t2 = (py - ay) * (bx - ax);
    const double cr = sign * (t1 - t2);
    return cr + kErr * (fabs(t1) + fabs(t2)) < -2.0 * delta * (px - ax);
}

// Points [lo, hi) of slab i of bucket [s, e), as the first pass filled it:
// chunks of 256 points from a0 (the first point at a 16-byte boundary of Y)
// to t0, merged evenly into kSlabs slabs when there are more, or split into
// their 64-point rows when there are at most kSlabs / 4; the points before a0
// belong to slab 0, those from t0 on to the slab of the last group.
struct SlabMap {
    int64_t s, e, a0, t0, nq, nchunks;
    bool fine;
    __device__ void init(const float *Y, int64_t s_, int64_t e_)
    {
        s = s_;
        e = e_;
        const uint64_t ya = (uint64_t)(uintptr_t)(Y + s);
        a0 = s + (int64_t)(((16u - (unsigned)(ya & 15u)) & 15u) >> 2);
        a0 = a0 < e ? a0 : e;
        nq = (e - a0) >> 2;
        t0 = a0 + 4 * nq;
        nchunks = (nq + 63) >> 6;
        fine = nchunks * 4 <= kSlabs;
    }
    __device__ int last_slab() const
    {
        if (nchunks == 0)
            return 0;
        if (fine)
            return (int)((nq - 1) >> 4);
        return (int)(nchunks <= kSlabs ? nchunks - 1 : ((nchunks - 1) * kSlabs) / nchunks);
    }
    __device__ void range(int i, int64_t &lo, int64_t &hi) const
    {
        int64_t c0, c1; // chunks [c0, c1), or 64-point rows when fine
        if (fine) {
            lo = a0 + 64 * (int64_t)i;
            hi = a0 + 64 * (int64_t)(i + 1);
            hi = hi < t0 ? hi : t0;
            if (i == 0)
                lo = s;
            if (i == last_slab())
                hi = e;
            if (hi < lo)
                hi = lo;
            return;
        }
        if (nchunks <= kSlabs) {
            c0 = i < nchunks ? i : nchunks;
            c1 = i < nchunks ? i + 1 : nchunks;
        } else {
            c0 = ((int64_t)i * nchunks + kSlabs - 1) / kSlabs;
            c1 = ((int64_t)(i + 1) * nchunks + kSlabs - 1) / kSlabs;
        }
        lo = a0 + 256 * c0;
        hi = a0 + 256 * c1;
        hi = hi < t0 ? hi : t0;
        if (i == 0)
            lo = s;
        if (i == last_slab())
            hi = e;
        if (hi < lo)
            hi = lo;
    }
};

// One workgroup of two waves per bucket b:
//  1. the slope bracket [g0, g1] of its possible predecessors and delta;
//  2. the arcs: wave 0 the upper (over the slab highs), wave 1 the lower
//     (slab lows) -- the touching points (lowest index with the largest
//     sign * (Y - g X)) of kArcSlopes slopes from the end slope gL to gR (upper:
//     g1 down to g0; lower: g0 up to g1), spread evenly in angle in the
//     bucket's own scale, in order of x, continued by the end lines;
//  3. per slab: whether it can hold a survivor -- none when its highest y lies
//     more than 2 delta (rounding included) below the upper arc's least value
//     over the slab's x range (the least of its values at the range's ends and
//     at the vertices inside) and its lowest y likewise above the lower arc;
//  4. the points of the other slabs through the exact tests: the survivors;
//  5. two monotone chains over the survivors: the candidates.
static_assert(kSlabs == 128, "k_lttb_hull tests slab i on thread i of its two waves");
__global__ __launch_bounds__(128) void k_lttb_hull(const int64_t *__restrict__ X, const float *__restrict__ Y,
                                                   int64_t n, int64_t B, const double *__restrict__ MX,
                                                   const double *__restrict__ MY, const float2 *__restrict__ YR,
                                                   const unsigned long long *__restrict__ slab_hi,
                                                   const unsigned long long *__restrict__ slab_lo,
                                                   int32_t *__restrict__ cand_cnt, int32_t *__restrict__ cand,
                                                   double *__restrict__ delta_out, double2 *__restrict__ brk)
{
    __shared__ double gx[2 * kSlabs], gy[2 * kSlabs], ex_[2], ey_[4];
    __shared__ int32_t go[2 * kSlabs];
    __shared__ Arc arc[2];
    __shared__ int64_t fl_lo[kSlabs];
    __shared__ int32_t fl_at[kSlabs + 1], s_wcnt[2], s_wlen[2];
    __shared__ double sx[kSurvMax], sy[kSurvMax], tx[kSurvMax], ty[kSurvMax];
    __shared__ int32_t si[kSurvMax], ti[kSurvMax];
    __shared__ double cxs[2][kChainMax], cys[2][kChainMax];
    __shared__ int32_t ci[2][kChainMax];
    __shared__ int32_t cn[2], nsurv, ovf;
    __shared__ double s_g0, s_g1, s_delta;
    const int tid = threadIdx.x, wid = tid >> 6, lane = tid & 63;
    const int64_t b = blockIdx.x;
    const Split bk = make_split(n - 2, B);
    const int64_t s = 1 + split_lo(bk, b), e = 1 + split_lo(bk, b + 1);
    const int32_t cnt = (int32_t)(e - s);
    const double inf = __longlong_as_double(0x7ff0000000000000ll);
    const double x0 = xval(X, s);
    if (tid == 0) {
        nsurv = 0;
        ovf = 0;
        // slopes from the possible predecessors (point 0, or the bounding box
        // of bucket b-1) to the mean, widened by a margin
        const double mx = MX[b] - x0, my = MY[b];
        double px0, px1, py0, py1;
        if (b == 0) {
            px0 = px1 = xval(X, 0) - x0;
            py0 = py1 = (double)Y[0];
        } else {
            px0 = xval(X, 1 + split_lo(bk, b - 1)) - x0;
            px1 = xval(X, s - 1) - x0;
            py0 = (double)YR[b - 1].x;
            py1 = (double)YR[b - 1].y;
        }
        const double c0 = (my - py0) / (mx - px0), c1 = (my - py0) / (mx - px1), c2 = (my - py1) / (mx - px0),
                     c3 = (my - py1) / (mx - px1);
        double g0 = fmin(fmin(c0, c1), fmin(c2, c3)), g1 = fmax(fmax(c0, c1), fmax(c2, c3));
        const double pad = 1e-6 * (g1 - g0) + 1e-9 * (fabs(g0) + fabs(g1)) + 1e-300;
        g0 -= pad;
        g1 += pad;
        if (!(g0 <= g1)) { // not a number: every slope
            g0 = -inf;
            g1 = inf;
        }
        s_g0 = g0;
        s_g1 = g1;
        const double span = (double)YR[b].y - (double)YR[b].x;
        s_delta = span > 0.0 && span < inf ? ldexp(span, -30) : 0.0;
        delta_out[b] = s_delta;
        brk[b] = make_double2(g0, g1); // the slopes the survivor test holds for
        ex_[0] = 0.0;
        ey_[0] = (double)Y[s];
        ex_[1] = xval(X, e - 1) - x0;
        ey_[1] = (double)Y[e - 1];
        ey_[2] = (double)YR[b].y;
        ey_[3] = (double)YR[b].x;
    }
    // the slab highs and lows (thread i: slab i): y from the keys, x
    // interpolated by position between the slab's first and last x (the
    // arcs' choice of vertices only; a vertex's own x is read exactly), and
    // the slab's x range for its test
    SlabMap sm;
    sm.init(Y, s, e);
    int64_t lo, hi;
    sm.range(tid, lo, hi);
    double xl = 0.0, xh = 0.0;
    {
        const unsigned long long ku = slab_hi[b * kSlabs + tid], kd = slab_lo[b * kSlabs + tid];
        if (hi > lo) {
            xl = xval(X, lo) - x0;
            xh = xval(X, hi - 1) - x0;
        }
        const double span = hi - 1 > lo ? (double)(hi - 1 - lo) : 1.0;
#pragma unroll
        for (int w = 0; w < 2; ++w) {
            const unsigned long long kk = w == 0 ? ku : kd;
            int32_t o = -1;
            if (kk != (w == 0 ? 0ull : ~0ull)) {
                const uint32_t lw = (uint32_t)kk;
                o = (int32_t)(w == 0 ? 0xffffffffu - lw : lw);
                o = o < 0 ? 0 : (o >= cnt ? cnt - 1 : o);
            }
            const double f = o >= 0 ? fmin(fmax((double)(s + o - lo) / span, 0.0), 1.0) : 0.0;
            gx[w * kSlabs + tid] = xl + (xh - xl) * f;
            gy[w * kSlabs + tid] = o >= 0 ? (double)f32_from_order_key((uint32_t)(kk >> 32)) : 0.0;
            go[w * kSlabs + tid] = o;
        }
    }
    __syncthreads();
    const double delta = s_delta;
    const float d2f = (float)(2.0 * delta) * 1.0001f;

    { // 2. the arcs: wave 0 the upper, wave 1 the lower
        Arc &A = arc[wid];
        const bool upper = wid == 0;
        const double sign = upper ? 1.0 : -1.0;
        const double g0 = s_g0, g1 = s_g1;
        const double gL = upper ? g1 : g0, gR = upper ? g0 : g1;
        constexpr int kPts = kSlabs + 2; // 0 the first point, 1..kSlabs the slabs, kSlabs+1 the last point
        auto pt = [&](int j, double &x, double &y) {
            if (j == 0 || j == kPts - 1) {
                x = ex_[j == 0 ? 0 : 1];
                y = ey_[j == 0 ? 0 : 1];
                return true;
            }
            const int q = (upper ? 0 : kSlabs) + j - 1;
            x = gx[q];
            y = gy[q];
            return go[q] >= 0;
        };
        // kArcSlopes slopes from gL to gR: the unit directions (1, g r) of the
        // two ends ((0, +-1) for an infinite slope), r = x span / y span,
        // mixed linearly. Any slopes in the bracket make a valid arc; these
        // spread its vertices along the hull.
        double gs[kArcSlopes];
        {
            const double ys = fmax(ey_[2] - ey_[3], 1e-300), xs = fmax(ex_[1], 1.0);
            const double r = xs / ys;
            double dxL, dyL, dxR, dyR;
            auto dir = [&](double g, double &dx, double &dy) {
                const double t = g * r;
                if (!(fabs(t) < 1e150)) {
                    dx = 0.0;
                    dy = t > 0.0 ? 1.0 : -1.0;
                } else {
                    const double h = 1.0 / sqrt(1.0 + t * t);
                    dx = h;
                    dy = t * h;
                }
            };
            dir(gL, dxL, dyL);
            dir(gR, dxR, dyR);
#pragma unroll
            for (int i = 0; i < kArcSlopes; ++i) {
                const double w = (double)i / (kArcSlopes - 1);
                const double dx = (1.0 - w) * dxL + w * dxR, dy = (1.0 - w) * dyL + w * dyR;
                gs[i] = dy / fmax(dx, 1e-150) / r;
            }
        }
        double best[kArcSlopes];
        int bi[kArcSlopes];
#pragma unroll
        for (int i = 0; i < kArcSlopes; ++i) {
            best[i] = -inf;
            bi[i] = 0x7fffffff;
        }
        for (int j = lane; j < kPts; j += 64) {
            double x, y;
            if (!pt(j, x, y))
                continue;
#pragma unroll
            for (int i = 0; i < kArcSlopes; ++i) {
                const double v = sign * (y - gs[i] * x);
                if (v > best[i]) { // increasing j per lane: the lowest keeps a tie
                    best[i] = v;
                    bi[i] = j;
                }
            }
        }
        // across the wave, all slopes at once
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
#pragma unroll
            for (int i = 0; i < kArcSlopes; ++i) {
                const double ob = __shfl_xor(best[i], off);
                const int oi = __shfl_xor(bi[i], off);
                if (ob > best[i] || (ob == best[i] && oi < bi[i])) {
                    best[i] = ob;
                    bi[i] = oi;
                }
            }
        }
        if (!(fabs(gL) < inf)) // vertical end slopes: the first or the last point
            bi[0] = 0;
        if (!(fabs(gR) < inf))
            bi[kArcSlopes - 1] = kPts - 1;
        // the vertices: slope i's touching point when it lies after every
        // earlier one (x increasing); lane i places slope i's
        int run = -1, m = 0, mine = -1, at = 0, next = -1;
#pragma unroll
        for (int i = 0; i < kArcSlopes; ++i) {
            const int j = bi[i] == 0x7fffffff ? (i == 0 ? 0 : kPts - 1) : bi[i];
            const bool keep = j > run;
            if (keep) {
                if (i == lane) {
                    mine = j;
                    at = m;
                } else if (i > lane && next < 0) {
                    next = j;
                }
                run = j;
                ++m;
            }
        }
        double vx = 0.0, vy = 0.0;
        if (mine >= 0) { // the vertex itself, x read exactly
            pt(mine, vx, vy);
            if (mine != 0 && mine != kPts - 1)
                vx = xval(X, s + go[(upper ? 0 : kSlabs) + mine - 1]) - x0;
            A.x[at] = vx;
            A.y[at] = vy;
            A.xf[at] = (float)vx;
            A.yf[at] = (float)vy;
        }
        if (lane == 0) {
            A.n = m;
            A.gl = gL;
            A.gr = gR;
            A.glf = (float)gL;
            A.grf = (float)gR;
        }
        __syncthreads();
        if (mine >= 0)
            A.sf[at] = next >= 0 ? (float)((A.y[at + 1] - vy) / (A.x[at + 1] - vx)) : 0.0f;
    }
    __syncthreads();

    // 3. the slabs that can hold a survivor (thread i tests slab i), listed
    // in order with their first point and their place in the list's points
    bool need = false;
    if (hi > lo) {
        for (int w = 0; w < 2 && !need; ++w) {
            const Arc &A = arc[w];
            const double sign = w == 0 ? 1.0 : -1.0;
            if (A.n < 1 || go[w * kSlabs + tid] < 0) {
                need = true;
                break;
            }
            // the least (upper) or greatest (lower) arc value over [xl, xh]
            double ea, eb;
            double v = sign * fmin(sign * arc_value(A, xl, ea), sign * arc_value(A, xh, eb));
            const double err = fmax(ea, eb);
            for (int q = 0; q < A.n; ++q)
                if (A.x[q] > xl && A.x[q] < xh)
                    v = sign > 0 ? fmin(v, A.y[q]) : fmax(v, A.y[q]);
            const double ext = gy[w * kSlabs + tid]; // the slab's highest (upper) or lowest (lower) y
            const double gap = sign * (v - ext);      // > 0 when the slab lies inside
            need = !(gap - err - 0x1p-50 * (fabs(v) + fabs(ext)) > 2.0 * delta);
        }
    }
    {
        const int len = need ? (int)(hi - lo) : 0;
        const unsigned long long bal = __ballot(need);
        int v = len; // inclusive prefix over the wave
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int t = __shfl_up(v, off);
            v += lane >= off ? t : 0;
        }
        if (lane == 63) {
            s_wcnt[wid] = __popcll(bal);
            s_wlen[wid] = v;
        }
        __syncthreads();
        if (need) {
            const int q = (wid ? s_wcnt[0] : 0) + __popcll(bal & ((1ull << lane) - 1ull));
            fl_lo[q] = lo;
            fl_at[q] = (wid ? s_wlen[0] : 0) + v - len;
        }
        if (tid == 0)
            fl_at[s_wcnt[0] + s_wcnt[1]] = s_wlen[0] + s_wlen[1];
    }
    __syncthreads();

    // 4. survivors: the points of those slabs not inside both arcs, kScanU
    // loads in flight per thread
    {
        const int F = s_wlen[0] + s_wlen[1];
        int iu = 0, il = 0, j = 0;
        for (int f0 = 0; f0 < F; f0 += kScanU * kSlabs) {
            int64_t p[kScanU];
#pragma unroll
            for (int u = 0; u < kScanU; ++u) {
                const int f = f0 + u * kSlabs + tid;
                if (f < F) {
                    while (fl_at[j + 1] <= f)
                        ++j;
                    p[u] = fl_lo[j] + (f - fl_at[j]);
                } else {
                    p[u] = -1;
                }
            }
            double xv[kScanU];
            float yv[kScanU];
#pragma unroll
            for (int u = 0; u < kScanU; ++u) {
                const int64_t q = p[u] >= 0 ? p[u] : s;
                xv[u] = xval(X, q);
                yv[u] = Y[q];
            }
#pragma unroll
            for (int u = 0; u < kScanU; ++u) {
                if (p[u] < 0)
                    continue;
                const double x = xv[u] - x0, y = (double)yv[u];
                const float xf = (float)x, yf = (float)y;
                const bool inside = arc_inside(arc[0], 1.0, delta, d2f, x, y, xf, yf, iu) &&
                                    arc_inside(arc[1], -1.0, delta, d2f, x, y, xf, yf, il);
                if (!inside) {
                    const int q = atomicAdd(&nsurv, 1);
                    if (q < kSurvMax) {
                        sx[q] = x;
                        sy[q] = y;
                        si[q] = (int32_t)(p[u] - s);
                    }
                }
            }
        }
    }
    __syncthreads();
    const int total = nsurv;
    const int ns = total < kSurvMax ? total : kSurvMax;
    for (int q = tid; q < ns; q += blockDim.x) { // rank sort by position (distinct)
        const int32_t me = si[q];
        int r = 0;
        for (int j = 0; j < ns; ++j)
            r += si[j] < me ? 1 : 0;
        tx[r] = sx[q];
        ty[r] = sy[q];
        ti[r] = me;
    }
    __syncthreads();

    // 5. chains: thread 0 the upper, thread 64 the lower (the two top
    // entries of the stack kept in registers)
    if ((tid & 63) == 0 && total <= kSurvMax) {
        const int c = tid >> 6;
        const double sign = c == 0 ? 1.0 : -1.0;
        int m = 0;
        double ax = 0.0, ay = 0.0, bx = 0.0, by = 0.0; // entries m-2 and m-1
        double x = ns > 0 ? tx[0] : 0.0, y = ns > 0 ? ty[0] : 0.0;
        for (int q = 0; q < ns; ++q) {
            const double nx = q + 1 < ns ? tx[q + 1] : 0.0, ny = q + 1 < ns ? ty[q + 1] : 0.0;
            while (m >= 2 && chain_drop(ax, ay, bx, by, x, y, sign, delta)) {
                --m;
                bx = ax;
                by = ay;
                if (m >= 2) {
                    ax = cxs[c][m - 2];
                    ay = cys[c][m - 2];
                }
            }
            if (m < kChainMax) {
                cxs[c][m] = x;
                cys[c][m] = y;
                ci[c][m] = ti[q];
                ax = bx;
                ay = by;
                bx = x;
                by = y;
                ++m;
            } else {
                ovf = 1;
            }
            x = nx;
            y = ny;
        }
        cn[c] = m;
    }
    __syncthreads();

    if (tid == 0) { // candidates: both chains merged by position
        int32_t *out = cand + b * (int64_t)kCandMax;
        int a = 0, c = 0, m = 0;
        bool full = ovf != 0 || total > kSurvMax;
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
        }
        cand_cnt[b] = full ? -1 : m;
    }
}

// ------------------------------------------------------------------ pass 3

// Table entries slots[0 .. nc-1] (candidates of bucket k-1, or point 0 alone
// for k = 0) of bucket k by a scan of every point [s, e) of bucket k. Each
// thread scans its points in increasing position with a strict comparison;
// the workgroup then keeps the largest area and the lowest position among
// equal ones; no area above -1 (every one NaN) leaves the bucket's first
// point, as in the sequential pass.
__device__ inline void table_group(const int64_t *__restrict__ X, const float *__restrict__ Y, int64_t k, int64_t B,
                                   int64_t s, int64_t e, int64_t sp, const int32_t *slots, int nc, double mx,
                                   double my, const int32_t *__restrict__ cand_cnt, const int32_t *__restrict__ cand,
                                   int2 *__restrict__ tab, double (*s_best)[kTabGroup], int32_t (*s_idx)[kTabGroup])
{
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
    double xa[kTabGroup], ya[kTabGroup], best[kTabGroup];
    int32_t bi[kTabGroup];
#pragma unroll
    for (int c = 0; c < kTabGroup; ++c) {
        const int64_t a = k == 0 ? 0 : sp + cand[(k - 1) * (int64_t)kCandMax + slots[c < nc ? c : 0]];
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
        tab[k * (int64_t)kCandMax + slots[tid]] = make_int2(off, next);
    }
    __syncthreads(); // s_best and s_idx are reused by the next group
}

// One workgroup per bucket k: every candidate a of bucket k-1 (point 0 for
// k = 0) against bucket k's candidates, one thread each; the entries the
// certificate does not cover scan the bucket in full, kTabGroup at a time.
constexpr int kTableThreads = 256;
__global__ __launch_bounds__(kTableThreads) void k_lttb_tables(const int64_t *__restrict__ X,
                                                               const float *__restrict__ Y, int64_t n, int64_t B,
                                                               const double *__restrict__ MX,
                                                               const double *__restrict__ MY,
                                                               const float2 *__restrict__ YR,
                                                               const int32_t *__restrict__ cand_cnt,
                                                               const int32_t *__restrict__ cand,
                                                               const double *__restrict__ delta,
                                                               const double2 *__restrict__ brk,
                                                               int2 *__restrict__ tab)
{
    __shared__ double s_best[kTableThreads / kWave][kTabGroup];
    __shared__ int32_t s_idx[kTableThreads / kWave][kTabGroup];
    __shared__ double cx[kCandMax], cy[kCandMax];
    __shared__ int32_t co[kCandMax], todo[kCandMax];
    __shared__ int ntodo;
    const int tid = threadIdx.x;
    const int64_t k = blockIdx.x;
    const int npred = k == 0 ? 1 : cand_cnt[k - 1];
    if (npred <= 0) // no candidates before: the walk scans this bucket itself
        return;
    const Split bk = make_split(n - 2, B);
    const int64_t s = 1 + split_lo(bk, k), e = 1 + split_lo(bk, k + 1);
    const int64_t sp = k == 0 ? 0 : 1 + split_lo(bk, k - 1);
    const double mx = MX[k], my = MY[k];
    const int nk = cand_cnt[k];
    if (tid < nk) {
        const int32_t o = cand[k * (int64_t)kCandMax + tid];
        co[tid] = o;
        cx[tid] = xval(X, s + o);
        cy[tid] = (double)Y[s + o];
    }
    if (tid == 0)
        ntodo = 0;
    __syncthreads();
    if (tid < npred) {
        const int64_t a = k == 0 ? 0 : sp + cand[(k - 1) * (int64_t)kCandMax + tid];
        const double xa = xval(X, a), ya = (double)Y[a];
        bool ok = nk > 0;
        int bo = 0;
        if (ok) {
            double best = -1.0;
            for (int j = 0; j < nk; ++j) { // increasing position, strict: the lowest wins ties
                const double ar = lttb_area2(xa, ya, cx[j], cy[j], mx, my);
                if (ar > best) {
                    best = ar;
                    bo = j;
                }
            }
            // certificate: the slope from a to the mean inside the bracket the
            // hull pass used, and the candidates' margin above the rounding
            const double A = fabs(xa - mx), D = my - ya, slope = D / (mx - xa);
            const float2 yr = YR[k];
            const double bmax = fmax(fabs((double)yr.y - ya), fabs((double)yr.x - ya));
            const double cmax = xval(X, e - 1) - xa;
            const double E = kErr * (A * bmax + cmax * fabs(D));
            const double2 br = brk[k];
            const double slack = 0x1p-48 * fabs(slope);
            ok = best > -1.0 && slope - slack > br.x && slope + slack < br.y && A * delta[k] > E * (1.0 + 0x1p-20);
        }
        if (ok)
            tab[k * (int64_t)kCandMax + tid] = make_int2(co[bo], k + 1 < B ? bo : -1);
        else
            todo[atomicAdd(&ntodo, 1)] = tid;
    }
    __syncthreads();
    const int nt = ntodo;
    for (int c0 = 0; c0 < nt; c0 += kTabGroup) {
        const int nc = nt - c0 < kTabGroup ? nt - c0 : kTabGroup;
        table_group(X, Y, k, B, s, e, sp, todo + c0, nc, mx, my, cand_cnt, cand, tab, s_best, s_idx);
    }
}

// One workgroup of 1024 threads. A window of up to kWalkWindow buckets from
// bucket k, entered at slot `slot`: every segment of kWalkSeg buckets is
// followed from every entry slot at once (one thread each), then every group
// of kWalkGroup segments from every entry slot (one thread each); thread 0
// links the groups from the true entry slot, and the picks of the window are
// written in parallel. The window ends early at the first bucket whose entry
// slot is not staged: -1 (the predecessor is not a candidate: the whole
// workgroup then scans that bucket for its pick) or past the staged ones (one
// step from global memory).
__global__ __launch_bounds__(1024) void k_lttb_table_walk(const int64_t *__restrict__ X, const float *__restrict__ Y,
                                                          int64_t n, int64_t B, const double *__restrict__ MX,
                                                          const double *__restrict__ MY,
                                                          const int32_t *__restrict__ cand_cnt,
                                                          const int32_t *__restrict__ cand,
                                                          const int2 *__restrict__ tab, int64_t *__restrict__ out)
{
    constexpr int kSegs = kWalkWindow / kWalkSeg, kGroups = kSegs / kWalkGroup;
    __shared__ uint8_t sN[kWalkWindow * kWalkSlots];        // next slot (kWalkOut: not staged)
    __shared__ uint8_t spath[kSegs][kWalkSlots][kWalkSeg];  // slot at each bucket of a segment, per entry
    __shared__ uint8_t sdone[kSegs][kWalkSlots], sexit[kSegs][kWalkSlots];
    __shared__ uint8_t gpath[kGroups][kWalkSlots][kWalkGroup]; // entry slot of each segment of a group, per entry
    __shared__ int16_t gdone[kGroups][kWalkSlots];          // buckets of the group walked from the tables
    __shared__ uint8_t gexit[kGroups][kWalkSlots], gent[kGroups];
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
            const int ngrp = (nseg + kWalkGroup - 1) / kWalkGroup;
            for (int q = tid; q < W * kWalkSlots; q += blockDim.x) {
                const int32_t nx = tab[(k + q / kWalkSlots) * kCandMax + q % kWalkSlots].y;
                sN[q] = nx >= 0 && nx < kWalkSlots ? (uint8_t)nx : kWalkOut;
            }
            __syncthreads();
            for (int q = tid; q < nseg * kWalkSlots; q += blockDim.x) { // segment g from entry slot e
                const int g = q / kWalkSlots, e = q % kWalkSlots;
                const int len = W - g * kWalkSeg < kWalkSeg ? W - g * kWalkSeg : kWalkSeg;
                int sl = e, i = 0;
                for (; i < len && sl != kWalkOut; ++i) {
                    spath[g][e][i] = (uint8_t)sl;
                    sl = sN[(g * kWalkSeg + i) * kWalkSlots + sl];
                }
                sdone[g][e] = (uint8_t)i; // buckets picked from the tables
                sexit[g][e] = (uint8_t)sl; // the entry slot of the next segment
            }
            __syncthreads();
            if (tid < ngrp * kWalkSlots) { // group G from entry slot e
                const int G = tid / kWalkSlots, e = tid % kWalkSlots;
                const int g0 = G * kWalkGroup, g1 = g0 + kWalkGroup < nseg ? g0 + kWalkGroup : nseg;
                int cur = e, done = 0;
                for (int g = g0; g < g1 && cur != kWalkOut; ++g) {
                    const int len = W - g * kWalkSeg < kWalkSeg ? W - g * kWalkSeg : kWalkSeg;
                    gpath[G][e][g - g0] = (uint8_t)cur;
                    const int d = sdone[g][cur];
                    done += d;
                    cur = d < len ? kWalkOut : sexit[g][cur];
                }
                gdone[G][e] = (int16_t)done;
                gexit[G][e] = (uint8_t)cur;
            }
            __syncthreads();
            if (tid == 0) {
                int cur = slot;
                int64_t stop = k1;
                for (int G = 0; G < ngrp; ++G) {
                    gent[G] = (uint8_t)cur;
                    const int glen = (G + 1) * kWalkGroup * kWalkSeg < W ? kWalkGroup * kWalkSeg : W - G * kWalkGroup * kWalkSeg;
                    const int d = gdone[G][cur];
                    cur = gexit[G][cur];
                    if (d < glen || cur == kWalkOut) { // the tables end inside or right after this group
                        stop = k + (int64_t)G * kWalkGroup * kWalkSeg + d;
                        break;
                    }
                }
                s_k = stop;
            }
            __syncthreads();
            const int64_t stop = s_k; // k < stop <= k1 <= B
            for (int t = tid; t < (int)(stop - k); t += blockDim.x) { // the picks of buckets k .. stop-1
                const int g = t / kWalkSeg, i = t % kWalkSeg, G = g / kWalkGroup;
                const int sl = spath[g][gpath[G][gent[G]][g - G * kWalkGroup]][i];
                const int2 te = tab[(k + t) * kCandMax + sl];
                const int64_t pick = 1 + split_lo(bk, k + t) + te.x;
                out[k + t + 1] = pick;
                if (k + t + 1 == stop) { // the last pick of the window and the slot it leads to
                    s_a = pick;
                    s_slot = te.y;
                }
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

hipError_t launch_lttb_scan(const int64_t *X, const float *Y, int64_t n, int64_t B, double *MX, double *MY, float2 *YR,
                            unsigned long long *slab_hi, unsigned long long *slab_lo, hipStream_t s)
{
    hipLaunchKernelGGL(k_lttb_scan, dim3((unsigned)B), dim3(256), 0, s, X, Y, n, B, MX, MY, YR, slab_hi, slab_lo);
    return hipGetLastError();
}

hipError_t launch_lttb_hull(const int64_t *X, const float *Y, int64_t n, int64_t B, const double *MX, const double *MY,
                            const float2 *YR, const unsigned long long *slab_hi, const unsigned long long *slab_lo,
                            int32_t *cand_cnt, int32_t *cand, double *delta, double2 *brk, hipStream_t s)
{
    hipLaunchKernelGGL(k_lttb_hull, dim3((unsigned)B), dim3(128), 0, s, X, Y, n, B, MX, MY, YR, slab_hi, slab_lo,
                       cand_cnt, cand, delta, brk);
    return hipGetLastError();
}

hipError_t launch_lttb_tables(const int64_t *X, const float *Y, int64_t n, int64_t B, const double *MX,
                              const double *MY, const float2 *YR, const int32_t *cand_cnt, const int32_t *cand,
                              const double *delta, const double2 *brk, int2 *tab, hipStream_t s)
{
    hipLaunchKernelGGL(k_lttb_tables, dim3((unsigned)B), dim3(kTableThreads), 0, s, X, Y, n, B, MX, MY, YR, cand_cnt,
                       cand, delta, brk, tab);
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
