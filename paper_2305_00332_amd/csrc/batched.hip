// Batched MinMaxLTTB: many series of uneven length in one call.
//
// The host plans every series into a BatchSeg (mode, bins, work ranges, pooled
// workspace slots) and copies the table into the workspace. The stream and
// chain kernels launch one wave or workgroup per unit of a flat work space
// (the hardware balances uneven units); a unit finds its series through a
// coarse owner table and a short binary search. Per-series kernels loop over
// the series with a grid-stride.
//
//   init      keys to their identities (only when large-bin series exist)
//   large     series whose bins hold more than tile / 4 points: one wave per
//             fixed-size chunk of the series, streaming across bin ends
//             (16-byte loads, one atomic key merge per bin part)
//   small     series with small bins: a workgroup stages a tile of whole bins
//             (<= tile points) in LDS; a power-of-two lane group reduces each
//             bin and stores its keys
//   compact_means  one workgroup per series: P, X_P, Y_P, m, then the exact
//             next-bucket means (identity series write their output here)
//   chain     segmented chain, walks: one wave per (series, chain segment)
//             walks the segment from every start point
//   chain_seq sequential chain for series whose buckets exceed kSegStarts
//   link_emit one workgroup per series: links its chain segments and writes
//             the picks mapped through P to the output
//
// Each series' result equals the single-series call on it alone: the same
// bins, keys, exact means and binary64 areas, evaluated in the same order.
#include "chain_device.hpp"
#include "device_common.hpp"
#include "kernels.hpp"
#include "minmax_device.hpp"

namespace mmlttb {

// Series owning unit i of a flat work space: the last series whose start is
// <= i (series with no work there start where the next one starts), searched
// between two neighbouring entries of the space's coarse owner table.
template <class StartOf>
__device__ inline int64_t find_owner(const BatchSeg *__restrict__ segs, const int32_t *__restrict__ table,
                                     int64_t total, int64_t i, StartOf start_of)
{
    const int64_t q = (i * kOwnerTable) / total;
    int64_t lo = table[q], hi = table[q + 1];
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (start_of(segs[mid]) <= i)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

__global__ __launch_bounds__(256) void k_batch_init(BatchPtrs b)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t i = t; i < b.n_keys; i += stride) {
        b.keys[2 * i] = ~0ull;
        b.keys[2 * i + 1] = 0ull;
    }
}

template <int U>
__global__ __launch_bounds__(256) void k_batch_large(BatchPtrs b)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int64_t i = (int64_t)blockIdx.x * (blockDim.x / kWave) + wave;
    const int64_t total = b.n_large_items;
    if (i >= total)
        return;
    const int64_t s = find_owner(b.segs, b.hdr->own_large, total, i, [](const BatchSeg &g) { return g.li0; });
    const BatchSeg &g = b.segs[s];
    const int64_t lo = 1 + (i - g.li0) * g.chunk;
    const int64_t hi = (lo + g.chunk < g.n - 1) ? lo + g.chunk : g.n - 1;
    wave_stream_bins<U>(b.y_base + g.offset, lo, hi, g.bins, b.keys + 2 * g.key0, lane);
}

// floor(t / d) for 0 <= t < 2^52 and d >= 1, given inv = RN(1/d): the
// binary64 product is within one of the quotient, and one integer step
// corrects it (cheaper than a 64-bit integer division on the GPU).
__device__ inline int64_t div_near(int64_t t, int64_t d, double inv)
{
    int64_t q = (int64_t)((double)t * inv);
    const int64_t r = t - q * d;
    q += (r < 0) ? -1 : (r >= d ? 1 : 0);
    return q;
}

// Reduce tile[q] for q = q0, q0 + step, ... < end (q0 < end) in increasing q:
// value and lowest position of the minimum and of the maximum.
__device__ inline void strided_minmax(const float *tile, int q0, int end, int step, float &vmin, int &imin,
                                      float &vmax, int &imax)
{
    vmin = vmax = tile[q0];
    imin = imax = q0;
    int q = q0 + step;
    for (; q + 3 * step < end; q += 4 * step) { // four independent LDS reads per wait
        const float v0 = tile[q], v1 = tile[q + step], v2 = tile[q + 2 * step], v3 = tile[q + 3 * step];
        const float v[4] = {v0, v1, v2, v3};
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (v[u] < vmin) {
                vmin = v[u];
                imin = q + u * step;
            }
            if (v[u] > vmax) {
                vmax = v[u];
                imax = q + u * step;
            }
        }
    }
    for (; q < end; q += step) {
        const float v = tile[q];
        if (v < vmin) {
            vmin = v;
            imin = q;
        }
        if (v > vmax) {
            vmax = v;
            imax = q;
        }
    }
}

static_assert(kTileThreads == 256, "k_batch_small derives lanes per bin from 2^8 threads");

// One small-bin tile: its bins, its point range [lo, hi) split into an
// aligned body of nvec float4 and at most 3 head and 3 tail points.
struct SmallTile {
    const float *y;
    unsigned long long *keys; // key pair of the tile's first bin
    int64_t lo, hi, body, nvec, tail0, nb, bq, br, rem0;
    double inv;
    int nbt, lg;
};

// Tile `tl` of one series (y: the series, keys: its first bin's key pair,
// bins over its interior, G bins a tile).
__device__ inline SmallTile plan_series_tile(const float *y, unsigned long long *keys, const Split &bins, int G,
                                             int64_t tl)
{
    SmallTile T;
    T.lg = 8 - __builtin_ctz((unsigned)G);     // log2 of the lanes per bin (kTileThreads = 2^8); G a power of two, 4..256
    T.nb = bins.parts;
    T.bq = bins.q;
    T.br = bins.r;
    const int64_t bb0 = tl * G;
    T.nbt = (int)((bb0 + G < T.nb) ? G : T.nb - bb0); // bins in this tile
    // Bin bb0 + i starts at split_lo(bb0) + i q + floor((rem0 + i r) / nb), with
    // rem0 = bb0 r mod nb; the planner routes only nb < 2^26 here, so every
    // numerator is below 2^52.
    T.inv = 1.0 / (double)T.nb;
    const int64_t t0 = bb0 * T.br;
    const int64_t f0 = div_near(t0, T.nb, T.inv);
    T.rem0 = t0 - f0 * T.nb;
    T.lo = 1 + bb0 * T.bq + f0;
    T.hi = T.lo + (int64_t)T.nbt * T.bq + div_near(T.rem0 + (int64_t)T.nbt * T.br, T.nb, T.inv);
    T.y = y;
    T.keys = keys + 2 * bb0;
    const uint64_t addr = (uint64_t)(uintptr_t)(T.y + T.lo);
    int64_t head = (int64_t)(((16u - (unsigned)(addr & 15u)) & 15u) >> 2);
    head = head < T.hi - T.lo ? head : T.hi - T.lo;
    T.body = T.lo + head;
    T.nvec = (T.hi - T.body) >> 2;
    T.tail0 = T.body + 4 * T.nvec;
    return T;
}

__device__ inline SmallTile plan_small_tile(const BatchPtrs &b, int64_t t)
{
    const int64_t s = find_owner(b.segs, b.hdr->own_small, b.n_small_tiles, t, [](const BatchSeg &g) { return g.ti0; });
    const BatchSeg &g = b.segs[s];
    return plan_series_tile(b.y_base + g.offset, b.keys + 2 * g.key0, g.bins, g.tile_bins, t - g.ti0);
}

// Issue the tile's loads: 16-byte loads of the body, plus one head or tail
// point for threads 0-2 and 4-6 (hq < 0: none).
template <int kVec>
__device__ inline void load_small_tile(const SmallTile &T, f32x4 (&d)[kVec], float &hv, int64_t &hq)
{
    const int tid = threadIdx.x;
    const f32x4 *__restrict__ v4 = reinterpret_cast<const f32x4 *>(T.y + T.body);
#pragma unroll
    for (int u = 0; u < kVec; ++u) {
        const int64_t q = tid + (int64_t)u * kTileThreads;
        if (q < T.nvec)
            d[u] = __builtin_nontemporal_load(v4 + q);
    }
    hv = 0.0f;
    hq = -1;
    if (tid < T.body - T.lo)
        hq = T.lo + tid;
    else if (tid >= 4 && tid < 4 + (T.hi - T.tail0))
        hq = T.tail0 + (tid - 4);
    if (hq >= 0)
        hv = T.y[hq];
}

// Stage the loaded tile and its bin starts in LDS (the caller then waits at a
// barrier before reduce_small_tile).
template <int kVec>
__device__ inline void stage_small_tile(const SmallTile &T, const f32x4 (&d)[kVec], float hv, int64_t hq, float *tile,
                                        int32_t *bstart)
{
    const int tid = threadIdx.x;
    for (int i = tid; i <= T.nbt; i += kTileThreads)
        bstart[i] = (int32_t)((int64_t)i * T.bq + div_near(T.rem0 + (int64_t)i * T.br, T.nb, T.inv));
#pragma unroll
    for (int u = 0; u < kVec; ++u) {
        const int64_t q = tid + (int64_t)u * kTileThreads;
        if (q < T.nvec) {
            float *dst = tile + (T.body - T.lo) + 4 * q;
            dst[0] = d[u].x;
            dst[1] = d[u].y;
            dst[2] = d[u].z;
            dst[3] = d[u].w;
        }
    }
    if (hq >= 0)
        tile[hq - T.lo] = hv;
}

// Every bin's key pair from the staged tile: a power-of-two group of
// 2^(8 - lg) lanes per bin.
__device__ inline void reduce_small_tile(const SmallTile &T, const float *tile, const int32_t *bstart)
{
    const int tid = threadIdx.x;
    const int tpb = 1 << T.lg; // lanes per bin: power of two <= 64
    const int gi = tid >> T.lg, sub = tid & (tpb - 1);
    unsigned long long kmin = ~0ull, kmax = 0ull; // identities: lanes with no point never win
    if (gi < T.nbt) {
        const int bs = bstart[gi], be = bstart[gi + 1];
        if (bs + sub < be) {
            float vmin, vmax;
            int imin, imax;
            strided_minmax(tile, bs + sub, be, tpb, vmin, imin, vmax, imax);
            kmin = pack_min_key(vmin, imin - bs);
            kmax = pack_max_key(vmax, imax - bs);
        }
    }
    group_minmax(tpb, kmin, kmax);
    if (sub == 0 && gi < T.nbt) {
        T.keys[2 * gi] = kmin;
        T.keys[2 * gi + 1] = kmax;
    }
}

// kSmallTilesPerBlock consecutive tiles per workgroup: a tile's loads are
// issued once the previous tile is staged in LDS, so they are in flight while
// that tile is reduced; the next tile's owner lookup overlaps the previous
// tile's loads.
constexpr int kSmallTilesPerBlock = 2;
static_assert(kSmallTilesPerBlock == 2, "k_batch_small is written for two tiles per workgroup");

// The tiles of this workgroup (plan(t) gives tile t of `total`), into the
// workgroup's LDS arrays.
template <int kTilePoints, class Plan>
__device__ inline void small_tile_pair(int64_t total, Plan plan, float *tile, int32_t *bstart)
{
    constexpr int kVec = kTilePoints / 4 / kTileThreads;
    const int64_t t0 = (int64_t)blockIdx.x * kSmallTilesPerBlock;
    if (t0 >= total)
        return;
    const int64_t t1 = t0 + 1 < total ? t0 + 1 : -1; // kSmallTilesPerBlock = 2
    f32x4 d0[kVec], d1[kVec];
    float hv0, hv1;
    int64_t hq0, hq1;
    const SmallTile T0 = plan(t0);
    load_small_tile(T0, d0, hv0, hq0);
    SmallTile T1;
    if (t1 >= 0)
        T1 = plan(t1);
    stage_small_tile(T0, d0, hv0, hq0, tile, bstart);
    if (t1 >= 0)
        load_small_tile(T1, d1, hv1, hq1);
    __syncthreads();
    reduce_small_tile(T0, tile, bstart);
    if (t1 >= 0) {
        __syncthreads(); // tile 0's readers are done with the LDS arrays
        stage_small_tile(T1, d1, hv1, hq1, tile, bstart);
        __syncthreads();
        reduce_small_tile(T1, tile, bstart);
    }
}

template <int kTilePoints>
__global__ __launch_bounds__(kTileThreads) void k_batch_small(BatchPtrs b)
{
    __shared__ float tile[kTilePoints];
    __shared__ int32_t bstart[kTileThreads + 1]; // bin starts, relative to the tile's first point
    small_tile_pair<kTilePoints>(b.n_small_tiles, [&](int64_t t) { return plan_small_tile(b, t); }, tile, bstart);
}

// One float32 series' short bins (at most a quarter tile each), G whole bins
// a tile: the batched small-bin body on a single series, writing every bin's
// key pair (no key initialisation).
template <int kTilePoints>
__global__ __launch_bounds__(kTileThreads) void k_minmax_small_tiles(const float *y, Split bins, int G, int64_t n_tiles,
                                                                     unsigned long long *keys)
{
    __shared__ float tile[kTilePoints];
    __shared__ int32_t bstart[kTileThreads + 1];
    small_tile_pair<kTilePoints>(n_tiles, [&](int64_t t) { return plan_series_tile(y, keys, bins, G, t); }, tile,
                                 bstart);
}

// One workgroup per series: compaction (the means follow in k_batch_means).
// Identity series (n <= n_out) write their output here. The compaction is a
// chain of dependent steps (keys, scan, x gathers, writes); workgroups of
// kCompactThreads let four series share a CU instead of one.
constexpr int kCompactThreads = 256;
__global__ __launch_bounds__(kCompactThreads) void k_batch_compact(BatchPtrs b)
{
    __shared__ int wave_tot[17];
    const int tid = threadIdx.x;
    for (int64_t s = blockIdx.x; s < b.n_segs; s += gridDim.x) {
        const BatchSeg &g = b.segs[s];
        const int64_t n = g.n;
        if (g.mode == kSegIdentity) {
            int64_t *out = b.out_base + g.out_offset;
            for (int64_t i = tid; i < n; i += blockDim.x)
                out[i] = i;
            continue;
        }
        const float *y = b.y_base + g.offset;
        const int64_t *x = b.xk ? b.x_base + g.offset : nullptr;
        int64_t *P = b.P + g.p0, *XP = b.XP + g.p0;
        float *YP = b.YP + g.p0;
        if (g.mode == kSegAll) {
            for (int64_t i = tid; i < n; i += blockDim.x) {
                P[i] = i;
                XP[i] = x ? x[i] : i;
                YP[i] = y[i];
            }
            if (tid == 0)
                b.m[s] = n;
        } else {
            compact_keys(b.keys + 2 * g.key0, g.bins, n, x, y, P, XP, YP, b.m + s, wave_tot);
        }
        __syncthreads();
    }
}

// Next-bucket means over P: series blockIdx.x, buckets blockIdx.y * 256 + t
// (+ gridDim.y * 256 ...), one thread per bucket. A kernel of its own so the
// register-heavy exact sums do not limit the compaction's occupancy.
__global__ __launch_bounds__(256) void k_batch_means(BatchPtrs b)
{
    const int64_t s = blockIdx.x;
    const BatchSeg &g = b.segs[s];
    if (g.mode == kSegIdentity)
        return;
    const int64_t m = b.m[s];
    const Split bk = make_split(m - 2, g.B);
    const int64_t *XP = b.XP + g.p0;
    const float *YP = b.YP + g.p0;
    for (int64_t k = (int64_t)blockIdx.y * blockDim.x + threadIdx.x; k < g.B; k += (int64_t)gridDim.y * blockDim.x)
        bucket_mean_one(XP, YP, bk, m, k, b.MX[g.b0 + k], b.MY[g.b0 + k]);
}

// Segmented chain, phase 1: one wave per (series, chain segment) walks the
// segment from every start point (seg_walk: transition tables, then lookups).
__global__ __launch_bounds__(kSegStarts) void k_batch_chain(BatchPtrs b)
{
    extern __shared__ double lds[];
    const int64_t u = blockIdx.x;
    const int64_t total = b.n_chain_units;
    if (u >= total)
        return;
    const int64_t s = find_owner(b.segs, b.hdr->own_chain, total, u, [](const BatchSeg &g) { return g.cw0; });
    const BatchSeg &g = b.segs[s];
    const int64_t m = b.m[s];
    const Split bk = make_split(m - 2, g.B);
    seg_walk(b.XP + g.p0, b.YP + g.p0, bk, b.MX + g.b0, b.MY + g.b0, u - g.cw0, g.stage_cap,
             reinterpret_cast<unsigned char *>(lds),
             b.path + (size_t)g.c0 * kSegStarts * kSegLen, b.finals + (size_t)g.c0 * kSegStarts, (int)threadIdx.x);
}

// Segmented chain, phases 2 and 3: one workgroup per series links its
// segments (seg_link) and writes every pick mapped through P.
__global__ __launch_bounds__(1024) void k_batch_link_emit(BatchPtrs b)
{
    __shared__ uint8_t F[kChaseWindow * kSegStarts];
    for (int64_t s = blockIdx.x; s < b.n_segs; s += gridDim.x) {
        const BatchSeg &g = b.segs[s];
        if (g.mode == kSegIdentity || g.seq)
            continue;
        const int64_t m = b.m[s];
        const Split bk = make_split(m - 2, g.B);
        const uint8_t *path = b.path + (size_t)g.c0 * kSegStarts * kSegLen;
        uint8_t *start = b.start + g.c0;
        seg_link(b.finals + (size_t)g.c0 * kSegStarts, start, g.cwn, F);
        const int64_t *P = b.P + g.p0;
        int64_t *out = b.out_base + g.out_offset;
        for (int64_t k = threadIdx.x; k < g.B; k += blockDim.x)
            out[k + 1] = P[seg_pick(path, start, bk, k)];
        if (threadIdx.x == 0) {
            out[0] = P[0];
            out[g.B + 1] = P[m - 1];
        }
        __syncthreads();
    }
}

// Sequential chain for series whose buckets exceed kSegStarts points: one
// wave walks the buckets in order reading the points from global memory.
__global__ __launch_bounds__(kWave) void k_batch_chain_seq(BatchPtrs b)
{
    const int lane = threadIdx.x;
    for (int64_t s = blockIdx.x; s < b.n_segs; s += gridDim.x) {
        const BatchSeg &g = b.segs[s];
        if (g.mode == kSegIdentity || !g.seq)
            continue;
        const int64_t m = b.m[s];
        const Split bk = make_split(m - 2, g.B);
        const int64_t *XP = b.XP + g.p0;
        const float *YP = b.YP + g.p0;
        int64_t *out = b.out_base + g.out_offset;
        double ax = (double)XP[0], ay = (double)YP[0];
        SplitWalker w;
        w.init(bk, 0);
        for (int64_t k = 0; k < g.B; ++k) {
            const int64_t s0 = 1 + w.lo, s1 = 1 + w.next_lo(bk);
            w.advance(bk);
            const double mx = b.MX[g.b0 + k], my = b.MY[g.b0 + k];
            double best = -1.0, bx = 0.0, by = 0.0;
            int64_t bj = INT64_MAX;
            for (int64_t j = s0 + lane; j < s1; j += kWave) {
                const double xj = (double)XP[j], yj = (double)YP[j];
                const double ar = lttb_area2(ax, ay, xj, yj, mx, my);
                if (ar > best) {
                    best = ar;
                    bj = j;
                    bx = xj;
                    by = yj;
                }
            }
            const double wb = wave_max_f64(best);
            const int64_t sel = wave_min_i64(best == wb ? bj : INT64_MAX);
            if (sel == INT64_MAX) { // no area above -1 (all NaN): the bucket's first point stands
                ax = (double)XP[s0];
                ay = (double)YP[s0];
                if (lane == 0)
                    out[k + 1] = s0;
                continue;
            }
            const int win = __builtin_ctzll(__builtin_amdgcn_ballot_w64(bj == sel));
            ax = readlane_f64(bx, win);
            ay = readlane_f64(by, win);
            if (lane == 0)
                out[k + 1] = sel;
        }
        if (lane == 0) {
            out[0] = 0;
            out[g.B + 1] = m - 1;
        }
        __threadfence_block();
        __syncthreads();
        for (int64_t i = lane; i < g.B + 2; i += kWave)
            out[i] = b.P[g.p0 + out[i]];
        __syncthreads();
    }
}

// ------------------------------------------------------------------ launches

static unsigned cap_grid(int64_t want, int64_t cap)
{
    return (unsigned)(want < 1 ? 1 : (want > cap ? cap : want));
}

hipError_t launch_batch_init(const BatchPtrs &b, hipStream_t s)
{
    hipLaunchKernelGGL(k_batch_init, dim3(cap_grid((b.n_keys + 255) / 256, 8192)), dim3(256), 0, s, b);
    return hipGetLastError();
}

hipError_t launch_batch_large(const BatchPtrs &b, int unroll, hipStream_t s)
{
    if (b.n_large_items == 0)
        return hipSuccess;
    const unsigned grid = cap_grid((b.n_large_items + 3) / 4, 0x7fffffff);
    switch (unroll) {
    case 1:
        hipLaunchKernelGGL(k_batch_large<1>, dim3(grid), dim3(256), 0, s, b);
        break;
    case 2:
        hipLaunchKernelGGL(k_batch_large<2>, dim3(grid), dim3(256), 0, s, b);
        break;
    case 8:
        hipLaunchKernelGGL(k_batch_large<8>, dim3(grid), dim3(256), 0, s, b);
        break;
    default:
        hipLaunchKernelGGL(k_batch_large<4>, dim3(grid), dim3(256), 0, s, b);
        break;
    }
    return hipGetLastError();
}

hipError_t launch_batch_small(const BatchPtrs &b, int tile, hipStream_t s)
{
    if (b.n_small_tiles == 0)
        return hipSuccess;
    const dim3 grid(cap_grid((b.n_small_tiles + kSmallTilesPerBlock - 1) / kSmallTilesPerBlock, 0x7fffffff));
    switch (tile) {
    case 2048:
        hipLaunchKernelGGL(k_batch_small<2048>, grid, dim3(kTileThreads), 0, s, b);
        break;
    case 8192:
        hipLaunchKernelGGL(k_batch_small<8192>, grid, dim3(kTileThreads), 0, s, b);
        break;
    default:
        hipLaunchKernelGGL(k_batch_small<4096>, grid, dim3(kTileThreads), 0, s, b);
        break;
    }
    return hipGetLastError();
}

int small_tile_bins(int64_t maxbin, int64_t nb, int tile)
{
    if (maxbin < 1 || maxbin > tile / 4 || nb >= ((int64_t)1 << 26))
        return 0;
    int G = 256;
    while ((int64_t)G * maxbin > tile)
        G >>= 1;
    return G;
}

hipError_t launch_minmax_small_tiles(const float *y, const Split &bins, int tile, unsigned long long *keys,
                                     hipStream_t s)
{
    const int64_t maxbin = bins.q + (bins.r ? 1 : 0);
    const int G = small_tile_bins(maxbin, bins.parts, tile);
    if (G == 0)
        return hipErrorInvalidValue;
    const int64_t n_tiles = (bins.parts + G - 1) / G;
    const dim3 grid(cap_grid((n_tiles + kSmallTilesPerBlock - 1) / kSmallTilesPerBlock, 0x7fffffff));
    switch (tile) {
    case 2048:
        hipLaunchKernelGGL(k_minmax_small_tiles<2048>, grid, dim3(kTileThreads), 0, s, y, bins, G, n_tiles, keys);
        break;
    case 8192:
        hipLaunchKernelGGL(k_minmax_small_tiles<8192>, grid, dim3(kTileThreads), 0, s, y, bins, G, n_tiles, keys);
        break;
    default:
        hipLaunchKernelGGL(k_minmax_small_tiles<4096>, grid, dim3(kTileThreads), 0, s, y, bins, G, n_tiles, keys);
        break;
    }
    return hipGetLastError();
}

hipError_t launch_batch_compact(const BatchPtrs &b, hipStream_t s)
{
    hipLaunchKernelGGL(k_batch_compact, dim3(cap_grid(b.n_segs, 16384)), dim3(kCompactThreads), 0, s, b);
    return hipGetLastError();
}

hipError_t launch_batch_means(const BatchPtrs &b, hipStream_t s)
{
    if (b.max_B <= 0)
        return hipSuccess;
    if (b.n_segs > 0x7fffffff)
        return hipErrorInvalidConfiguration;
    const dim3 grid((unsigned)b.n_segs, cap_grid((b.max_B + 255) / 256, 65535));
    hipLaunchKernelGGL(k_batch_means, grid, dim3(256), 0, s, b);
    return hipGetLastError();
}

hipError_t launch_batch_chain(const BatchPtrs &b, hipStream_t s)
{
    if (b.n_chain_units == 0)
        return hipSuccess;
    const size_t lds = seg_walk_lds_bytes(b.stage_cap_max);
    hipLaunchKernelGGL(k_batch_chain, dim3(cap_grid(b.n_chain_units, 0x7fffffff)), dim3(kSegStarts), lds, s, b);
    return hipGetLastError();
}

hipError_t launch_batch_chain_seq(const BatchPtrs &b, hipStream_t s)
{
    hipLaunchKernelGGL(k_batch_chain_seq, dim3(cap_grid(b.n_segs, 8192)), dim3(kWave), 0, s, b);
    return hipGetLastError();
}

hipError_t launch_batch_link_emit(const BatchPtrs &b, hipStream_t s)
{
    hipLaunchKernelGGL(k_batch_link_emit, dim3(cap_grid(b.n_segs, 4096)), dim3(1024), 0, s, b);
    return hipGetLastError();
}

} // namespace mmlttb
