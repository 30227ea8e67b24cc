// Batched MinMaxLTTB: many series of uneven length in one call.
//
// The host plans every series into a BatchSeg (mode, bins, work ranges, pooled
// workspace slots) and copies the table into the workspace. Persistent
// kernels then walk flat work spaces; each workgroup (or wave) takes one
// contiguous range of work units, finds the series of its first unit by a
// binary search over the per-series starts and steps forward from there.
//
//   init      keys of every series to their identities, link counters to 0
//   large     series whose bins hold > kSmallBinMax points: one wave per
//             (bin, chunk) item, as in the single-series stream (16-byte
//             loads, atomic key merge)
//   small     series with small bins: a workgroup stages a tile of whole bins
//             (<= kTilePoints points) in LDS; a power-of-two lane group
//             reduces each bin and stores its keys
//   compact   one workgroup per series: P, X_P, Y_P, m (identity series write
//             their output here)
//   means     one workgroup per series: exact next-bucket means
//   chain     segmented chain: one wave per (series, chain segment) walks from
//             every start; the last wave of each series links its segments
//   chain_seq sequential chain for series whose buckets exceed kSegStarts
//   emit      one workgroup per series: picks mapped through P to the output
//
// Each series' result equals the single-series call on it alone: the same
// bins, keys, exact means and binary64 areas, evaluated in the same order.
#include "chain_device.hpp"
#include "device_common.hpp"
#include "kernels.hpp"
#include "minmax_device.hpp"

namespace mmlttb {

// Last series whose start (in one flat space) is <= i. Series with no work in
// that space start where the next series starts, so this is the owner.
template <class StartOf>
__device__ inline int64_t find_owner(const BatchSeg *segs, int64_t n_segs, int64_t i, StartOf start_of)
{
    int64_t lo = 0, hi = n_segs - 1;
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
    for (int64_t i = t; i < b.n_segs; i += stride)
        b.counter[i] = 0u;
}

template <int U>
__global__ __launch_bounds__(256) void k_batch_large(BatchPtrs b)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int64_t W = (int64_t)gridDim.x * (blockDim.x / kWave);
    const int64_t w = (int64_t)blockIdx.x * (blockDim.x / kWave) + wave;
    const int64_t total = b.n_large_items;
    const int64_t per = (total + W - 1) / W;
    const int64_t i0 = w * per, i1 = (i0 + per < total) ? i0 + per : total;
    if (i0 >= i1)
        return;
    int64_t s = find_owner(b.segs, b.n_segs, i0, [](const BatchSeg &g) { return g.li0; });
    for (int64_t i = i0; i < i1; ++i) {
        while (i >= b.segs[s].li0 + b.segs[s].ln)
            ++s;
        const BatchSeg &g = b.segs[s];
        const int64_t li = i - g.li0;
        const int64_t bb = li / g.chunks_per_bin;
        const int64_t j = li - bb * g.chunks_per_bin;
        const int64_t blo = 1 + split_lo(g.bins, bb);
        const int64_t bhi = 1 + split_lo(g.bins, bb + 1);
        const int64_t lo = blo + j * g.chunk;
        if (lo >= bhi)
            continue;
        const int64_t hi = (lo + g.chunk < bhi) ? lo + g.chunk : bhi;
        float vmin, vmax;
        int64_t imin, imax;
        wave_reduce_range<U>(b.y_base + g.offset, lo, hi, lane, vmin, imin, vmax, imax);
        if (lane == 0) {
            atomicMin(&b.keys[2 * (g.key0 + bb)], pack_min_key(vmin, imin - blo));
            atomicMax(&b.keys[2 * (g.key0 + bb) + 1], pack_max_key(vmax, imax - blo));
        }
    }
}

__global__ __launch_bounds__(kTileThreads) void k_batch_small(BatchPtrs b)
{
    __shared__ float tile[kTilePoints];
    const int tid = threadIdx.x;
    const int64_t T = gridDim.x;
    const int64_t total = b.n_small_tiles;
    const int64_t per = (total + T - 1) / T;
    const int64_t t0 = (int64_t)blockIdx.x * per, t1 = (t0 + per < total) ? t0 + per : total;
    if (t0 >= t1)
        return;
    int64_t s = find_owner(b.segs, b.n_segs, t0, [](const BatchSeg &g) { return g.ti0; });
    const float kInf = __int_as_float(0x7f800000);
    for (int64_t t = t0; t < t1; ++t) {
        while (t >= b.segs[s].ti0 + b.segs[s].tn)
            ++s;
        const BatchSeg &g = b.segs[s];
        const int G = g.tile_bins;
        const int tpb = kTileThreads / G; // lanes per bin: power of two <= 64
        const int64_t nb = g.bins.parts;
        const int64_t bb0 = (t - g.ti0) * G;
        const int64_t bb1 = (bb0 + G < nb) ? bb0 + G : nb;
        const int64_t lo = 1 + split_lo(g.bins, bb0), hi = 1 + split_lo(g.bins, bb1);
        const float *__restrict__ y = b.y_base + g.offset;
        __syncthreads(); // the previous tile's readers are done
        for (int64_t q = tid; q < hi - lo; q += kTileThreads)
            tile[q] = y[lo + q];
        __syncthreads();
        const int64_t bin = bb0 + tid / tpb;
        const int sub = tid % tpb;
        float vmin = kInf, vmax = -kInf;
        int64_t imin = INT64_MAX, imax = INT64_MAX, bl = 0;
        if (bin < bb1) {
            bl = 1 + split_lo(g.bins, bin);
            const int64_t bh = 1 + split_lo(g.bins, bin + 1);
            for (int64_t q = bl + sub; q < bh; q += tpb) { // increasing index: strict keeps the lowest
                const float v = tile[q - lo];
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
        for (int off = tpb >> 1; off >= 1; off >>= 1) {
            const float ov = __shfl_xor(vmin, off);
            const int64_t oi = __shfl_xor(imin, off);
            if (ov < vmin || (ov == vmin && oi < imin)) {
                vmin = ov;
                imin = oi;
            }
            const float ow = __shfl_xor(vmax, off);
            const int64_t oj = __shfl_xor(imax, off);
            if (ow > vmax || (ow == vmax && oj < imax)) {
                vmax = ow;
                imax = oj;
            }
        }
        if (sub == 0 && bin < bb1) {
            b.keys[2 * (g.key0 + bin)] = pack_min_key(vmin, imin - bl);
            b.keys[2 * (g.key0 + bin) + 1] = pack_max_key(vmax, imax - bl);
        }
    }
}

__global__ __launch_bounds__(1024) void k_batch_compact(BatchPtrs b)
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
            continue;
        }
        compact_keys(b.keys + 2 * g.key0, g.bins, n, x, y, P, XP, YP, b.m + s, wave_tot);
    }
}

__global__ __launch_bounds__(256) void k_batch_means(BatchPtrs b)
{
    for (int64_t s = blockIdx.x; s < b.n_segs; s += gridDim.x) {
        const BatchSeg &g = b.segs[s];
        if (g.mode == kSegIdentity)
            continue;
        const int64_t m = b.m[s];
        const Split bk = make_split(m - 2, g.B);
        for (int64_t k = threadIdx.x; k < g.B; k += blockDim.x)
            bucket_mean_one(b.XP + g.p0, b.YP + g.p0, bk, m, k, b.MX[g.b0 + k], b.MY[g.b0 + k]);
    }
}

__global__ __launch_bounds__(kSegStarts) void k_batch_chain(BatchPtrs b)
{
    extern __shared__ double lds[];
    __shared__ uint8_t F[kChaseWindow * kSegStarts];
    __shared__ unsigned int s_ticket;
    const int64_t T = gridDim.x;
    const int64_t total = b.n_chain_units;
    const int64_t per = (total + T - 1) / T;
    const int64_t u0 = (int64_t)blockIdx.x * per, u1 = (u0 + per < total) ? u0 + per : total;
    if (u0 >= u1)
        return;
    int64_t s = find_owner(b.segs, b.n_segs, u0, [](const BatchSeg &g) { return g.cw0; });
    for (int64_t u = u0; u < u1; ++u) {
        while (u >= b.segs[s].cw0 + b.segs[s].cwn)
            ++s;
        const BatchSeg &g = b.segs[s];
        const int64_t m = b.m[s];
        const Split bk = make_split(m - 2, g.B);
        uint8_t *path = b.path + (size_t)g.c0 * kSegStarts * kSegLen;
        uint8_t *finals = b.finals + (size_t)g.c0 * kSegStarts;
        __syncthreads(); // LDS of the previous unit is no longer read
        seg_walk(b.XP + g.p0, b.YP + g.p0, bk, b.MX + g.b0, b.MY + g.b0, u - g.cw0, g.stage_cap, lds, path, finals);
        __threadfence();
        __syncthreads();
        if (threadIdx.x == 0)
            s_ticket = atomicAdd(&b.counter[s], 1u);
        __syncthreads();
        if (s_ticket == (unsigned int)(g.cwn - 1)) {
            __threadfence();
            seg_link(finals, b.start + g.c0, g.cwn, F);
        }
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

__global__ __launch_bounds__(256) void k_batch_emit(BatchPtrs b)
{
    for (int64_t s = blockIdx.x; s < b.n_segs; s += gridDim.x) {
        const BatchSeg &g = b.segs[s];
        if (g.mode == kSegIdentity || g.seq)
            continue;
        const int64_t m = b.m[s];
        const Split bk = make_split(m - 2, g.B);
        const int64_t *P = b.P + g.p0;
        int64_t *out = b.out_base + g.out_offset;
        const uint8_t *path = b.path + (size_t)g.c0 * kSegStarts * kSegLen;
        for (int64_t k = threadIdx.x; k < g.B; k += blockDim.x)
            out[k + 1] = P[seg_pick(path, b.start + g.c0, bk, k)];
        if (threadIdx.x == 0) {
            out[0] = P[0];
            out[g.B + 1] = P[m - 1];
        }
    }
}

// ------------------------------------------------------------------ launches

static unsigned cap_grid(int64_t want, int64_t cap)
{
    return (unsigned)(want < 1 ? 1 : (want > cap ? cap : want));
}

hipError_t launch_batch_init(const BatchPtrs &b, hipStream_t s)
{
    const int64_t work = b.n_keys > b.n_segs ? b.n_keys : b.n_segs;
    hipLaunchKernelGGL(k_batch_init, dim3(cap_grid((work + 255) / 256, 8192)), dim3(256), 0, s, b);
    return hipGetLastError();
}

hipError_t launch_batch_large(const BatchPtrs &b, int unroll, hipStream_t s)
{
    if (b.n_large_items == 0)
        return hipSuccess;
    const unsigned grid = cap_grid((b.n_large_items + 3) / 4, 8192);
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

hipError_t launch_batch_small(const BatchPtrs &b, hipStream_t s)
{
    if (b.n_small_tiles == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_batch_small, dim3(cap_grid(b.n_small_tiles, 4096)), dim3(kTileThreads), 0, s, b);
    return hipGetLastError();
}

hipError_t launch_batch_compact(const BatchPtrs &b, hipStream_t s)
{
    hipLaunchKernelGGL(k_batch_compact, dim3(cap_grid(b.n_segs, 4096)), dim3(1024), 0, s, b);
    return hipGetLastError();
}

hipError_t launch_batch_means(const BatchPtrs &b, hipStream_t s)
{
    hipLaunchKernelGGL(k_batch_means, dim3(cap_grid(b.n_segs, 8192)), dim3(256), 0, s, b);
    return hipGetLastError();
}

hipError_t launch_batch_chain(const BatchPtrs &b, hipStream_t s)
{
    if (b.n_chain_units == 0)
        return hipSuccess;
    const size_t lds = (size_t)(2 * b.stage_cap_max + 2 * kSegLen) * sizeof(double);
    hipLaunchKernelGGL(k_batch_chain, dim3(cap_grid(b.n_chain_units, 16384)), dim3(kSegStarts), lds, s, b);
    return hipGetLastError();
}

hipError_t launch_batch_chain_seq(const BatchPtrs &b, hipStream_t s)
{
    hipLaunchKernelGGL(k_batch_chain_seq, dim3(cap_grid(b.n_segs, 8192)), dim3(kWave), 0, s, b);
    return hipGetLastError();
}

hipError_t launch_batch_emit(const BatchPtrs &b, hipStream_t s)
{
    hipLaunchKernelGGL(k_batch_emit, dim3(cap_grid(b.n_segs, 8192)), dim3(256), 0, s, b);
    return hipGetLastError();
}

} // namespace mmlttb
