// MinMax preselection kernels (section 2.2.1 MinMax; section 3 step (i)).
//
// minmax_bin_reduce streams y once. The interior points 1..n-2 are cut into
// nb equal-index bins (part b starts at 1 + floor(b*(n-2)/nb)); each bin is
// cut into work items of at most `chunk` points and one wave reduces one
// item: 16-byte loads in batches of U per lane, per-lane running min/max by
// value with the batch where each was first reached, a full-wave DPP
// reduction of the values, then a re-read of only the winning batch to find
// the lowest index holding the extreme (a wave takes items in a grid-stride
// loop when the grid is capped). The item's (value, index) pairs merge
// into the bin's two 64-bit keys with order-independent atomic min/max, so
// the result does not depend on chunking, grid size or timing; when every bin
// is a single item, the item stores its keys instead and the keys need no
// initialising launch.
//
// Key layout: high 32 bits = order key of the value (f32_order_key, -0 == +0),
// low 32 bits = offset of the index inside its bin (min key) or its
// complement (max key), so a larger value wins the max, a smaller the min,
// and among equal values the lowest index wins both.
#include "chain_device.hpp"
#include "device_common.hpp"
#include "kernels.hpp"
#include "minmax_device.hpp"

namespace mmlttb {

__global__ __launch_bounds__(256) void k_init_keys(unsigned long long *__restrict__ keys, int64_t nb,
                                                   unsigned int *__restrict__ ticket)
{
    if (ticket && blockIdx.x == 0 && threadIdx.x == 0) // for the tail kernel that follows
        *ticket = 0u;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < nb; b += stride) {
        keys[2 * b] = ~0ull;
        keys[2 * b + 1] = 0ull;
    }
}

template <int U>
__global__ __launch_bounds__(256) void k_minmax_bin_reduce(const float *__restrict__ y, MinMaxGeom g,
                                                           unsigned long long *__restrict__ keys,
                                                           unsigned int *__restrict__ ticket)
{
    if (ticket && blockIdx.x == 0 && threadIdx.x == 0) // for the tail kernel that follows
        *ticket = 0u;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x / kWave);
    const bool whole = g.chunks_per_bin == 1; // an item is a whole bin: keys stored, not merged
    for (int64_t item = (int64_t)blockIdx.x * (blockDim.x / kWave) + wave; item < g.n_items; item += waves) {
        int64_t b, j;
        if (whole) {
            b = item;
            j = 0;
        } else {
            b = item / g.chunks_per_bin;
            j = item - b * g.chunks_per_bin;
        }
        const int64_t blo = 1 + split_lo(g.bins, b);
        const int64_t bhi = 1 + split_lo(g.bins, b + 1);
        const int64_t lo = blo + j * g.chunk;
        if (lo >= bhi) { // trailing chunk of a shorter bin, or an empty bin
            if (whole && lane == 0)
                put_bin_keys(keys, b, true, ~0ull, 0ull);
            continue;
        }
        const int64_t hi = (lo + g.chunk < bhi) ? lo + g.chunk : bhi;
        float vmin, vmax;
        int64_t imin, imax;
        wave_reduce_range<U>(y, lo, hi, lane, vmin, imin, vmax, imax);
        if (lane == 0)
            put_bin_keys(keys, b, whole, pack_min_key(vmin, imin - blo), pack_max_key(vmax, imax - blo));
    }
}

// Short bins: one wave per fixed chunk of the interior, streaming across bin
// ends (wave_stream_bins, as the batched large-bin kernel), the parts merged
// into keys that start at the identities.
template <int U>
__global__ __launch_bounds__(256) void k_minmax_stream_chunks(const float *__restrict__ y, Split bins, int64_t chunk,
                                                              int64_t items, unsigned long long *__restrict__ keys)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int64_t i = (int64_t)blockIdx.x * (blockDim.x / kWave) + wave;
    if (i >= items)
        return;
    const int64_t lo = 1 + i * chunk;
    const int64_t end = 1 + bins.len;
    const int64_t hi = (lo + chunk < end) ? lo + chunk : end;
    wave_stream_bins<U>(y, lo, hi, bins, keys, lane);
}

// One workgroup of 1024 threads builds P for one series.
__global__ __launch_bounds__(1024) void k_preselect_compact(const unsigned long long *__restrict__ keys, Split bins,
                                                            int64_t n, const int64_t *__restrict__ x,
                                                            const float *__restrict__ y, int64_t *__restrict__ P,
                                                            int64_t *__restrict__ XP, float *__restrict__ YP,
                                                            int64_t *__restrict__ m_out)
{
    __shared__ int wave_tot[17];
    compact_keys(keys, bins, n, x, y, P, XP, YP, m_out, wave_tot);
}

// Compaction followed, in the same workgroup, by the next-bucket means over P
// (one thread per bucket).
__global__ __launch_bounds__(1024) void k_preselect_compact_means(
    const unsigned long long *__restrict__ keys, Split bins, int64_t n, const int64_t *__restrict__ x,
    const float *__restrict__ y, int64_t *__restrict__ P, int64_t *__restrict__ XP, float *__restrict__ YP,
    int64_t *__restrict__ m_out, int64_t B, double *__restrict__ MX, double *__restrict__ MY)
{
    __shared__ int wave_tot[17];
    __shared__ int64_t s_m;
    compact_keys(keys, bins, n, x, y, P, XP, YP, m_out, wave_tot);
    __threadfence_block();
    __syncthreads();
    if (threadIdx.x == 0)
        s_m = *m_out;
    __syncthreads();
    const int64_t m = s_m;
    const Split bk = make_split(m - 2, B);
    for (int64_t k = threadIdx.x; k < B; k += blockDim.x)
        bucket_mean_one(XP, YP, bk, m, k, MX[k], MY[k]);
}

// The whole tail of a small preselection, one workgroup per chain segment
// (buckets [g*kSegLen, (g+1)*kSegLen)), two launches per call in all: every
// workgroup counts the points each bin keeps (the same decoding as the
// compaction) into per-bin start slots in LDS, so it knows m and every
// bucket's place in P; it decodes just the points its segment reads (the
// bucket before it for the start points, its own buckets, the one after for
// the last mean), takes the next-bucket means and walks its segment as
// k_lttb_chain_seg does (section 2.2.1, LTTB). It stores the original index of
// its own buckets' points in P; the last workgroup to finish (a device-scope
// ticket, cleared by the stream kernel before this launch) links the segments
// and writes every pick.
__global__ __launch_bounds__(kTailThreads) void k_preselect_tail(
    const unsigned long long *__restrict__ keys, Split bins, int64_t n, const int64_t *__restrict__ x,
    const float *__restrict__ y, int64_t B, int stage_cap, int64_t *__restrict__ P, uint8_t *__restrict__ path,
    uint8_t *__restrict__ finals, uint8_t *__restrict__ start, unsigned int *__restrict__ ticket,
    int64_t *__restrict__ out)
{
    __shared__ int32_t cum[kTailBins + 1]; // points kept by the bins before bin b
    __shared__ int64_t sxv[kTailPts];
    __shared__ float syv[kTailPts];
    __shared__ double smx[kSegLen], smy[kSegLen];
    __shared__ int wave_tot[17];
    __shared__ int s_last;
    // dynamic LDS: the bins' keys (bin b at b + b/16, one pad entry per 16
    // bins), then the segment walk's area, then the link's window
    extern __shared__ double dyn_lds[];
    unsigned char *dyn = reinterpret_cast<unsigned char *>(dyn_lds);
    ulonglong2 *skeys = reinterpret_cast<ulonglong2 *>(dyn_lds);
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    const int64_t nb = bins.parts;
    const ulonglong2 *keys2 = reinterpret_cast<const ulonglong2 *>(keys);
    for (int64_t b = tid; b < nb; b += kTailThreads)
        skeys[b + (b >> 4)] = keys2[b];
    __syncthreads();
    constexpr int kPer = (kTailBins + kTailThreads - 1) / kTailThreads;
    int c[kPer], own = 0;
    {
        const int64_t b0 = (int64_t)tid * kPer;
        SplitWalker bw; // this thread's consecutive bins, one division in all
        bw.init(bins, b0 < nb ? b0 : nb);
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int64_t b = b0 + u;
            c[u] = 0;
            if (b < nb) {
                const int64_t blo = bw.lo, len = bw.next_lo(bins) - blo;
                const ulonglong2 kk = skeys[b + (b >> 4)];
                int64_t i0, i1;
                float v0, v1;
                c[u] = decode_bin(kk.x, kk.y, blo, len, i0, i1, v0, v1);
                bw.advance(bins);
            }
            own += c[u];
        }
    }
    int total;
    int run = block_exclusive_scan(own, wave_tot, total);
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const int64_t b = (int64_t)tid * kPer + u;
        if (b < nb)
            cum[b] = run;
        run += c[u];
    }
    if (tid == 0)
        cum[nb] = total;
    __syncthreads();
    const int64_t m = (int64_t)total + 2;
    const Split bk = make_split(m - 2, B);
    const int64_t g = blockIdx.x, k0 = g * kSegLen, k1 = (k0 + kSegLen < B) ? k0 + kSegLen : B;
    const int64_t pa = k0 == 0 ? 0 : 1 + split_lo(bk, k0 - 1);
    const int64_t pb = k1 < B ? 1 + split_lo(bk, k1 + 1) : m;
    const int64_t own0 = 1 + split_lo(bk, k0), own1 = 1 + split_lo(bk, k1);
    for (int64_t p = pa + tid; p < pb; p += kTailThreads) {
        int64_t idx;
        float yv;
        if (p == 0 || p == m - 1) {
            idx = p == 0 ? 0 : n - 1;
            yv = y[idx];
        } else {
            const int32_t q = (int32_t)(p - 1);
            int lo = 0, hi = (int)nb; // the bin of kept point q: the last b with cum[b] <= q
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (cum[mid] <= q)
                    lo = mid;
                else
                    hi = mid;
            }
            const int64_t blo = split_lo(bins, lo), len = split_lo(bins, lo + 1) - blo;
            const ulonglong2 kk = skeys[lo + (lo >> 4)];
            int64_t i0, i1;
            float v0, v1;
            (void)decode_bin(kk.x, kk.y, blo, len, i0, i1, v0, v1);
            const bool second = q > cum[lo];
            idx = second ? i1 : i0;
            yv = second ? v1 : v0;
        }
        sxv[p - pa] = x ? x[idx] : idx;
        syv[p - pa] = yv;
        if (p >= own0 && p < own1)
            P[p] = idx;
    }
    __syncthreads();
    const int64_t *XPl = sxv - pa; // indexed by position in P
    const float *YPl = syv - pa;
    for (int64_t k = k0 + tid; k < k1; k += kTailThreads)
        bucket_mean_one(XPl, YPl, bk, m, k, smx[k - k0], smy[k - k0]);
    __syncthreads();
    seg_walk(XPl, YPl, bk, smx - k0, smy - k0, g, stage_cap, dyn, path, finals, lane, wave == 0);
    __threadfence(); // this segment's path, finals and P before the ticket
    __syncthreads();
    if (tid == 0)
        s_last = atomicAdd(ticket, 1u) == gridDim.x - 1;
    __syncthreads();
    if (!s_last)
        return;
    __threadfence(); // every other segment's writes after the ticket
    const int64_t S = gridDim.x;
    seg_link(finals, start, S, dyn);
    for (int64_t k = tid; k < B; k += kTailThreads)
        out[k + 1] = P[seg_pick(path, start, bk, k)];
    if (tid == 0) {
        out[0] = 0;
        out[B + 1] = n - 1;
    }
}

// Tiled compaction, for many bins: tile t is bins [t*kCompactTileBins,
// (t+1)*kCompactTileBins), one workgroup of 1024 threads (one round of
// compact_bin_range) each. Three launches: the tiles' point counts; one
// workgroup turning them into each tile's first slot in P (after the first
// point) and writing the first and last points and m; the tiles writing P.
static_assert(kCompactTileBins == 1024 * kCompactBins, "a compaction tile is one round of 1024 threads");

__global__ __launch_bounds__(1024) void k_compact_count(const unsigned long long *__restrict__ keys, Split bins,
                                                        int64_t *__restrict__ tile_slot)
{
    __shared__ int wave_tot[17];
    const int64_t b0 = (int64_t)blockIdx.x * kCompactTileBins;
    int c = 0;
#pragma unroll
    for (int u = 0; u < kCompactBins; ++u) {
        const int64_t b = b0 + (int64_t)u * blockDim.x + threadIdx.x;
        if (b < bins.parts)
            c += bin_kept(keys, bins, b);
    }
    int total;
    (void)block_exclusive_scan(c, wave_tot, total);
    if (threadIdx.x == 0)
        tile_slot[blockIdx.x] = total;
}

__global__ __launch_bounds__(1024) void k_compact_slots(int64_t *__restrict__ tile_slot, int64_t tiles, int64_t n,
                                                        const int64_t *__restrict__ x, const float *__restrict__ y,
                                                        int64_t *__restrict__ P, int64_t *__restrict__ XP,
                                                        float *__restrict__ YP, int64_t *__restrict__ m_out)
{
    __shared__ int wave_tot[17];
    int64_t running = 1; // slot 0 is the first point
    for (int64_t base = 0; base < tiles; base += blockDim.x) {
        const int64_t t = base + threadIdx.x;
        const int c = t < tiles ? (int)tile_slot[t] : 0; // at most 2 * kCompactTileBins
        int total;
        const int off = block_exclusive_scan(c, wave_tot, total);
        if (t < tiles)
            tile_slot[t] = running + off;
        running += total;
    }
    if (threadIdx.x == 0) {
        put_end_point(0, 0, x, y, P, XP, YP);
        put_end_point(running, n - 1, x, y, P, XP, YP);
        *m_out = running + 1;
    }
}

__global__ __launch_bounds__(1024) void k_compact_tiles(const unsigned long long *__restrict__ keys, Split bins,
                                                        const int64_t *__restrict__ tile_slot,
                                                        const int64_t *__restrict__ x, int64_t *__restrict__ P,
                                                        int64_t *__restrict__ XP, float *__restrict__ YP)
{
    __shared__ int wave_tot[17];
    const int64_t b0 = (int64_t)blockIdx.x * kCompactTileBins;
    const int64_t b1 = b0 + kCompactTileBins < bins.parts ? b0 + kCompactTileBins : bins.parts;
    (void)compact_bin_range(keys, bins, b0, b1, tile_slot[blockIdx.x], x, P, XP, YP, wave_tot);
}

// ---------------------------------------------------------------- launches

hipError_t launch_init_keys(unsigned long long *keys, int64_t nb, hipStream_t s, unsigned int *ticket)
{
    int64_t blocks = (nb + 255) / 256;
    blocks = blocks < 1 ? 1 : (blocks > 4096 ? 4096 : blocks);
    hipLaunchKernelGGL(k_init_keys, dim3((unsigned)blocks), dim3(256), 0, s, keys, nb, ticket);
    return hipGetLastError();
}

hipError_t launch_minmax_bin_reduce(const float *y, const MinMaxGeom &g, int unroll, unsigned long long *keys,
                                    hipStream_t s, unsigned int *ticket)
{
    const int64_t blocks = stream_blocks(g);
    if (blocks > 0x7fffffff)
        return hipErrorInvalidConfiguration;
    switch (unroll) {
    case 1:
        hipLaunchKernelGGL(k_minmax_bin_reduce<1>, dim3((unsigned)blocks), dim3(256), 0, s, y, g, keys, ticket);
        break;
    case 2:
        hipLaunchKernelGGL(k_minmax_bin_reduce<2>, dim3((unsigned)blocks), dim3(256), 0, s, y, g, keys, ticket);
        break;
    case 8:
        hipLaunchKernelGGL(k_minmax_bin_reduce<8>, dim3((unsigned)blocks), dim3(256), 0, s, y, g, keys, ticket);
        break;
    default:
        hipLaunchKernelGGL(k_minmax_bin_reduce<4>, dim3((unsigned)blocks), dim3(256), 0, s, y, g, keys, ticket);
        break;
    }
    return hipGetLastError();
}

hipError_t launch_minmax_stream_chunks(const float *y, const Split &bins, int unroll, unsigned long long *keys,
                                      hipStream_t s)
{
    const int64_t items = (bins.len + kShortBinChunk - 1) / kShortBinChunk;
    const int64_t blocks = (items + 3) / 4;
    if (blocks > 0x7fffffff)
        return hipErrorInvalidConfiguration;
    switch (unroll) {
    case 1:
        hipLaunchKernelGGL(k_minmax_stream_chunks<1>, dim3((unsigned)blocks), dim3(256), 0, s, y, bins,
                           kShortBinChunk, items, keys);
        break;
    case 2:
        hipLaunchKernelGGL(k_minmax_stream_chunks<2>, dim3((unsigned)blocks), dim3(256), 0, s, y, bins,
                           kShortBinChunk, items, keys);
        break;
    case 8:
        hipLaunchKernelGGL(k_minmax_stream_chunks<8>, dim3((unsigned)blocks), dim3(256), 0, s, y, bins,
                           kShortBinChunk, items, keys);
        break;
    default:
        hipLaunchKernelGGL(k_minmax_stream_chunks<4>, dim3((unsigned)blocks), dim3(256), 0, s, y, bins,
                           kShortBinChunk, items, keys);
        break;
    }
    return hipGetLastError();
}

hipError_t launch_preselect_compact_means(const unsigned long long *keys, const Split &bins, int64_t n,
                                          const int64_t *x, const float *y, int64_t *P, int64_t *XP, float *YP,
                                          int64_t *m_out, int64_t B, double *MX, double *MY, hipStream_t s)
{
    hipLaunchKernelGGL(k_preselect_compact_means, dim3(1), dim3(1024), 0, s, keys, bins, n, x, y, P, XP, YP, m_out, B,
                       MX, MY);
    return hipGetLastError();
}

bool preselect_tail_fits(int64_t nb, int64_t maxb_bound)
{
    return nb <= kTailBins && (kSegLen + 2) * maxb_bound + 2 <= kTailPts;
}

hipError_t launch_preselect_tail(const unsigned long long *keys, const Split &bins, int64_t n, const int64_t *x,
                                 const float *y, int64_t B, int stage_cap, int64_t *P, uint8_t *path, uint8_t *finals,
                                 uint8_t *start, unsigned int *ticket, int64_t *out, hipStream_t s)
{
    const int64_t S = (B + kSegLen - 1) / kSegLen;
    if (S > 0x7fffffff)
        return hipErrorInvalidConfiguration;
    const int64_t nb = bins.parts;
    const size_t keyb = (size_t)(nb + nb / 16 + 1) * 16, walk = seg_walk_lds_bytes(stage_cap),
                 link = (size_t)kChaseWindow * kSegStarts;
    size_t lds = keyb > walk ? keyb : walk;
    lds = lds > link ? lds : link;
    hipLaunchKernelGGL(k_preselect_tail, dim3((unsigned)S), dim3(kTailThreads), lds, s, keys,
                       bins, n, x, y, B, stage_cap, P, path, finals, start, ticket, out);
    return hipGetLastError();
}

hipError_t launch_compact_tiled(const unsigned long long *keys, const Split &bins, int64_t n, const int64_t *x,
                                const float *y, int64_t *P, int64_t *XP, float *YP, int64_t *m_out, int64_t *tile_slot,
                                hipStream_t s)
{
    const int64_t tiles = compact_tiles(bins.parts);
    if (tiles > 0x7fffffff)
        return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(k_compact_count, dim3((unsigned)tiles), dim3(1024), 0, s, keys, bins, tile_slot);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_compact_slots, dim3(1), dim3(1024), 0, s, tile_slot, tiles, n, x, y, P, XP, YP, m_out);
    if ((e = hipGetLastError()) != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_compact_tiles, dim3((unsigned)tiles), dim3(1024), 0, s, keys, bins, tile_slot, x, P, XP, YP);
    return hipGetLastError();
}

hipError_t launch_preselect_compact(const unsigned long long *keys, const Split &bins, int64_t n, const int64_t *x,
                                    const float *y, int64_t *P, int64_t *XP, float *YP, int64_t *m_out, hipStream_t s)
{
    hipLaunchKernelGGL(k_preselect_compact, dim3(1), dim3(1024), 0, s, keys, bins, n, x, y, P, XP, YP, m_out);
    return hipGetLastError();
}

} // namespace mmlttb
