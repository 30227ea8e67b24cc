// The other downsamplers of Table 1 on the MinMax stream (section 2.2.1).
//
// M4 keeps, per equal-index bin over all points [0, n), the first and the
// last point and the points holding the minimum and the maximum (lowest index
// on ties). Its stream is the MinMax stream with the bins starting at point 0
// instead of point 1: one wave per (bin, chunk) work item, the same packed
// 64-bit keys and atomic merge, so the result does not depend on chunking.
// The first and last points of a bin follow from the bin boundaries and need
// no load. The compaction then writes each bin's (up to) four indices in
// index order; bins are disjoint and ordered, so the output is sorted.
//
// EveryNth keeps n_out evenly spaced indices floor(k n / n_out) and reads no
// data at all.
#include "device_common.hpp"
#include "kernels.hpp"
#include "minmax_device.hpp"

namespace mmlttb {

template <int U>
__global__ __launch_bounds__(256) void k_m4_bin_reduce(const float *__restrict__ y, MinMaxGeom g,
                                                       unsigned long long *__restrict__ keys)
{
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
        const int64_t blo = split_lo(g.bins, b);
        const int64_t bhi = split_lo(g.bins, b + 1);
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

// One workgroup of 1024 threads; one thread per bin and round.
__global__ __launch_bounds__(1024) void k_m4_compact(const unsigned long long *__restrict__ keys, Split bins,
                                                     int64_t *__restrict__ out, int64_t *__restrict__ count)
{
    __shared__ int wave_tot[17];
    const int64_t nb = bins.parts;
    int64_t running = 0;
    for (int64_t base = 0; base < nb; base += blockDim.x) {
        const int64_t b = base + threadIdx.x;
        int c = 0;
        int64_t lo = 0, a0 = 0, a1 = 0, last = 0;
        bool k0 = false, k1 = false, k2 = false;
        if (b < nb) {
            lo = split_lo(bins, b);
            last = split_lo(bins, b + 1) - 1;
            const int64_t len = last - lo + 1;
            int64_t omin = min_key_offset(keys[2 * b]), omax = max_key_offset(keys[2 * b + 1]);
            omin = omin < len ? omin : 0; // keys always decode inside their bin
            omax = omax < len ? omax : 0;
            const int64_t imin = lo + omin, imax = lo + omax;
            a0 = imin < imax ? imin : imax;
            a1 = imin < imax ? imax : imin;
            // lo <= a0 <= a1 <= last: keep each value that differs from the one before
            k0 = a0 != lo;
            k1 = a1 != a0;
            k2 = last != a1;
            c = 1 + (int)k0 + (int)k1 + (int)k2;
        }
        int total;
        int64_t off = running + block_exclusive_scan(c, wave_tot, total);
        if (c > 0) {
            out[off++] = lo;
            if (k0)
                out[off++] = a0;
            if (k1)
                out[off++] = a1;
            if (k2)
                out[off++] = last;
        }
        running += total;
    }
    if (threadIdx.x == 0)
        *count = running;
}

__global__ __launch_bounds__(256) void k_everynth(Split s, int64_t *__restrict__ out)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < s.parts; k += stride)
        out[k] = split_lo(s, k);
}

// ---------------------------------------------------------------- launches

hipError_t launch_m4_bin_reduce(const float *y, const MinMaxGeom &g, int unroll, unsigned long long *keys,
                                hipStream_t s)
{
    const int64_t blocks = stream_blocks(g);
    if (blocks > 0x7fffffff)
        return hipErrorInvalidConfiguration;
    switch (unroll) {
    case 1:
        hipLaunchKernelGGL(k_m4_bin_reduce<1>, dim3((unsigned)blocks), dim3(256), 0, s, y, g, keys);
        break;
    case 2:
        hipLaunchKernelGGL(k_m4_bin_reduce<2>, dim3((unsigned)blocks), dim3(256), 0, s, y, g, keys);
        break;
    case 8:
        hipLaunchKernelGGL(k_m4_bin_reduce<8>, dim3((unsigned)blocks), dim3(256), 0, s, y, g, keys);
        break;
    default:
        hipLaunchKernelGGL(k_m4_bin_reduce<4>, dim3((unsigned)blocks), dim3(256), 0, s, y, g, keys);
        break;
    }
    return hipGetLastError();
}

hipError_t launch_m4_compact(const unsigned long long *keys, const Split &bins, int64_t *out, int64_t *count,
                             hipStream_t s)
{
    hipLaunchKernelGGL(k_m4_compact, dim3(1), dim3(1024), 0, s, keys, bins, out, count);
    return hipGetLastError();
}

hipError_t launch_everynth(int64_t n, int64_t n_out, int64_t *out, hipStream_t s)
{
    const Split sp = make_split(n, n_out);
    int64_t blocks = (n_out + 255) / 256;
    blocks = blocks < 1 ? 1 : (blocks > 4096 ? 4096 : blocks);
    hipLaunchKernelGGL(k_everynth, dim3((unsigned)blocks), dim3(256), 0, s, sp, out);
    return hipGetLastError();
}

} // namespace mmlttb
