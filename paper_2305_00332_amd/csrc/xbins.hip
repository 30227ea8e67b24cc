// MinMax preselection with bins of equal x width (irregular timestamps).
//
// The interior points 1..n-2 fall into nb bins with integer x edges
// e_b = x_1 + floor(b (x_{n-1} - x_1) / nb); point i is in bin b when
// e_b <= x_i < e_{b+1}. For x_i = i these are exactly the equal-index bins.
//
//  1. k_xbin_bounds: bin b starts at the first interior position whose x
//     reaches e_b (one binary search over x per edge).
//  2. k_xbin_reduce<U>: the interior positions are cut into equal work items
//     (independent of the bins, so one long bin still spreads over many
//     waves); a wave walks the bins its item overlaps and reduces each part
//     with the MinMax stream body, merging into the bin's keys with the same
//     order-independent atomics as the equal-index stream. Empty bins (gaps
//     in x) are skipped by a search, not one by one.
//  3. k_xbin_compact: P = {0, n-1} + per-bin extrema, sorted; for MinMaxLTTB
//     also x_P, y_P and the next-bucket means. Bins may be empty, so P can
//     hold n_out points or fewer; LTTB then keeps all of P. The LTTB pass
//     runs on P padded to n_out+1 points (copies of the last point, so every
//     bucket is non-empty), and k_xbin_finish replaces its output by P itself
//     in that case.
//
// x increasing is a precondition the device does not check. Every search
// below keeps bounds[b] <= cur < bounds[b+1] for the bin it returns whatever
// x holds, and the compaction drops decoded indices outside their bin, so
// unsorted x gives wrong indices but no access out of bounds and no endless
// loop.
#include "chain_device.hpp"
#include "device_common.hpp"
#include "kernels.hpp"
#include "minmax_device.hpp"

namespace mmlttb {

// Largest b in [b_lo, nb) with bounds[b] <= p, given bounds[b_lo] <= p < bounds[nb].
__device__ inline int64_t xbin_find(const int64_t *__restrict__ bounds, int64_t b_lo, int64_t nb, int64_t p)
{
    int64_t lo = b_lo, hi = nb;
    while (hi - lo > 1) {
        const int64_t mid = lo + ((hi - lo) >> 1);
        if (bounds[mid] <= p)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(256) void k_xbin_bounds(const int64_t *__restrict__ x, int64_t n, int64_t nb,
                                                     int64_t *__restrict__ bounds)
{
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b > nb)
        return;
    if (b == 0) {
        bounds[0] = 1;
        return;
    }
    if (b == nb) {
        bounds[nb] = n - 1;
        return;
    }
    const uint64_t x1 = (uint64_t)x[1];
    const uint64_t span = (uint64_t)x[n - 1] - x1; // < 2^64 for increasing x
    const uint64_t q = span / (uint64_t)nb, r = span % (uint64_t)nb;
    // floor(b * span / nb) = b*q + floor(b*r / nb), both terms exact in 64 bits
    const int64_t e = (int64_t)(x1 + (uint64_t)b * q + ((uint64_t)b * r) / (uint64_t)nb);
    int64_t lo = 1, hi = n - 1; // first position in [1, n-1) with x >= e, else n-1
    while (lo < hi) {
        const int64_t mid = lo + ((hi - lo) >> 1);
        if (x[mid] < e)
            lo = mid + 1;
        else
            hi = mid;
    }
    bounds[b] = lo;
}

template <int U>
__global__ __launch_bounds__(256) void k_xbin_reduce(const float *__restrict__ y, const int64_t *__restrict__ bounds,
                                                     int64_t n, int64_t nb, int64_t chunk, int64_t n_items,
                                                     unsigned long long *__restrict__ keys)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int64_t item = (int64_t)blockIdx.x * (blockDim.x / kWave) + wave;
    if (item >= n_items)
        return;
    const int64_t lo = 1 + item * chunk;
    const int64_t hi = (lo + chunk < n - 1) ? lo + chunk : n - 1;
    int64_t cur = lo;
    int64_t b = xbin_find(bounds, 0, nb, cur);
    for (;;) {
        const int64_t bs = bounds[b], be = bounds[b + 1]; // bs <= cur < be
        const int64_t sh = be < hi ? be : hi;
        float vmin, vmax;
        int64_t imin, imax;
        wave_reduce_range<U>(y, cur, sh, lane, vmin, imin, vmax, imax);
        if (lane == 0) {
            atomicMin(&keys[2 * b], pack_min_key(vmin, imin - bs));
            atomicMax(&keys[2 * b + 1], pack_max_key(vmax, imax - bs));
        }
        if (sh >= hi)
            break;
        cur = sh; // == be: the next non-empty bin starts here
        b = (bounds[b + 2] > cur) ? b + 1 : xbin_find(bounds, b + 1, nb, cur);
    }
}

// One workgroup of 1024 threads. Writes P (and, when XP != NULL, x_P, y_P),
// the preselected count to *m_true and, for the LTTB pass, max(m, pad_to)
// to *m_eff with P, x_P, y_P padded by copies of the last point. With
// MX != NULL it then computes the B next-bucket means over the padded P.
__global__ __launch_bounds__(1024) void k_xbin_compact(const unsigned long long *__restrict__ keys,
                                                       const int64_t *__restrict__ bounds, int64_t nb, int64_t n,
                                                       const int64_t *__restrict__ x, const float *__restrict__ y,
                                                       int64_t *__restrict__ P, int64_t *__restrict__ XP,
                                                       float *__restrict__ YP, int64_t *__restrict__ m_true,
                                                       int64_t *__restrict__ m_eff, int64_t pad_to, int64_t B,
                                                       double *__restrict__ MX, double *__restrict__ MY)
{
    __shared__ int wave_tot[17];
    __shared__ int64_t s_m;
    const int tid = threadIdx.x;
    int64_t running = 1;
    if (tid == 0) {
        P[0] = 0;
        if (XP) {
            XP[0] = x[0];
            YP[0] = y[0];
        }
    }
    for (int64_t base = 0; base < nb; base += blockDim.x) {
        const int64_t b = base + tid;
        int c = 0;
        int64_t i0 = 0, i1 = 0;
        float v0 = 0.0f, v1 = 0.0f;
        if (b < nb) {
            const int64_t bs = bounds[b], be = bounds[b + 1];
            if (be > bs) {
                const unsigned long long kmin = keys[2 * b], kmax = keys[2 * b + 1];
                const int64_t imin = bs + min_key_offset(kmin);
                const int64_t imax = bs + max_key_offset(kmax);
                if (imin < be && imax < be) { // always, for increasing x
                    const bool lo_min = imin < imax;
                    i0 = lo_min ? imin : imax;
                    i1 = lo_min ? imax : imin;
                    v0 = key_value(lo_min ? kmin : kmax); // y from the key, not a second read
                    v1 = key_value(lo_min ? kmax : kmin);
                    c = (imin == imax) ? 1 : 2;
                }
            }
        }
        int total;
        const int64_t off = running + block_exclusive_scan(c, wave_tot, total);
        if (c >= 1) {
            P[off] = i0;
            if (XP) {
                XP[off] = x[i0];
                YP[off] = v0;
            }
        }
        if (c == 2) {
            P[off + 1] = i1;
            if (XP) {
                XP[off + 1] = x[i1];
                YP[off + 1] = v1;
            }
        }
        running += total;
    }
    const int64_t m = running + 1;
    const int64_t me = m < pad_to ? pad_to : m;
    for (int64_t i = running + tid; i < me; i += blockDim.x) {
        P[i] = n - 1;
        if (XP) {
            XP[i] = x[n - 1];
            YP[i] = y[n - 1];
        }
    }
    if (tid == 0) {
        *m_true = m;
        if (m_eff)
            *m_eff = me;
        s_m = me;
    }
    if (!MX)
        return;
    __threadfence_block();
    __syncthreads();
    const int64_t mm = s_m;
    const Split bk = make_split(mm - 2, B);
    for (int64_t k = tid; k < B; k += blockDim.x)
        bucket_mean_one(XP, YP, bk, mm, k, MX[k], MY[k]);
}

// When P holds n_out points or fewer, LTTB keeps all of them.
__global__ __launch_bounds__(256) void k_xbin_finish(const int64_t *__restrict__ P, const int64_t *__restrict__ m_true,
                                                     int64_t n_out, int64_t *__restrict__ out,
                                                     int64_t *__restrict__ count)
{
    const int64_t m = *m_true;
    if (m <= n_out) {
        for (int64_t i = threadIdx.x; i < m; i += blockDim.x)
            out[i] = P[i];
    }
    if (threadIdx.x == 0)
        *count = m < n_out ? m : n_out;
}

// ---------------------------------------------------------------- launches

hipError_t launch_xbin_bounds(const int64_t *x, int64_t n, int64_t nb, int64_t *bounds, hipStream_t s)
{
    const int64_t blocks = (nb + 1 + 255) / 256;
    hipLaunchKernelGGL(k_xbin_bounds, dim3((unsigned)blocks), dim3(256), 0, s, x, n, nb, bounds);
    return hipGetLastError();
}

hipError_t launch_xbin_reduce(const float *y, const int64_t *bounds, int64_t n, int64_t nb, int64_t chunk,
                              int unroll, unsigned long long *keys, hipStream_t s)
{
    const int64_t n_items = (n - 2 + chunk - 1) / chunk;
    const int64_t blocks = (n_items + 3) / 4;
    if (blocks > 0x7fffffff)
        return hipErrorInvalidConfiguration;
    switch (unroll) {
    case 1:
        hipLaunchKernelGGL(k_xbin_reduce<1>, dim3((unsigned)blocks), dim3(256), 0, s, y, bounds, n, nb, chunk,
                           n_items, keys);
        break;
    case 2:
        hipLaunchKernelGGL(k_xbin_reduce<2>, dim3((unsigned)blocks), dim3(256), 0, s, y, bounds, n, nb, chunk,
                           n_items, keys);
        break;
    case 8:
        hipLaunchKernelGGL(k_xbin_reduce<8>, dim3((unsigned)blocks), dim3(256), 0, s, y, bounds, n, nb, chunk,
                           n_items, keys);
        break;
    default:
        hipLaunchKernelGGL(k_xbin_reduce<4>, dim3((unsigned)blocks), dim3(256), 0, s, y, bounds, n, nb, chunk,
                           n_items, keys);
        break;
    }
    return hipGetLastError();
}

hipError_t launch_xbin_compact(const unsigned long long *keys, const int64_t *bounds, int64_t nb, int64_t n,
                               const int64_t *x, const float *y, int64_t *P, int64_t *XP, float *YP, int64_t *m_true,
                               int64_t *m_eff, int64_t pad_to, int64_t B, double *MX, double *MY, hipStream_t s)
{
    hipLaunchKernelGGL(k_xbin_compact, dim3(1), dim3(1024), 0, s, keys, bounds, nb, n, x, y, P, XP, YP, m_true, m_eff,
                       pad_to, B, MX, MY);
    return hipGetLastError();
}

hipError_t launch_xbin_finish(const int64_t *P, const int64_t *m_true, int64_t n_out, int64_t *out, int64_t *count,
                              hipStream_t s)
{
    hipLaunchKernelGGL(k_xbin_finish, dim3(1), dim3(256), 0, s, P, m_true, n_out, out, count);
    return hipGetLastError();
}

} // namespace mmlttb
