// MinMax and MinMaxLTTB for other value types (float64 or int32 y; int64,
// float64 or implicit x). Same bins, ties and preselection as the float32
// path (section 2.2.1 MinMax, section 3); the LTTB pass runs on binary64
// coordinates, with next-bucket means from exact sums.
//
//  k_typed_bin_reduce<T, U>  one wave per (bin, chunk) work item writes that
//                            item's (min key, index, max key, index) partial
//  k_typed_bin_merge         one wave per bin merges its partials
//  k_typed_compact<XK, T>    one workgroup: sorted P = {0, n-1} + extrema,
//                            with binary64 X_P, Y_P for the LTTB pass
//  k_typed_preselect_all     P = every point (each bin holds at most one)
//  k_typed_bucket_means<XK>  one thread per bucket, exact sums in LDS rows
#include "chain_device.hpp"
#include "device_common.hpp"
#include "kernels.hpp"
#include "minmax_device.hpp"
#include "typed_device.hpp"

namespace mmlttb {

enum { kXImplicit = 0, kXInt64 = 1, kXF64 = 2 };

template <int XK>
__device__ inline double x_coord(const void *x, int64_t i)
{
    if (XK == kXInt64)
        return (double)static_cast<const int64_t *>(x)[i];
    if (XK == kXF64)
        return static_cast<const double *>(x)[i];
    return (double)i;
}

template <class T, int U>
__global__ __launch_bounds__(256) void k_typed_bin_reduce(const T *__restrict__ y, MinMaxGeom g,
                                                          TypedPartial *__restrict__ part)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int64_t item = (int64_t)blockIdx.x * (blockDim.x / kWave) + wave;
    if (item >= g.n_items)
        return;
    const int64_t b = item / g.chunks_per_bin;
    const int64_t j = item - b * g.chunks_per_bin;
    const int64_t blo = 1 + split_lo(g.bins, b);
    const int64_t bhi = 1 + split_lo(g.bins, b + 1);
    const int64_t lo = blo + j * g.chunk;
    TypedPartial r;
    r.kmin = ~0ull;
    r.imin = INT64_MAX;
    r.kmax = 0ull;
    r.imax = INT64_MAX;
    if (lo < bhi) { // else: trailing chunk of a shorter bin, an identity partial
        const int64_t hi = (lo + g.chunk < bhi) ? lo + g.chunk : bhi;
        typename ValueTraits<T>::Key kmin, kmax;
        wave_reduce_keys<T, U>(y, lo, hi, lane, kmin, r.imin, kmax, r.imax);
        r.kmin = kmin;
        r.kmax = kmax;
    }
    if (lane == 0)
        part[item] = r;
}

__global__ __launch_bounds__(256) void k_typed_bin_merge(const TypedPartial *__restrict__ part, int64_t nb,
                                                         int64_t cpb, int64_t *__restrict__ pairs)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t b = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (b >= nb)
        return;
    uint64_t kmin = ~0ull, kmax = 0ull;
    int64_t imin = INT64_MAX, imax = INT64_MAX;
    for (int64_t j = lane; j < cpb; j += kWave) {
        const TypedPartial p = part[b * cpb + j];
        if (p.kmin < kmin || (p.kmin == kmin && p.imin < imin)) {
            kmin = p.kmin;
            imin = p.imin;
        }
        if (p.kmax > kmax || (p.kmax == kmax && p.imax < imax)) {
            kmax = p.kmax;
            imax = p.imax;
        }
    }
    const uint64_t wmin = wave_min_key<uint64_t>(kmin);
    const uint64_t wmax = wave_max_key<uint64_t>(kmax);
    const int64_t i0 = wave_min_i64(kmin == wmin ? imin : INT64_MAX);
    const int64_t i1 = wave_min_i64(kmax == wmax ? imax : INT64_MAX);
    if (lane == 0) {
        pairs[2 * b] = i0;
        pairs[2 * b + 1] = i1;
    }
}

// One workgroup of 1024 threads. XD/YD may be NULL (MinMax alone).
template <int XK, class T>
__global__ __launch_bounds__(1024) void k_typed_compact(const int64_t *__restrict__ pairs, Split bins, int64_t n,
                                                        const void *__restrict__ x, const T *__restrict__ y,
                                                        int64_t *__restrict__ P, double *__restrict__ XD,
                                                        double *__restrict__ YD, int64_t *__restrict__ m_out)
{
    __shared__ int wave_tot[17];
    const int tid = threadIdx.x;
    int64_t running = 1;
    if (tid == 0) {
        P[0] = 0;
        if (XD) {
            XD[0] = x_coord<XK>(x, 0);
            YD[0] = ValueTraits<T>::widen(y[0]);
        }
    }
    const int64_t nb = bins.parts;
    for (int64_t base = 0; base < nb; base += blockDim.x) {
        const int64_t b = base + tid;
        int c = 0;
        int64_t i0 = 0, i1 = 0;
        if (b < nb) {
            const int64_t imin = pairs[2 * b], imax = pairs[2 * b + 1];
            const int64_t blo = 1 + split_lo(bins, b), bhi = 1 + split_lo(bins, b + 1);
            if (imin >= blo && imin < bhi && imax >= blo && imax < bhi) { // always, for a non-empty bin
                i0 = imin < imax ? imin : imax;
                i1 = imin < imax ? imax : imin;
                c = (imin == imax) ? 1 : 2;
            }
        }
        int total;
        const int64_t off = running + block_exclusive_scan(c, wave_tot, total);
        if (c >= 1) {
            P[off] = i0;
            if (XD) {
                XD[off] = x_coord<XK>(x, i0);
                YD[off] = ValueTraits<T>::widen(y[i0]);
            }
        }
        if (c == 2) {
            P[off + 1] = i1;
            if (XD) {
                XD[off + 1] = x_coord<XK>(x, i1);
                YD[off + 1] = ValueTraits<T>::widen(y[i1]);
            }
        }
        running += total;
    }
    if (tid == 0) {
        P[running] = n - 1;
        if (XD) {
            XD[running] = x_coord<XK>(x, n - 1);
            YD[running] = ValueTraits<T>::widen(y[n - 1]);
        }
        *m_out = running + 1;
    }
}

template <int XK, class T>
__global__ __launch_bounds__(256) void k_typed_preselect_all(int64_t n, const void *__restrict__ x,
                                                             const T *__restrict__ y, int64_t *__restrict__ P,
                                                             double *__restrict__ XD, double *__restrict__ YD,
                                                             int64_t *__restrict__ m_out)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        P[i] = i;
        if (XD) {
            XD[i] = x_coord<XK>(x, i);
            YD[i] = ValueTraits<T>::widen(y[i]);
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0)
        *m_out = n;
}

// One thread per bucket, 64 per workgroup; each thread's exact binary64
// accumulator is a row of LDS.
template <int XK>
__global__ __launch_bounds__(64) void k_typed_bucket_means(const int64_t *__restrict__ P, const void *__restrict__ x,
                                                           const double *__restrict__ YD,
                                                           const int64_t *__restrict__ m_ptr, int64_t B,
                                                           double *__restrict__ MX, double *__restrict__ MY)
{
    __shared__ int64_t rows[64 * F64ExactSum::kLimbs];
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= B)
        return;
    const int64_t m = *m_ptr;
    const Split bk = make_split(m - 2, B);
    int64_t g0, g1;
    next_bucket_range(bk, m, k, g0, g1);
    const double c = (double)(g1 - g0);
    F64ExactSum acc(rows + threadIdx.x * F64ExactSum::kLimbs);
    if (XK == kXF64) {
        acc.clear();
        for (int64_t i = g0; i < g1; ++i)
            acc.add(static_cast<const double *>(x)[P[i]]);
        MX[k] = acc.round() / c;
    } else {
        I64ExactSum sx;
        sx.clear();
        for (int64_t i = g0; i < g1; ++i)
            sx.add(XK == kXInt64 ? static_cast<const int64_t *>(x)[P[i]] : P[i]);
        MX[k] = sx.round() / c;
    }
    acc.clear();
    for (int64_t i = g0; i < g1; ++i)
        acc.add(YD[i]);
    MY[k] = acc.round() / c;
}

// ---------------------------------------------------------------- launches

template <class T>
static hipError_t launch_bin_reduce_t(const T *y, const MinMaxGeom &g, int unroll, TypedPartial *part, hipStream_t s)
{
    const int64_t blocks = (g.n_items + 3) / 4;
    if (blocks > 0x7fffffff)
        return hipErrorInvalidConfiguration;
    switch (unroll) {
    case 1:
        hipLaunchKernelGGL((k_typed_bin_reduce<T, 1>), dim3((unsigned)blocks), dim3(256), 0, s, y, g, part);
        break;
    case 2:
        hipLaunchKernelGGL((k_typed_bin_reduce<T, 2>), dim3((unsigned)blocks), dim3(256), 0, s, y, g, part);
        break;
    case 8:
        hipLaunchKernelGGL((k_typed_bin_reduce<T, 8>), dim3((unsigned)blocks), dim3(256), 0, s, y, g, part);
        break;
    default:
        hipLaunchKernelGGL((k_typed_bin_reduce<T, 4>), dim3((unsigned)blocks), dim3(256), 0, s, y, g, part);
        break;
    }
    return hipGetLastError();
}

hipError_t launch_typed_bin_reduce(int yk, const void *y, const MinMaxGeom &g, int unroll, TypedPartial *part,
                                   hipStream_t s)
{
    switch (yk) {
    case kYF32:
        return launch_bin_reduce_t(static_cast<const float *>(y), g, unroll, part, s);
    case kYF64:
        return launch_bin_reduce_t(static_cast<const double *>(y), g, unroll, part, s);
    default:
        return launch_bin_reduce_t(static_cast<const int32_t *>(y), g, unroll, part, s);
    }
}

hipError_t launch_typed_bin_merge(const TypedPartial *part, int64_t nb, int64_t cpb, int64_t *pairs, hipStream_t s)
{
    const int64_t blocks = (nb + 3) / 4;
    hipLaunchKernelGGL(k_typed_bin_merge, dim3((unsigned)blocks), dim3(256), 0, s, part, nb, cpb, pairs);
    return hipGetLastError();
}

template <int XK, class T>
static hipError_t compact_xk_t(const int64_t *pairs, const Split &bins, int64_t n, const void *x, const T *y,
                               int64_t *P, double *XD, double *YD, int64_t *m_out, bool all, hipStream_t s)
{
    if (all) {
        int64_t blocks = (n + 255) / 256;
        blocks = blocks < 1 ? 1 : (blocks > 8192 ? 8192 : blocks);
        auto kern = k_typed_preselect_all<XK, T>;
        hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(256), 0, s, n, x, y, P, XD, YD, m_out);
    } else {
        auto kern = k_typed_compact<XK, T>;
        hipLaunchKernelGGL(kern, dim3(1), dim3(1024), 0, s, pairs, bins, n, x, y, P, XD, YD, m_out);
    }
    return hipGetLastError();
}

template <int XK>
static hipError_t compact_xk(int yk, const int64_t *pairs, const Split &bins, int64_t n, const void *x, const void *y,
                             int64_t *P, double *XD, double *YD, int64_t *m_out, bool all, hipStream_t s)
{
    switch (yk) {
    case kYF32:
        return compact_xk_t<XK>(pairs, bins, n, x, static_cast<const float *>(y), P, XD, YD, m_out, all, s);
    case kYF64:
        return compact_xk_t<XK>(pairs, bins, n, x, static_cast<const double *>(y), P, XD, YD, m_out, all, s);
    default:
        return compact_xk_t<XK>(pairs, bins, n, x, static_cast<const int32_t *>(y), P, XD, YD, m_out, all, s);
    }
}

hipError_t launch_typed_compact(int xk, int yk, const int64_t *pairs, const Split &bins, int64_t n, const void *x,
                                const void *y, int64_t *P, double *XD, double *YD, int64_t *m_out, bool all,
                                hipStream_t s)
{
    switch (xk) {
    case kXInt64:
        return compact_xk<kXInt64>(yk, pairs, bins, n, x, y, P, XD, YD, m_out, all, s);
    case kXF64:
        return compact_xk<kXF64>(yk, pairs, bins, n, x, y, P, XD, YD, m_out, all, s);
    default:
        return compact_xk<kXImplicit>(yk, pairs, bins, n, x, y, P, XD, YD, m_out, all, s);
    }
}

hipError_t launch_typed_bucket_means(int xk, const int64_t *P, const void *x, const double *YD, const int64_t *m_ptr,
                                     int64_t B, double *MX, double *MY, hipStream_t s)
{
    const int64_t blocks = (B + 63) / 64;
    if (blocks > 0x7fffffff)
        return hipErrorInvalidConfiguration;
    switch (xk) {
    case kXInt64:
        hipLaunchKernelGGL(k_typed_bucket_means<kXInt64>, dim3((unsigned)blocks), dim3(64), 0, s, P, x, YD, m_ptr, B,
                           MX, MY);
        break;
    case kXF64:
        hipLaunchKernelGGL(k_typed_bucket_means<kXF64>, dim3((unsigned)blocks), dim3(64), 0, s, P, x, YD, m_ptr, B,
                           MX, MY);
        break;
    default:
        hipLaunchKernelGGL(k_typed_bucket_means<kXImplicit>, dim3((unsigned)blocks), dim3(64), 0, s, P, x, YD, m_ptr,
                           B, MX, MY);
        break;
    }
    return hipGetLastError();
}

} // namespace mmlttb
