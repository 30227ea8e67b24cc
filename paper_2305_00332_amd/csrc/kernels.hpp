// Launch interface of the libmmlttb kernels (host side of the library only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_common.hpp"

namespace mmlttb {

// Work decomposition of minmax_bin_reduce: bins.parts bins over the interior
// (bins.len = n - 2 points), each cut into chunks_per_bin items of at most
// `chunk` points (a multiple of 4 * 64 * unroll). One wave per item.
struct MinMaxGeom {
    Split bins;
    int64_t chunk;
    int64_t chunks_per_bin;
    int64_t n_items;
};

// LDS window of the sequential chain, in points.
constexpr int kChainStage = 1024;

hipError_t launch_init_keys(unsigned long long *keys, int64_t nb, hipStream_t s);
hipError_t launch_minmax_bin_reduce(const float *y, const MinMaxGeom &g, int unroll, unsigned long long *keys,
                                    hipStream_t s);
hipError_t launch_preselect_compact(const unsigned long long *keys, const Split &bins, int64_t n, const int64_t *x,
                                    const float *y, int64_t *P, int64_t *XP, float *YP, int64_t *m_out, hipStream_t s);
hipError_t launch_preselect_all(int64_t n, const int64_t *x, const float *y, int64_t *P, int64_t *XP, float *YP,
                                int64_t *m_out, hipStream_t s);
hipError_t launch_iota(int64_t *out, int64_t n, int64_t *count_out, hipStream_t s);

hipError_t launch_bucket_mean_small(const int64_t *XP, const float *YP, const int64_t *m_ptr, int64_t m_const,
                                    int64_t B, double *MX, double *MY, hipStream_t s);
hipError_t launch_bucket_mean_wide(const int64_t *X, const float *Y, int64_t m, int64_t B, double *MX, double *MY,
                                   hipStream_t s);
hipError_t launch_lttb_chain(const int64_t *XP, const float *YP, const int64_t *m_ptr, int64_t m_const, int64_t B,
                             const double *MX, const double *MY, const int64_t *Pmap, int64_t *out, hipStream_t s);
hipError_t launch_lttb_chain_wide(const int64_t *X, const float *Y, int64_t m, int64_t B, const double *MX,
                                  const double *MY, int64_t *out, hipStream_t s);

} // namespace mmlttb
