// LTTB kernels (section 2.2.1 LTTB; Fig. 3), run either on the MinMax
// preselection (section 3 step (ii)) or on a whole series (the comparator).
//
// Points are addressed by position 0..m-1 in the array LTTB runs on; X is the
// raw int64 abscissa (or the position itself when XP is NULL: implicit x) and
// Y the float32 ordinate. Interior bucket k (0 <= k < B = n_out-2) holds
// positions [1 + floor(k (m-2)/B), 1 + floor((k+1) (m-2)/B)).
//
// bucket_mean: for bucket k the mean of bucket k+1 (the last point alone for
// k = B-1), as exact sums of X and of Y each rounded once to binary64, then
// one binary64 division by the count.
//
// lttb_chain: the sequential pass. a = position 0; for each bucket in order
// the candidate with the largest doubled area
// |(Xa - MX)(Yj - Ya) - (Xa - Xj)(MY - Ya)| (binary64, no contraction) wins,
// the lowest position on ties, and becomes a.
#include "chain_device.hpp"
#include "device_common.hpp"
#include "kernels.hpp"

namespace mmlttb {

// ------------------------------------------------------------------ identity

__global__ __launch_bounds__(256) void k_iota(int64_t *__restrict__ out, int64_t n, int64_t *__restrict__ count_out)
{
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        out[i] = i;
    if (count_out && blockIdx.x == 0 && threadIdx.x == 0)
        *count_out = n;
}

// Preselection that keeps every point (each MinMax bin holds at most one point).
__global__ __launch_bounds__(256) void k_preselect_all(int64_t n, const int64_t *__restrict__ x,
                                                       const float *__restrict__ y, int64_t *__restrict__ P,
                                                       int64_t *__restrict__ XP, float *__restrict__ YP,
                                                       int64_t *__restrict__ m_out)
{
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        P[i] = i;
        XP[i] = x ? x[i] : i;
        YP[i] = y[i];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0)
        *m_out = n;
}

// ------------------------------------------------------------------ means

// One thread per bucket (preselected points: a handful per bucket).
__global__ __launch_bounds__(256) void k_bucket_mean_small(const int64_t *__restrict__ XP, const float *__restrict__ YP,
                                                           const int64_t *__restrict__ m_ptr, int64_t m_const,
                                                           int64_t B, double *__restrict__ MX,
                                                           double *__restrict__ MY)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= B)
        return;
    const int64_t m = m_ptr ? *m_ptr : m_const;
    const Split bk = make_split(m - 2, B);
    bucket_mean_one(XP, YP, bk, m, k, MX[k], MY[k]);
}

// One workgroup (256 threads) per bucket (whole-series LTTB: large buckets).
// Wide buckets: one workgroup per bucket k sums bucket k+1 (16-byte loads,
// 8 points per thread in flight). With YR != NULL it also records the y range
// of the bucket it reads (YR[k + 1]; workgroup 0 adds YR[0] by one more
// pass), which the table form of the chain uses.
__global__ __launch_bounds__(256) void k_bucket_mean_wide(const int64_t *__restrict__ X, const float *__restrict__ Y,
                                                          int64_t m, int64_t B, double *__restrict__ MX,
                                                          double *__restrict__ MY, float2 *__restrict__ YR)
{
    __shared__ BlockMeanLds sm;
    __shared__ float s_lo[4], s_hi[4];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const Split bk = make_split(m - 2, B);
    const float kInf = __int_as_float(0x7f800000);
    // the block's y range from per-thread lo, hi into *out (all threads call)
    auto yrange = [&](float lo, float hi, float2 *out) {
        lo = wave_min_f32(lo);
        hi = wave_max_f32(hi);
        if (lane == 0) {
            s_lo[wid] = lo;
            s_hi[wid] = hi;
        }
        __syncthreads();
        if (tid == 0) {
            for (int w = 1; w < (int)(blockDim.x >> 6); ++w) {
                lo = fminf(lo, s_lo[w]);
                hi = fmaxf(hi, s_hi[w]);
            }
            *out = make_float2(lo, hi);
        }
        __syncthreads();
    };
    if (YR && blockIdx.x == 0) { // bucket 0, which no mean reads
        const int64_t g0 = 1, g1 = 1 + split_lo(bk, 1);
        float lo = kInf, hi = -kInf;
        for (int64_t i = g0 + tid; i < g1; i += blockDim.x) {
            lo = fminf(lo, Y[i]);
            hi = fmaxf(hi, Y[i]);
        }
        yrange(lo, hi, &YR[0]);
    }
    for (int64_t k = blockIdx.x; k < B; k += gridDim.x) {
        int64_t g0, g1;
        next_bucket_range(bk, m, k, g0, g1);
        I64ExactSum sx;
        F32ExactSum sy;
        sx.clear();
        sy.clear();
        float lo = kInf, hi = -kInf;
        scan_groups<2>(X, Y, g0, g1, tid, (int)blockDim.x, [&](int64_t, int64_t x, float y) {
            sx.add(x);
            sy.add(y);
            lo = fminf(lo, y);
            hi = fmaxf(hi, y);
        });
        if (YR && k + 1 < B)
            yrange(lo, hi, &YR[k + 1]);
        block_store_mean(sx, sy, g1 - g0, sm, &MX[k], &MY[k]);
    }
}

// ------------------------------------------------------------------ chain

// Sequential chain in one workgroup of 256 threads. Buckets are walked in
// groups whose points fit an LDS window; waves 1-3 stage the next group's
// points (as binary64) and means into the other LDS buffer while wave 0
// walks the current group: lane l takes candidate s_k + l (+64, ...), the
// wave takes the largest area (DPP), then the lowest position holding it
// (ballot), and the winner's coordinates move to the next step through
// readlane. Buckets wider than the window fall back to direct global reads.
// Positions are written to out[] during the walk and mapped through Pmap
// (when given) once the walk is over.
template <class XT, class YT>
__global__ __launch_bounds__(256) void k_lttb_chain(const XT *__restrict__ XP, const YT *__restrict__ YP,
                                                    const int64_t *__restrict__ m_ptr, int64_t m_const, int64_t B,
                                                    const double *__restrict__ MX, const double *__restrict__ MY,
                                                    const int64_t *__restrict__ Pmap, int64_t *__restrict__ out)
{
    __shared__ double sx[2][kChainStage], sy[2][kChainStage];
    __shared__ double smx[2][kChainStage / 2], smy[2][kChainStage / 2];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int64_t m = m_ptr ? *m_ptr : m_const;
    const Split bk = make_split(m - 2, B);
    const int64_t maxb = bk.q + (bk.r ? 1 : 0);
    const bool staged = maxb <= kChainStage;
    int64_t GB = staged ? (int64_t)kChainStage / maxb : 0;
    GB = GB > kChainStage / 2 ? kChainStage / 2 : GB;
    const int64_t ngroups = staged ? (B + GB - 1) / GB : 0;

    auto stage = [&](int64_t grp, int buf, int t0, int nt) {
        const int64_t k0 = grp * GB, k1 = (k0 + GB < B) ? k0 + GB : B;
        const int64_t p0 = 1 + split_lo(bk, k0), p1 = 1 + split_lo(bk, k1);
        for (int64_t p = p0 + t0; p < p1; p += nt) {
            sx[buf][p - p0] = (double)(XP ? XP[p] : p);
            sy[buf][p - p0] = (double)YP[p];
        }
        for (int64_t k = k0 + t0; k < k1; k += nt) {
            smx[buf][k - k0] = MX[k];
            smy[buf][k - k0] = MY[k];
        }
    };

    double ax = (double)(XP ? XP[0] : 0);
    double ay = (double)YP[0];
    SplitWalker w;
    w.init(bk, 0);

    // one chain step over positions [s0, s1) given a fetch of candidate j
    auto step = [&](int64_t s0, int64_t s1, double mx, double my, auto fetch) -> int64_t {
        const int64_t cnt = s1 - s0;
        double best = -1.0, bx = 0.0, by = 0.0;
        int64_t bj = INT64_MAX;
        for (int64_t off = lane; off < cnt; off += kWave) {
            double xj, yj;
            fetch(s0 + off, xj, yj);
            double ar = lttb_area2(ax, ay, xj, yj, mx, my);
            // a lane's first candidate stands until an area beats -1, so a
            // bucket whose areas are all NaN (overflowing binary64 means)
            // still yields its first point
            if (ar > best || bj == INT64_MAX) {
                best = ar > best ? ar : best;
                bj = s0 + off;
                bx = xj;
                by = yj;
            }
        }
        const double wb = wave_max_f64(best);
        int64_t sel;
        int win;
        if (cnt <= kWave) {
            // lane order is position order: the lowest lane holding the max wins
            unsigned long long mask = __builtin_amdgcn_ballot_w64(best == wb);
            win = __builtin_ctzll(mask);
            sel = s0 + win;
        } else {
            sel = wave_min_i64(best == wb ? bj : INT64_MAX);
            unsigned long long mask = __builtin_amdgcn_ballot_w64(bj == sel);
            win = __builtin_ctzll(mask);
        }
        ax = readlane_f64(bx, win);
        ay = readlane_f64(by, win);
        return sel;
    };

    if (staged) {
        stage(0, 0, tid, blockDim.x);
        __syncthreads();
        for (int64_t g = 0; g < ngroups; ++g) {
            const int buf = (int)(g & 1);
            if (wid != 0) {
                if (g + 1 < ngroups)
                    stage(g + 1, buf ^ 1, tid - kWave, blockDim.x - kWave);
            } else {
                const int64_t k0 = g * GB, k1 = (k0 + GB < B) ? k0 + GB : B;
                const int64_t p0 = 1 + w.lo;
                for (int64_t k = k0; k < k1; ++k) {
                    const int64_t s0 = 1 + w.lo, s1 = 1 + w.next_lo(bk);
                    w.advance(bk);
                    auto fetch = [&](int64_t j, double &xj, double &yj) {
                        xj = sx[buf][j - p0];
                        yj = sy[buf][j - p0];
                    };
                    const int64_t sel = step(s0, s1, smx[buf][k - k0], smy[buf][k - k0], fetch);
                    if (lane == 0)
                        out[k + 1] = sel;
                }
            }
            __syncthreads();
        }
    } else if (wid == 0) {
        for (int64_t k = 0; k < B; ++k) {
            const int64_t s0 = 1 + w.lo, s1 = 1 + w.next_lo(bk);
            w.advance(bk);
            auto fetch = [&](int64_t j, double &xj, double &yj) {
                xj = (double)(XP ? XP[j] : j);
                yj = (double)YP[j];
            };
            const int64_t sel = step(s0, s1, MX[k], MY[k], fetch);
            if (lane == 0)
                out[k + 1] = sel;
        }
    }
    if (tid == 0) {
        out[0] = 0;
        out[B + 1] = m - 1;
    }
    if (Pmap) {
        __threadfence_block();
        __syncthreads();
        for (int64_t i = tid; i < B + 2; i += blockDim.x)
            out[i] = Pmap[out[i]];
    }
}

// Segmented chain (same picks as k_lttb_chain, in O(B / kSegLen + kSegLen)
// dependent steps instead of B). Buckets are cut into segments of kSegLen.
// k_lttb_chain_seg (one wave per segment) walks each segment from every
// possible start point (seg_walk); k_lttb_chain_link_emit (one workgroup)
// then follows the true start from point 0 through the segments (seg_link)
// and writes every pick, mapped through Pmap when given.
template <class Args>
__global__ __launch_bounds__(kSegStarts) void k_lttb_chain_seg(Args a)
{
    extern __shared__ double lds[];
    const int64_t m = a.m_ptr ? *a.m_ptr : a.m_const;
    const Split bk = make_split(m - 2, a.B);
    seg_walk(a.XP, a.YP, bk, a.MX, a.MY, (int64_t)blockIdx.x, a.stage_cap, reinterpret_cast<unsigned char *>(lds), a.path,
             a.finals, (int)threadIdx.x);
}

// Two-level link, step 1: chunk c's composed map, lane l following start
// lane l through the chunk's transitions (staged in LDS).
__global__ __launch_bounds__(kSegStarts) void k_link_chunk_maps(const uint8_t *__restrict__ finals, int64_t S,
                                                               uint8_t *__restrict__ maps)
{
    __shared__ uint8_t F[kLinkChunk * kSegStarts];
    const int64_t t0 = (int64_t)blockIdx.x * kLinkChunk;
    const int nt = (int)((t0 + kLinkChunk < S - 1) ? kLinkChunk : S - 1 - t0);
    for (int q = threadIdx.x; q < nt * kSegStarts; q += blockDim.x)
        F[q] = finals[t0 * kSegStarts + q];
    __syncthreads();
    int cur = threadIdx.x;
    for (int t = 0; t < nt; ++t)
        cur = F[t * kSegStarts + cur];
    maps[(int64_t)blockIdx.x * kSegStarts + threadIdx.x] = (uint8_t)cur;
}

// Step 2: the chain over the chunk maps from lane 0 (seg_link on them).
__global__ __launch_bounds__(1024) void k_link_chunk_starts(const uint8_t *__restrict__ maps, int64_t chunks,
                                                            uint8_t *__restrict__ cstart)
{
    __shared__ uint8_t F[kChaseWindow * kSegStarts];
    seg_link(maps, cstart, chunks + 1, F);
}

// Step 3: chunk c's segment starts from its known start.
__global__ __launch_bounds__(kSegStarts) void k_link_chunk_fill(const uint8_t *__restrict__ finals, int64_t S,
                                                               const uint8_t *__restrict__ cstart,
                                                               uint8_t *__restrict__ start)
{
    __shared__ uint8_t F[kLinkChunk * kSegStarts];
    const int64_t t0 = (int64_t)blockIdx.x * kLinkChunk;
    const int nt = (int)((t0 + kLinkChunk < S - 1) ? kLinkChunk : S - 1 - t0);
    for (int q = threadIdx.x; q < nt * kSegStarts; q += blockDim.x)
        F[q] = finals[t0 * kSegStarts + q];
    __syncthreads();
    if (threadIdx.x == 0) {
        int cur = cstart[blockIdx.x];
        if (blockIdx.x == 0)
            start[0] = (uint8_t)cur;
        for (int t = 0; t < nt; ++t) {
            cur = F[t * kSegStarts + cur];
            start[t0 + t + 1] = (uint8_t)cur;
        }
    }
}

template <class Args>
__global__ __launch_bounds__(1024) void k_lttb_chain_link_emit(Args a, const int64_t *__restrict__ Pmap,
                                                               int64_t *__restrict__ out)
{
    __shared__ uint8_t F[kChaseWindow * kSegStarts];
    const int64_t m = a.m_ptr ? *a.m_ptr : a.m_const;
    const Split bk = make_split(m - 2, a.B);
    seg_link(a.finals, a.start, a.S, F);
    for (int64_t k = threadIdx.x; k < a.B; k += blockDim.x) {
        const int64_t sel = seg_pick(a.path, a.start, bk, k);
        out[k + 1] = Pmap ? Pmap[sel] : sel;
    }
    if (threadIdx.x == 0) {
        out[0] = Pmap ? Pmap[0] : 0;
        out[a.B + 1] = Pmap ? Pmap[m - 1] : m - 1;
    }
}

// After the two-level link: every pick written by a grid over the buckets.
template <class Args>
__global__ __launch_bounds__(256) void k_lttb_chain_emit(Args a, const int64_t *__restrict__ Pmap,
                                                         int64_t *__restrict__ out)
{
    const int64_t m = a.m_ptr ? *a.m_ptr : a.m_const;
    const Split bk = make_split(m - 2, a.B);
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < a.B) {
        const int64_t sel = seg_pick(a.path, a.start, bk, k);
        out[k + 1] = Pmap ? Pmap[sel] : sel;
    }
    if (k == 0) {
        out[0] = Pmap ? Pmap[0] : 0;
        out[a.B + 1] = Pmap ? Pmap[m - 1] : m - 1;
    }
}

// Whole-series chain for wide buckets: one workgroup of 1024 threads computes
// each bucket's areas together; per-wave winners meet in LDS.
__global__ __launch_bounds__(1024) void k_lttb_chain_wide(const int64_t *__restrict__ X, const float *__restrict__ Y,
                                                          int64_t m, int64_t B, const double *__restrict__ MX,
                                                          const double *__restrict__ MY, int64_t *__restrict__ out)
{
    __shared__ double s_area[16], s_x[16], s_y[16];
    __shared__ int64_t s_idx[16];
    __shared__ double s_ax, s_ay;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int nw = blockDim.x >> 6;
    const Split bk = make_split(m - 2, B);
    double ax = (double)(X ? X[0] : 0), ay = (double)Y[0];
    SplitWalker w;
    w.init(bk, 0);
    for (int64_t k = 0; k < B; ++k) {
        const int64_t s0 = 1 + w.lo, s1 = 1 + w.next_lo(bk);
        w.advance(bk);
        const double mx = MX[k], my = MY[k];
        double best = -1.0, bx = 0.0, by = 0.0;
        int64_t bj = INT64_MAX;
        for (int64_t j = s0 + tid; j < s1; j += blockDim.x) {
            const double xj = (double)(X ? X[j] : j);
            const double yj = (double)Y[j];
            const double ar = lttb_area2(ax, ay, xj, yj, mx, my);
            if (ar > best) {
                best = ar;
                bj = j;
                bx = xj;
                by = yj;
            }
        }
        const double wb = wave_max_f64(best);
        const int64_t wsel = wave_min_i64(best == wb ? bj : INT64_MAX);
        const unsigned long long mask = __builtin_amdgcn_ballot_w64(bj == wsel && best == wb);
        if (mask != 0ull) {
            const int win = __builtin_ctzll(mask);
            const double wx = readlane_f64(bx, win), wy = readlane_f64(by, win);
            if (lane == 0) {
                s_area[wid] = wb;
                s_idx[wid] = wsel;
                s_x[wid] = wx;
                s_y[wid] = wy;
            }
        } else if (lane == 0) {
            s_area[wid] = -1.0;
            s_idx[wid] = INT64_MAX;
        }
        __syncthreads();
        if (tid == 0) {
            double ba = -1.0;
            int64_t bi = INT64_MAX;
            int bw = 0;
            for (int q = 0; q < nw; ++q) {
                const double a = s_area[q];
                const int64_t i = s_idx[q];
                if (a > ba || (a == ba && i < bi)) {
                    ba = a;
                    bi = i;
                    bw = q;
                }
            }
            if (bi == INT64_MAX) { // no area above -1 (all NaN): the bucket's first point stands
                bi = s0;
                s_ax = (double)(X ? X[s0] : s0);
                s_ay = (double)Y[s0];
            } else {
                s_ax = s_x[bw];
                s_ay = s_y[bw];
            }
            out[k + 1] = bi;
        }
        __syncthreads();
        ax = s_ax;
        ay = s_ay;
        __syncthreads();
    }
    if (tid == 0) {
        out[0] = 0;
        out[B + 1] = m - 1;
    }
}

// ------------------------------------------------------------------ launches

static unsigned grid_for(int64_t n, int threads, int64_t cap)
{
    int64_t b = (n + threads - 1) / threads;
    b = b < 1 ? 1 : (b > cap ? cap : b);
    return (unsigned)b;
}

hipError_t launch_iota(int64_t *out, int64_t n, int64_t *count_out, hipStream_t s)
{
    hipLaunchKernelGGL(k_iota, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, out, n, count_out);
    return hipGetLastError();
}

hipError_t launch_preselect_all(int64_t n, const int64_t *x, const float *y, int64_t *P, int64_t *XP, float *YP,
                                int64_t *m_out, hipStream_t s)
{
    hipLaunchKernelGGL(k_preselect_all, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, n, x, y, P, XP, YP, m_out);
    return hipGetLastError();
}

hipError_t launch_bucket_mean_small(const int64_t *XP, const float *YP, const int64_t *m_ptr, int64_t m_const,
                                    int64_t B, double *MX, double *MY, hipStream_t s)
{
    hipLaunchKernelGGL(k_bucket_mean_small, dim3(grid_for(B, 256, 1 << 30)), dim3(256), 0, s, XP, YP, m_ptr, m_const,
                       B, MX, MY);
    return hipGetLastError();
}

hipError_t launch_bucket_mean_wide(const int64_t *X, const float *Y, int64_t m, int64_t B, double *MX, double *MY,
                                   float2 *YR, hipStream_t s)
{
    hipLaunchKernelGGL(k_bucket_mean_wide, dim3(grid_for(B, 1, 65536)), dim3(256), 0, s, X, Y, m, B, MX, MY, YR);
    return hipGetLastError();
}

template <class Args>
static hipError_t launch_chain_seg_impl(const Args &a, const int64_t *Pmap, int64_t *out, hipStream_t s)
{
    if (a.S > 0x7fffffff)
        return hipErrorInvalidConfiguration;
    const size_t lds = seg_walk_lds_bytes(a.stage_cap);
    hipLaunchKernelGGL(k_lttb_chain_seg<Args>, dim3((unsigned)a.S), dim3(kSegStarts), lds, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    const bool two_level = a.S > kTwoLevelLink;
    if (two_level) {
        const int64_t chunks = (a.S - 1 + kLinkChunk - 1) / kLinkChunk;
        uint8_t *maps = a.start + seg_maps_offset(a.S), *cstart = maps + chunks * kSegStarts;
        hipLaunchKernelGGL(k_link_chunk_maps, dim3((unsigned)chunks), dim3(kSegStarts), 0, s, a.finals, a.S, maps);
        if ((e = hipGetLastError()) != hipSuccess)
            return e;
        hipLaunchKernelGGL(k_link_chunk_starts, dim3(1), dim3(1024), 0, s, maps, chunks, cstart);
        if ((e = hipGetLastError()) != hipSuccess)
            return e;
        hipLaunchKernelGGL(k_link_chunk_fill, dim3((unsigned)chunks), dim3(kSegStarts), 0, s, a.finals, a.S, cstart,
                           a.start);
        if ((e = hipGetLastError()) != hipSuccess)
            return e;
    }
    if (two_level)
        hipLaunchKernelGGL(k_lttb_chain_emit<Args>, dim3(grid_for(a.B, 256, 1 << 30)), dim3(256), 0, s, a, Pmap, out);
    else
        hipLaunchKernelGGL(k_lttb_chain_link_emit<Args>, dim3(1), dim3(1024), 0, s, a, Pmap, out);
    return hipGetLastError();
}

hipError_t launch_lttb_chain_seg(const SegChainArgs &a, const int64_t *Pmap, int64_t *out, hipStream_t s)
{
    return launch_chain_seg_impl(a, Pmap, out, s);
}

hipError_t launch_lttb_chain_seg(const SegChainArgsD &a, const int64_t *Pmap, int64_t *out, hipStream_t s)
{
    return launch_chain_seg_impl(a, Pmap, out, s);
}

hipError_t launch_lttb_chain(const int64_t *XP, const float *YP, const int64_t *m_ptr, int64_t m_const, int64_t B,
                             const double *MX, const double *MY, const int64_t *Pmap, int64_t *out, hipStream_t s)
{
    auto kern = k_lttb_chain<int64_t, float>;
    hipLaunchKernelGGL(kern, dim3(1), dim3(256), 0, s, XP, YP, m_ptr, m_const, B, MX, MY, Pmap, out);
    return hipGetLastError();
}

hipError_t launch_lttb_chain(const double *XP, const double *YP, const int64_t *m_ptr, int64_t m_const, int64_t B,
                             const double *MX, const double *MY, const int64_t *Pmap, int64_t *out, hipStream_t s)
{
    auto kern = k_lttb_chain<double, double>;
    hipLaunchKernelGGL(kern, dim3(1), dim3(256), 0, s, XP, YP, m_ptr, m_const, B, MX, MY, Pmap, out);
    return hipGetLastError();
}

hipError_t launch_lttb_chain_wide(const int64_t *X, const float *Y, int64_t m, int64_t B, const double *MX,
                                  const double *MY, int64_t *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_lttb_chain_wide, dim3(1), dim3(1024), 0, s, X, Y, m, B, MX, MY, out);
    return hipGetLastError();
}

} // namespace mmlttb
