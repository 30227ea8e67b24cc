// C ABI of libmmlttb: single-series, typed, x-width, simplifier and
// downsampler entry points, tuning and profiling (batched calls in
// api_batched.hip; shared host code in host.hip).
#include <stdio.h>
#include <string.h>

#include "errors.hpp"
#include "host.hpp"

using namespace mmlttb;
using namespace mmlttb::host;

extern "C" {

const char *mmlttb_version(void) { return "libmmlttb 0.1.0 (gfx950)"; }

const char *mmlttb_last_error(void) { return g_err.c_str(); }

size_t mmlttb_workspace_size(int64_t n, int64_t n_out, int32_t r_ps)
{
    (void)n;
    if (n_out < 3 || n_out > kMaxI32 || r_ps < 1 || n_out * (int64_t)r_ps / 2 > kMaxI32)
        return 0;
    return mm_layout(n_out, r_ps).total;
}

size_t mmlttb_lttb_workspace_size(int64_t n, int64_t n_out)
{
    (void)n;
    if (n_out < 3 || n_out > kMaxI32)
        return 0;
    return lt_layout(n_out).total;
}

int mmlttb_minmax(int xk, const int64_t *x, const float *y, int64_t n, int64_t n_out, int32_t r_ps, int64_t *out_idx,
                  int64_t *out_count, void *ws, size_t ws_bytes, void *stream)
{
    int rc = check_series(xk, x, y, n, n_out);
    if (rc)
        return rc;
    if ((rc = check_rps(n, n_out, r_ps, 1)))
        return rc;
    if (!out_idx || !out_count)
        return fail(MMLTTB_EINVAL, "out_idx and out_count must not be NULL");
    hipStream_t s = (hipStream_t)stream;
    if (n <= 2) {
        MMLTTB_LAUNCH("iota", s, launch_iota(out_idx, n, out_count, s));
        return ok();
    }
    const MmLayout L = mm_layout(n_out, r_ps);
    const int64_t nb = n_out * (int64_t)r_ps / 2;
    if (nb < n - 2) {
        if (!ws)
            return fail(MMLTTB_EINVAL, "ws must not be NULL");
        if (ws_bytes < L.total)
            return fail(MMLTTB_ENOMEM, "workspace of %zu bytes is below the %zu required", ws_bytes, L.total);
    }
    rc = enqueue_preselect(x, y, n, n_out, r_ps, ws, L, out_idx, nullptr, nullptr, out_count, s);
    return rc ? rc : ok();
}

int mmlttb_lttb(int xk, const int64_t *x, const float *y, int64_t n, int64_t n_out, int64_t *out_idx, void *ws,
                size_t ws_bytes, void *stream)
{
    int rc = check_series(xk, x, y, n, n_out);
    if (rc)
        return rc;
    if (!out_idx)
        return fail(MMLTTB_EINVAL, "out_idx must not be NULL");
    hipStream_t s = (hipStream_t)stream;
    if (n <= n_out) {
        MMLTTB_LAUNCH("iota", s, launch_iota(out_idx, n, nullptr, s));
        return ok();
    }
    const LtLayout L = lt_layout(n_out);
    if (!ws)
        return fail(MMLTTB_EINVAL, "ws must not be NULL");
    if (ws_bytes < L.total)
        return fail(MMLTTB_ENOMEM, "workspace of %zu bytes is below the %zu required", ws_bytes, L.total);
    const int64_t B = n_out - 2;
    double *MX = at<double>(ws, L.MX), *MY = at<double>(ws, L.MY);
    const Split bk = make_split(n - 2, B);
    const int64_t maxb = bk.q + (bk.r ? 1 : 0);
    const bool seg = use_segmented_chain(maxb);
    // wide buckets: transition tables unless the sequential pass is asked for
    const bool tables = !seg && maxb > 64 && tuning().chain != kChainSequential && B <= kTableMaxBuckets &&
                        maxb < kTableMaxBucket;
    if (maxb <= 64) {
        MMLTTB_LAUNCH("bucket_mean", s, launch_bucket_mean_small(x, y, nullptr, n, B, MX, MY, s));
    } else if (!tables) {
        MMLTTB_LAUNCH("bucket_mean_wide", s, launch_bucket_mean_wide(x, y, n, B, MX, MY, nullptr, s));
    }
    if (seg) {
        const SegChainArgs a = seg_args(ws, L.path, L.finals, L.start, x, y, nullptr, n, B, MX, MY, maxb);
        MMLTTB_LAUNCH("lttb_chain_seg", s, launch_lttb_chain_seg(a, nullptr, out_idx, s));
    } else if (tables) {
        int32_t *cnt = at<int32_t>(ws, L.cand_cnt), *cand = at<int32_t>(ws, L.cand);
        int2 *tab = at<int2>(ws, L.tab);
        float2 *yr = at<float2>(ws, L.yr);
        unsigned long long *shi = at<unsigned long long>(ws, L.slab_hi), *slo = at<unsigned long long>(ws, L.slab_lo);
        double *delta = at<double>(ws, L.delta);
        double2 *brk = at<double2>(ws, L.brk);
        // pass 1: means, y ranges, slab highs and lows; pass 2: candidates; then the tables
        MMLTTB_LAUNCH("lttb_scan", s, launch_lttb_scan(x, y, n, B, MX, MY, yr, shi, slo, s));
        MMLTTB_LAUNCH("lttb_hull", s, launch_lttb_hull(x, y, n, B, MX, MY, yr, shi, slo, cnt, cand, delta, brk, s));
        MMLTTB_LAUNCH("lttb_tables", s, launch_lttb_tables(x, y, n, B, MX, MY, yr, cnt, cand, delta, brk, tab, s));
        MMLTTB_LAUNCH("lttb_table_walk", s, launch_lttb_table_walk(x, y, n, B, MX, MY, cnt, cand, tab, out_idx, s));
    } else if (maxb <= kChainStage) {
        MMLTTB_LAUNCH("lttb_chain", s, launch_lttb_chain(x, y, nullptr, n, B, MX, MY, nullptr, out_idx, s));
    } else {
        MMLTTB_LAUNCH("lttb_chain_wide", s, launch_lttb_chain_wide(x, y, n, B, MX, MY, out_idx, s));
    }
    return ok();
}

int mmlttb_lttb_means(int xk, const int64_t *x, const float *y, int64_t m, int64_t n_out, double *MX, double *MY,
                      void *stream)
{
    int rc = check_series(xk, x, y, m, n_out);
    if (rc)
        return rc;
    if (m <= n_out)
        return fail(MMLTTB_EINVAL, "m must exceed n_out (LTTB keeps every point otherwise), got m=%lld n_out=%lld",
                    (long long)m, (long long)n_out);
    if (!MX || !MY || ((uintptr_t)MX & 7u) || ((uintptr_t)MY & 7u))
        return fail(MMLTTB_EINVAL, "MX and MY must be non-NULL and 8-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    const int64_t B = n_out - 2;
    const Split bk = make_split(m - 2, B);
    const int64_t maxb = bk.q + (bk.r ? 1 : 0);
    // as in mmlttb_lttb: one thread per bucket up to 64 points, else a workgroup per bucket
    if (maxb <= 64) {
        MMLTTB_LAUNCH("bucket_mean", s, launch_bucket_mean_small(x, y, nullptr, m, B, MX, MY, s));
    } else {
        MMLTTB_LAUNCH("bucket_mean_wide", s, launch_bucket_mean_wide(x, y, m, B, MX, MY, nullptr, s));
    }
    return ok();
}

int mmlttb_minmaxlttb(int xk, const int64_t *x, const float *y, int64_t n, int64_t n_out, int32_t r_ps,
                      int64_t *out_idx, void *ws, size_t ws_bytes, void *stream)
{
    int rc = check_series(xk, x, y, n, n_out);
    if (rc)
        return rc;
    if ((rc = check_rps(n, n_out, r_ps)))
        return rc;
    if (!out_idx)
        return fail(MMLTTB_EINVAL, "out_idx must not be NULL");
    hipStream_t s = (hipStream_t)stream;
    if (n <= n_out) {
        CallSpan span("call_minmaxlttb", s);
        MMLTTB_LAUNCH("iota", s, launch_iota(out_idx, n, nullptr, s));
        span.close();
        return ok();
    }
    const MmLayout L = mm_layout(n_out, r_ps);
    if (!ws)
        return fail(MMLTTB_EINVAL, "ws must not be NULL");
    if (ws_bytes < L.total)
        return fail(MMLTTB_ENOMEM, "workspace of %zu bytes is below the %zu required", ws_bytes, L.total);
    CallSpan span("call_minmaxlttb", s);
    int64_t *P = at<int64_t>(ws, L.P), *XP = at<int64_t>(ws, L.XP), *m = at<int64_t>(ws, L.m);
    float *YP = at<float>(ws, L.YP);
    double *MX = at<double>(ws, L.MX), *MY = at<double>(ws, L.MY);
    const int64_t B = n_out - 2;
    const int64_t nb = n_out * (int64_t)r_ps / 2;
    if (nb >= n - 2) { // every bin holds at most one point: P is every index
        MMLTTB_LAUNCH("preselect_all", s, launch_preselect_all(n, x, y, P, XP, YP, m, s));
        MMLTTB_LAUNCH("bucket_mean", s, launch_bucket_mean_small(XP, YP, m, 0, B, MX, MY, s));
    } else {
        unsigned long long *keys = at<unsigned long long>(ws, L.keys);
        const MinMaxGeom g = minmax_geom(n - 2, nb);
        const int64_t maxb_bound = (2 * nb + B - 1) / B;
        if (use_segmented_chain(maxb_bound) && preselect_tail_fits(nb, maxb_bound)) {
            // two launches: the stream (clearing the tail's ticket, kept in the slot of m) and the fused tail
            unsigned int *ticket = at<unsigned int>(ws, L.m);
            MMLTTB_TRY(enqueue_minmax_stream(y, g, keys, s, ticket));
            const SegChainArgs a = seg_args(ws, L.path, L.finals, L.start, XP, YP, m, 0, B, MX, MY, maxb_bound);
            MMLTTB_LAUNCH("preselect_tail", s,
                          launch_preselect_tail(keys, g.bins, n, x, y, B, a.stage_cap, P, a.path, a.finals, a.start,
                                                ticket, out_idx, s));
            span.close();
            return ok();
        }
        MMLTTB_TRY(enqueue_minmax_stream(y, g, keys, s));
        if (nb <= kFusedCompactBins) { // one workgroup: compaction, then the means
            MMLTTB_LAUNCH("preselect_compact_means", s,
                          launch_preselect_compact_means(keys, g.bins, n, x, y, P, XP, YP, m, B, MX, MY, s));
        } else { // many bins: tiled compaction, then the means over many workgroups
            MMLTTB_LAUNCH("preselect_compact", s,
                          launch_compact_tiled(keys, g.bins, n, x, y, P, XP, YP, m, at<int64_t>(ws, L.tiles), s));
            MMLTTB_LAUNCH("bucket_mean", s, launch_bucket_mean_small(XP, YP, m, 0, B, MX, MY, s));
        }
    }
    // preselected points per bucket: at most ceil((m-2)/B) with m - 2 <= 2*nb
    const int64_t maxb_bound = (2 * nb + B - 1) / B;
    if (use_segmented_chain(maxb_bound)) {
        const SegChainArgs a = seg_args(ws, L.path, L.finals, L.start, XP, YP, m, 0, B, MX, MY, maxb_bound);
        MMLTTB_LAUNCH("lttb_chain_seg", s, launch_lttb_chain_seg(a, P, out_idx, s));
    } else {
        MMLTTB_LAUNCH("lttb_chain", s, launch_lttb_chain(XP, YP, m, 0, B, MX, MY, P, out_idx, s));
    }
    span.close();
    return ok();
}

size_t mmlttb_simplify_workspace_size(int64_t n, int64_t n_out, int32_t r_ps)
{
    (void)n;
    if (n_out < 3 || n_out > kMaxI32 || r_ps < 2 || n_out * (int64_t)r_ps / 2 > kMaxI32)
        return 0;
    const int64_t cap = 2 * (n_out * (int64_t)r_ps / 2) + 2;
    return mm_layout(n_out, r_ps).total + align_up((size_t)simplify_scratch_bytes(cap));
}

int mmlttb_minmax_simplify(int alg, int xk, const int64_t *x, const float *y, int64_t n, int64_t n_out, int32_t r_ps,
                           int64_t *out_idx, void *ws, size_t ws_bytes, void *stream)
{
    if (alg != MMLTTB_SIMPLIFY_VW && alg != MMLTTB_SIMPLIFY_DP && alg != MMLTTB_SIMPLIFY_LLB)
        return fail(MMLTTB_EINVAL, "alg must be MMLTTB_SIMPLIFY_VW, _DP or _LLB, got %d", alg);
    int rc = check_series(xk, x, y, n, n_out);
    if (rc)
        return rc;
    if ((rc = check_rps(n, n_out, r_ps)))
        return rc;
    const int64_t nb = n_out * (int64_t)r_ps / 2;
    const int64_t cap = 2 * nb + 2;
    if (cap > kMaxI32)
        return fail(MMLTTB_EINVAL, "2*floor(n_out*r_ps/2)+2 must be <= 2^31-1 for the simplifiers");
    if (!out_idx)
        return fail(MMLTTB_EINVAL, "out_idx must not be NULL");
    hipStream_t s = (hipStream_t)stream;
    if (n <= n_out) {
        MMLTTB_LAUNCH("iota", s, launch_iota(out_idx, n, nullptr, s));
        return ok();
    }
    const MmLayout L = mm_layout(n_out, r_ps);
    const size_t need = mmlttb_simplify_workspace_size(n, n_out, r_ps);
    if (!ws)
        return fail(MMLTTB_EINVAL, "ws must not be NULL");
    if (ws_bytes < need)
        return fail(MMLTTB_ENOMEM, "workspace of %zu bytes is below the %zu required", ws_bytes, need);
    int64_t *P = at<int64_t>(ws, L.P), *XP = at<int64_t>(ws, L.XP), *m = at<int64_t>(ws, L.m);
    float *YP = at<float>(ws, L.YP);
    if ((rc = enqueue_preselect(x, y, n, n_out, r_ps, ws, L, P, XP, YP, m, s)))
        return rc;
    // per-point state in LDS when it fits the device's per-workgroup limit
    const int64_t bytes = simplify_state_lds_bytes(cap);
    const int64_t tbytes = simplify_tree_lds_bytes(cap);
    int dev = 0, lds_max = 0, lds_optin = 0;
    if (hipGetDevice(&dev) == hipSuccess) {
        if (hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
            lds_max = 0;
        if (hipDeviceGetAttribute(&lds_optin, hipDeviceAttributeSharedMemPerBlockOptin, dev) != hipSuccess)
            lds_optin = 0;
        lds_max = lds_optin > lds_max ? lds_optin : lds_max;
    }
    bool in_lds = bytes <= (int64_t)lds_max;
    bool tree_in_lds = alg == MMLTTB_SIMPLIFY_DP && tbytes + simplify_tree_static_lds() <= (int64_t)lds_max;
    const size_t want_state = in_lds && bytes > 65536 ? (size_t)bytes : 0;
    const size_t want_tree = tree_in_lds && tbytes > 65536 ? (size_t)tbytes : 0;
    if ((want_state || want_tree) && simplify_allow_lds(want_state, want_tree) != hipSuccess)
        in_lds = tree_in_lds = false;
    SimplifyArgs a;
    a.XP = XP;
    a.YP = YP;
    a.m_ptr = m;
    a.Pmap = P;
    a.out = out_idx;
    a.n_out = n_out;
    a.cap = cap;
    a.cap_bucket = (cap - 2 + (n_out - 2) - 1) / (n_out - 2); // ceil((m - 2) / B) for any m <= cap
    a.scratch = static_cast<unsigned char *>(ws) + L.total;
    a.in_lds = in_lds ? 1 : 0;
    a.tree_in_lds = tree_in_lds ? 1 : 0;
    static const char *names[] = {"", "simplify_vw", "simplify_dp", "simplify_llb"};
    MMLTTB_LAUNCH(names[alg], s, launch_simplify(alg, a, s));
    return ok();
}

size_t mmlttb_typed_workspace_size(int64_t n, int64_t n_out, int32_t r_ps)
{
    (void)n;
    if (n_out < 3 || n_out > kMaxI32 || r_ps < 1 || n_out * (int64_t)r_ps / 2 > kMaxI32)
        return 0;
    return ty_layout(n_out, r_ps).total;
}

int mmlttb_minmax_typed(int yk, const void *y, int64_t n, int64_t n_out, int32_t r_ps, int64_t *out_idx,
                        int64_t *out_count, void *ws, size_t ws_bytes, void *stream)
{
    int rc = check_typed(MMLTTB_X_IMPLICIT, nullptr, yk, y, n, n_out, r_ps, 1);
    if (rc)
        return rc;
    if (!out_idx || !out_count)
        return fail(MMLTTB_EINVAL, "out_idx and out_count must not be NULL");
    hipStream_t s = (hipStream_t)stream;
    if (n <= 2) {
        MMLTTB_LAUNCH("iota", s, launch_iota(out_idx, n, out_count, s));
        return ok();
    }
    const TyLayout L = ty_layout(n_out, r_ps);
    if (!ws)
        return fail(MMLTTB_EINVAL, "ws must not be NULL");
    if (ws_bytes < L.total)
        return fail(MMLTTB_ENOMEM, "workspace of %zu bytes is below the %zu required", ws_bytes, L.total);
    const int64_t nb = n_out * (int64_t)r_ps / 2;
    rc = enqueue_typed_preselect(MMLTTB_X_IMPLICIT, nullptr, yk, y, n, nb, ws, L, out_idx, nullptr, nullptr,
                                 out_count, s);
    return rc ? rc : ok();
}

int mmlttb_minmaxlttb_typed(int xk, const void *x, int yk, const void *y, int64_t n, int64_t n_out, int32_t r_ps,
                            int64_t *out_idx, void *ws, size_t ws_bytes, void *stream)
{
    int rc = check_typed(xk, x, yk, y, n, n_out, r_ps, 2);
    if (rc)
        return rc;
    if (!out_idx)
        return fail(MMLTTB_EINVAL, "out_idx must not be NULL");
    hipStream_t s = (hipStream_t)stream;
    if (n <= n_out) {
        MMLTTB_LAUNCH("iota", s, launch_iota(out_idx, n, nullptr, s));
        return ok();
    }
    const TyLayout L = ty_layout(n_out, r_ps);
    if (!ws)
        return fail(MMLTTB_EINVAL, "ws must not be NULL");
    if (ws_bytes < L.total)
        return fail(MMLTTB_ENOMEM, "workspace of %zu bytes is below the %zu required", ws_bytes, L.total);
    const int64_t nb = n_out * (int64_t)r_ps / 2;
    const int64_t B = n_out - 2;
    int64_t *P = at<int64_t>(ws, L.P), *m = at<int64_t>(ws, L.m);
    double *XD = at<double>(ws, L.XD), *YD = at<double>(ws, L.YD);
    double *MX = at<double>(ws, L.MX), *MY = at<double>(ws, L.MY);
    if ((rc = enqueue_typed_preselect(xk, x, yk, y, n, nb, ws, L, P, XD, YD, m, s)))
        return rc;
    MMLTTB_LAUNCH("typed_bucket_means", s, launch_typed_bucket_means(xk, P, x, YD, m, B, MX, MY, s));
    const int64_t maxb_bound = (2 * nb + B - 1) / B;
    if (use_segmented_chain(maxb_bound)) {
        const SegChainArgsD a = seg_args(ws, L.path, L.finals, L.start, (const double *)XD, (const double *)YD, m, 0,
                                         B, MX, MY, maxb_bound);
        MMLTTB_LAUNCH("lttb_chain_seg", s, launch_lttb_chain_seg(a, P, out_idx, s));
    } else {
        MMLTTB_LAUNCH("lttb_chain", s, launch_lttb_chain((const double *)XD, (const double *)YD, m, 0, B, MX, MY, P,
                                                         out_idx, s));
    }
    return ok();
}

size_t mmlttb_xbins_workspace_size(int64_t n, int64_t n_out, int32_t r_ps)
{
    (void)n;
    if (n_out < 3 || n_out > kMaxI32 || r_ps < 1 || n_out * (int64_t)r_ps / 2 > kMaxI32)
        return 0;
    return xb_layout(n_out, r_ps).total;
}

int mmlttb_minmax_xbins(const int64_t *x, const float *y, int64_t n, int64_t n_out, int32_t r_ps, int64_t *out_idx,
                        int64_t *out_count, void *ws, size_t ws_bytes, void *stream)
{
    int rc = check_xbins(x, y, n, n_out, r_ps, 1);
    if (rc)
        return rc;
    if (!out_idx || !out_count)
        return fail(MMLTTB_EINVAL, "out_idx and out_count must not be NULL");
    hipStream_t s = (hipStream_t)stream;
    if (n <= 2) {
        MMLTTB_LAUNCH("iota", s, launch_iota(out_idx, n, out_count, s));
        return ok();
    }
    const XbLayout L = xb_layout(n_out, r_ps);
    if (!ws)
        return fail(MMLTTB_EINVAL, "ws must not be NULL");
    if (ws_bytes < L.total)
        return fail(MMLTTB_ENOMEM, "workspace of %zu bytes is below the %zu required", ws_bytes, L.total);
    const int64_t nb = n_out * (int64_t)r_ps / 2;
    if ((rc = enqueue_xbin_stream(x, y, n, nb, ws, L, s)))
        return rc;
    MMLTTB_LAUNCH("xbin_compact", s,
                  launch_xbin_compact(at<unsigned long long>(ws, L.mm.keys), at<int64_t>(ws, L.bounds), nb, n, x, y,
                                      out_idx, nullptr, nullptr, out_count, nullptr, 0, 0, nullptr, nullptr, s));
    return ok();
}

int mmlttb_minmaxlttb_xbins(const int64_t *x, const float *y, int64_t n, int64_t n_out, int32_t r_ps,
                            int64_t *out_idx, int64_t *out_count, void *ws, size_t ws_bytes, void *stream)
{
    int rc = check_xbins(x, y, n, n_out, r_ps, 2);
    if (rc)
        return rc;
    if (!out_idx || !out_count)
        return fail(MMLTTB_EINVAL, "out_idx and out_count must not be NULL");
    hipStream_t s = (hipStream_t)stream;
    if (n <= n_out) {
        MMLTTB_LAUNCH("iota", s, launch_iota(out_idx, n, out_count, s));
        return ok();
    }
    const XbLayout L = xb_layout(n_out, r_ps);
    if (!ws)
        return fail(MMLTTB_EINVAL, "ws must not be NULL");
    if (ws_bytes < L.total)
        return fail(MMLTTB_ENOMEM, "workspace of %zu bytes is below the %zu required", ws_bytes, L.total);
    const int64_t nb = n_out * (int64_t)r_ps / 2;
    const int64_t B = n_out - 2;
    if ((rc = enqueue_xbin_stream(x, y, n, nb, ws, L, s)))
        return rc;
    int64_t *P = at<int64_t>(ws, L.mm.P), *XP = at<int64_t>(ws, L.mm.XP), *m = at<int64_t>(ws, L.mm.m);
    int64_t *m_eff = at<int64_t>(ws, L.m_eff);
    float *YP = at<float>(ws, L.mm.YP);
    double *MX = at<double>(ws, L.mm.MX), *MY = at<double>(ws, L.mm.MY);
    MMLTTB_LAUNCH("xbin_compact", s,
                  launch_xbin_compact(at<unsigned long long>(ws, L.mm.keys), at<int64_t>(ws, L.bounds), nb, n, x, y, P,
                                      XP, YP, m, m_eff, n_out + 1, B, MX, MY, s));
    // the LTTB pass runs on at most max(2*nb + 2, n_out + 1) points
    const int64_t maxb_bound = (2 * nb + B - 1) / B;
    if (use_segmented_chain(maxb_bound)) {
        const SegChainArgs a = seg_args(ws, L.mm.path, L.mm.finals, L.mm.start, XP, YP, m_eff, 0, B, MX, MY,
                                        maxb_bound);
        MMLTTB_LAUNCH("lttb_chain_seg", s, launch_lttb_chain_seg(a, P, out_idx, s));
    } else {
        MMLTTB_LAUNCH("lttb_chain", s, launch_lttb_chain(XP, YP, m_eff, 0, B, MX, MY, P, out_idx, s));
    }
    MMLTTB_LAUNCH("xbin_finish", s, launch_xbin_finish(P, m, n_out, out_idx, out_count, s));
    return ok();
}

size_t mmlttb_m4_workspace_size(int64_t n, int64_t n_out)
{
    (void)n;
    if (n_out < 4 || n_out > kMaxI32)
        return 0;
    return align_up(16 * (size_t)(n_out / 4));
}

int mmlttb_m4(const float *y, int64_t n, int64_t n_out, int64_t *out_idx, int64_t *out_count, void *ws,
              size_t ws_bytes, void *stream)
{
    if (!y || ((uintptr_t)y & 3u))
        return fail(MMLTTB_EINVAL, "y must be a non-NULL 4-byte aligned pointer");
    if (n < 1 || n > kMaxN)
        return fail(MMLTTB_EINVAL, "n must be in [1, 2^62], got %lld", (long long)n);
    if (n_out < 4 || n_out > kMaxI32)
        return fail(MMLTTB_EINVAL, "n_out must be in [4, 2^31-1], got %lld", (long long)n_out);
    if (!out_idx || !out_count)
        return fail(MMLTTB_EINVAL, "out_idx and out_count must not be NULL");
    hipStream_t s = (hipStream_t)stream;
    if (n <= n_out) {
        MMLTTB_LAUNCH("iota", s, launch_iota(out_idx, n, out_count, s));
        return ok();
    }
    const int64_t nb = n_out / 4;
    const int64_t maxbin = n / nb + (n % nb ? 1 : 0);
    if (maxbin >= ((int64_t)1 << 32))
        return fail(MMLTTB_EINVAL, "M4 bins of %lld points exceed 2^32-1", (long long)maxbin);
    const size_t need = mmlttb_m4_workspace_size(n, n_out);
    if (!ws)
        return fail(MMLTTB_EINVAL, "ws must not be NULL");
    if (ws_bytes < need)
        return fail(MMLTTB_ENOMEM, "workspace of %zu bytes is below the %zu required", ws_bytes, need);
    unsigned long long *keys = static_cast<unsigned long long *>(ws);
    const MinMaxGeom g = minmax_geom(n, nb);
    if (keys_need_init(g))
        MMLTTB_LAUNCH("init_keys", s, launch_init_keys(keys, nb, s));
    MMLTTB_LAUNCH("m4_bin_reduce", s, launch_m4_bin_reduce(y, g, tuning().unroll, keys, s));
    MMLTTB_LAUNCH("m4_compact", s, launch_m4_compact(keys, g.bins, out_idx, out_count, s));
    return ok();
}

int mmlttb_everynth(int64_t n, int64_t n_out, int64_t *out_idx, void *stream)
{
    if (n < 1 || n > kMaxN)
        return fail(MMLTTB_EINVAL, "n must be in [1, 2^62], got %lld", (long long)n);
    if (n_out < 1 || n_out > kMaxI32)
        return fail(MMLTTB_EINVAL, "n_out must be in [1, 2^31-1], got %lld", (long long)n_out);
    if (!out_idx)
        return fail(MMLTTB_EINVAL, "out_idx must not be NULL");
    hipStream_t s = (hipStream_t)stream;
    if (n <= n_out) {
        MMLTTB_LAUNCH("iota", s, launch_iota(out_idx, n, nullptr, s));
    } else {
        MMLTTB_LAUNCH("everynth", s, launch_everynth(n, n_out, out_idx, s));
    }
    return ok();
}

int mmlttb_set_tuning(int unroll, int64_t chunk, int chain, int tile, int batch_unroll, int64_t batch_chunk)
{
    Tuning &t = tuning();
    if (tile != 0 && !valid_tile(tile))
        return fail(MMLTTB_EINVAL, "tile must be 2048, 4096 or 8192");
    if ((unroll != 0 && !valid_unroll(unroll)) || (batch_unroll != 0 && !valid_unroll(batch_unroll)))
        return fail(MMLTTB_EINVAL, "unroll and batch_unroll must be 1, 2, 4 or 8");
    if ((chunk != 0 && chunk < 256) || (batch_chunk != 0 && batch_chunk < 256))
        return fail(MMLTTB_EINVAL, "chunk and batch_chunk must be >= 256");
    if (chain < 0 || chain > 3)
        return fail(MMLTTB_EINVAL, "chain must be 0 (keep), 1 (sequential), 2 (segmented) or 3 (automatic)");
    if (unroll)
        t.unroll = unroll;
    if (chunk)
        t.chunk = chunk;
    if (chain)
        t.chain = chain;
    if (tile)
        t.tile = tile;
    if (batch_unroll)
        t.batch_unroll = batch_unroll;
    if (batch_chunk)
        t.batch_chunk = batch_chunk;
    t.chunk = round_chunk(t.chunk, t.unroll);
    t.batch_chunk = round_chunk(t.batch_chunk, t.batch_unroll);
    return ok();
}

int mmlttb_get_tuning(int *unroll, int64_t *chunk, int *chain, int *tile, int *batch_unroll, int64_t *batch_chunk)
{
    if (!unroll || !chunk || !chain || !tile || !batch_unroll || !batch_chunk)
        return fail(MMLTTB_EINVAL, "NULL argument");
    const Tuning &t = tuning();
    *unroll = t.unroll;
    *chunk = t.chunk;
    *chain = t.chain;
    *tile = t.tile;
    *batch_unroll = t.batch_unroll;
    *batch_chunk = t.batch_chunk;
    return ok();
}

int mmlttb_profile_enable(int on)
{
    g_prof = on != 0;
    return MMLTTB_OK;
}

int mmlttb_profile_reset(void)
{
    drain_pending();
    g_totals.clear();
    g_samples.clear();
    return MMLTTB_OK;
}

int mmlttb_profile_read(const char *kernel, double *total_ms, int64_t *launches)
{
    if (!kernel || !total_ms || !launches)
        return fail(MMLTTB_EINVAL, "NULL argument");
    drain_pending();
    auto it = g_totals.find(kernel);
    *total_ms = it == g_totals.end() ? 0.0 : it->second.first;
    *launches = it == g_totals.end() ? 0 : it->second.second;
    return MMLTTB_OK;
}

int mmlttb_profile_samples(const char *name, float *ms, int64_t cap, int64_t *count)
{
    if (!name || !count || cap < 0 || (cap > 0 && !ms))
        return fail(MMLTTB_EINVAL, "NULL argument or negative capacity");
    drain_pending();
    auto it = g_samples.find(name);
    const int64_t have = it == g_samples.end() ? 0 : (int64_t)it->second.size();
    for (int64_t i = 0; i < have && i < cap; i++)
        ms[i] = it->second[(size_t)i];
    *count = have;
    return MMLTTB_OK;
}

} // extern "C"
