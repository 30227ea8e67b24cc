// C ABI of libmmlttb: argument checks, workspace layout, launch sequences.
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>

#include <map>
#include <string>
#include <vector>

#include "kernels.hpp"
#include "libmmlttb.h"

using namespace mmlttb;

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int ok()
{
    g_err.clear();
    return MMLTTB_OK;
}

// ---------------------------------------------------------------- tuning

enum ChainMode { kChainAuto = 0, kChainSequential = 1, kChainSegmented = 2 };

struct Tuning {
    int unroll = 4;        // float4 loads per lane per batch in minmax_bin_reduce
    int64_t chunk = 16384; // points per minmax work item (multiple of 256 * unroll)
    int chain = kChainAuto;
};

Tuning &tuning()
{
    static Tuning t = [] {
        Tuning r;
        if (const char *e = getenv("MMLTTB_UNROLL")) {
            int u = atoi(e);
            if (u == 1 || u == 2 || u == 4 || u == 8)
                r.unroll = u;
        }
        if (const char *e = getenv("MMLTTB_CHUNK")) {
            long long c = atoll(e);
            if (c >= 256)
                r.chunk = c;
        }
        if (const char *e = getenv("MMLTTB_CHAIN")) {
            int c = atoi(e);
            if (c >= 0 && c <= 2)
                r.chain = c;
        }
        int64_t q = 256 * (int64_t)r.unroll;
        r.chunk = ((r.chunk + q - 1) / q) * q;
        return r;
    }();
    return t;
}

// ---------------------------------------------------------------- profiling

struct Pending {
    std::string name;
    hipEvent_t a, b;
};
bool g_prof = false;
std::vector<Pending> g_pending;
std::map<std::string, std::pair<double, int64_t>> g_totals;

template <class F>
hipError_t timed(const char *name, hipStream_t s, F &&launch)
{
    if (!g_prof)
        return launch();
    hipEvent_t a = nullptr, b = nullptr;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess)
        return launch();
    (void)hipEventRecord(a, s);
    hipError_t e = launch();
    (void)hipEventRecord(b, s);
    g_pending.push_back({name, a, b});
    return e;
}

void drain_pending()
{
    for (auto &p : g_pending) {
        float ms = 0.f;
        if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            auto &t = g_totals[p.name];
            t.first += ms;
            t.second += 1;
        }
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
    g_pending.clear();
}

// ---------------------------------------------------------------- layout

constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct MmLayout {
    size_t keys, m, P, XP, YP, MX, MY, path, finals, start, counter, total;
};

MmLayout mm_layout(int64_t n_out, int32_t r_ps)
{
    const int64_t nb = n_out * (int64_t)r_ps / 2;
    const int64_t cap = 2 * nb + 2;
    const int64_t B = n_out - 2;
    MmLayout L;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align_up(off + bytes);
        return o;
    };
    L.keys = take(16 * (size_t)nb);
    L.m = take(8);
    L.P = take(8 * (size_t)cap);
    L.XP = take(8 * (size_t)cap);
    L.YP = take(4 * (size_t)cap);
    L.MX = take(8 * (size_t)B);
    L.MY = take(8 * (size_t)B);
    L.path = take(seg_path_bytes(B));
    L.finals = take(seg_finals_bytes(B));
    L.start = take((size_t)seg_count(B));
    L.counter = take(sizeof(unsigned int));
    L.total = off;
    return L;
}

struct LtLayout {
    size_t MX, MY, path, finals, start, counter, total;
};

LtLayout lt_layout(int64_t n_out)
{
    const int64_t B = n_out - 2;
    LtLayout L;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align_up(off + bytes);
        return o;
    };
    L.MX = take(8 * (size_t)B);
    L.MY = take(8 * (size_t)B);
    L.path = take(seg_path_bytes(B));
    L.finals = take(seg_finals_bytes(B));
    L.start = take((size_t)seg_count(B));
    L.counter = take(sizeof(unsigned int));
    L.total = off;
    return L;
}

template <class T>
T *at(void *ws, size_t off)
{
    return reinterpret_cast<T *>(static_cast<char *>(ws) + off);
}

// ---------------------------------------------------------------- checks

constexpr int64_t kMaxN = (int64_t)1 << 62;
constexpr int64_t kMaxI32 = 0x7fffffff;

int check_series(int xk, const int64_t *x, const float *y, int64_t n, int64_t n_out)
{
    if (xk != MMLTTB_X_IMPLICIT && xk != MMLTTB_X_INT64)
        return fail(MMLTTB_EINVAL, "xk must be MMLTTB_X_IMPLICIT (0) or MMLTTB_X_INT64 (1), got %d", xk);
    if (xk == MMLTTB_X_IMPLICIT && x)
        return fail(MMLTTB_EINVAL, "x must be NULL with MMLTTB_X_IMPLICIT");
    if (xk == MMLTTB_X_INT64 && !x)
        return fail(MMLTTB_EINVAL, "x must not be NULL with MMLTTB_X_INT64");
    if (!y)
        return fail(MMLTTB_EINVAL, "y must not be NULL");
    if (((uintptr_t)y & 3u) || ((uintptr_t)x & 7u))
        return fail(MMLTTB_EINVAL, "y must be 4-byte and x 8-byte aligned");
    if (n < 1 || n > kMaxN)
        return fail(MMLTTB_EINVAL, "n must be in [1, 2^62], got %lld", (long long)n);
    if (n_out < 3 || n_out > kMaxI32)
        return fail(MMLTTB_EINVAL, "n_out must be in [3, 2^31-1], got %lld", (long long)n_out);
    return MMLTTB_OK;
}

int check_rps(int64_t n, int64_t n_out, int32_t r_ps)
{
    if (r_ps < 2)
        return fail(MMLTTB_EINVAL, "r_ps must be >= 2, got %d", r_ps);
    const int64_t nb = n_out * (int64_t)r_ps / 2;
    if (nb > kMaxI32)
        return fail(MMLTTB_EINVAL, "floor(n_out*r_ps/2) must be <= 2^31-1, got %lld", (long long)nb);
    if (n > 2) {
        const int64_t L = n - 2;
        const int64_t nbe = nb < L ? nb : L;
        const int64_t maxbin = L / nbe + (L % nbe ? 1 : 0);
        if (maxbin >= ((int64_t)1 << 32))
            return fail(MMLTTB_EINVAL, "MinMax bins of %lld points exceed 2^32-1", (long long)maxbin);
    }
    return MMLTTB_OK;
}

#define MMLTTB_LAUNCH(name, stream, expr)                                                                              \
    do {                                                                                                               \
        hipError_t e_ = timed(name, stream, [&] { return (expr); });                                                   \
        if (e_ != hipSuccess)                                                                                          \
            return fail(MMLTTB_EDEVICE, "%s launch failed: %s", name, hipGetErrorString(e_));                          \
    } while (0)

MinMaxGeom minmax_geom(int64_t n, int64_t nb)
{
    const Tuning &t = tuning();
    MinMaxGeom g;
    g.bins = make_split(n - 2, nb);
    const int64_t maxbin = g.bins.q + (g.bins.r ? 1 : 0);
    g.chunk = t.chunk;
    g.chunks_per_bin = (maxbin + g.chunk - 1) / g.chunk;
    if (g.chunks_per_bin < 1)
        g.chunks_per_bin = 1;
    g.n_items = nb * g.chunks_per_bin;
    return g;
}

bool use_segmented_chain(int64_t maxb_bound)
{
    const int mode = tuning().chain;
    return mode != kChainSequential && maxb_bound <= kSegStarts;
}

SegChainArgs seg_args(void *ws, size_t path, size_t finals, size_t start, size_t counter, const int64_t *XP,
                      const float *YP, const int64_t *m_ptr, int64_t m_const, int64_t B, const double *MX,
                      const double *MY, int64_t maxb_bound)
{
    SegChainArgs a;
    a.XP = XP;
    a.YP = YP;
    a.m_ptr = m_ptr;
    a.m_const = m_const;
    a.B = B;
    a.MX = MX;
    a.MY = MY;
    a.path = at<uint8_t>(ws, path);
    a.finals = at<uint8_t>(ws, finals);
    a.start = at<uint8_t>(ws, start);
    a.counter = at<unsigned int>(ws, counter);
    a.S = seg_count(B);
    a.stage_cap = (int)(kSegLen * maxb_bound);
    return a;
}

// Preselection into P (and, when XP != NULL, the gathered XP/YP); m to *m_out.
int enqueue_preselect(const int64_t *x, const float *y, int64_t n, int64_t n_out, int32_t r_ps, void *ws,
                      const MmLayout &L, int64_t *P, int64_t *XP, float *YP, int64_t *m_out, hipStream_t s)
{
    const int64_t nb = n_out * (int64_t)r_ps / 2;
    const int64_t Lint = n - 2;
    if (nb >= Lint) { // every bin holds at most one point: P is every index
        if (XP) {
            MMLTTB_LAUNCH("preselect_all", s, launch_preselect_all(n, x, y, P, XP, YP, m_out, s));
        } else {
            MMLTTB_LAUNCH("iota", s, launch_iota(P, n, m_out, s));
        }
        return MMLTTB_OK;
    }
    unsigned long long *keys = at<unsigned long long>(ws, L.keys);
    const MinMaxGeom g = minmax_geom(n, nb);
    MMLTTB_LAUNCH("init_keys", s, launch_init_keys(keys, nb, s));
    MMLTTB_LAUNCH("minmax_bin_reduce", s, launch_minmax_bin_reduce(y, g, tuning().unroll, keys, s));
    MMLTTB_LAUNCH("preselect_compact", s, launch_preselect_compact(keys, g.bins, n, x, y, P, XP, YP, m_out, s));
    return MMLTTB_OK;
}

} // namespace

extern "C" {

const char *mmlttb_version(void) { return "libmmlttb 0.1.0 (gfx950)"; }

const char *mmlttb_last_error(void) { return g_err.c_str(); }

size_t mmlttb_workspace_size(int64_t n, int64_t n_out, int32_t r_ps)
{
    (void)n;
    if (n_out < 3 || n_out > kMaxI32 || r_ps < 2 || n_out * (int64_t)r_ps / 2 > kMaxI32)
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
    if ((rc = check_rps(n, n_out, r_ps)))
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
    unsigned int *counter = at<unsigned int>(ws, L.counter);
    if (maxb <= 64) {
        MMLTTB_LAUNCH("bucket_mean", s, launch_bucket_mean_small(x, y, nullptr, n, B, MX, MY, counter, s));
    } else {
        MMLTTB_LAUNCH("bucket_mean_wide", s, launch_bucket_mean_wide(x, y, n, B, MX, MY, counter, s));
    }
    if (use_segmented_chain(maxb)) {
        const SegChainArgs a = seg_args(ws, L.path, L.finals, L.start, L.counter, x, y, nullptr, n, B, MX, MY, maxb);
        MMLTTB_LAUNCH("lttb_chain_seg", s, launch_lttb_chain_seg(a, nullptr, out_idx, s));
    } else if (maxb <= kChainStage) {
        MMLTTB_LAUNCH("lttb_chain", s, launch_lttb_chain(x, y, nullptr, n, B, MX, MY, nullptr, out_idx, s));
    } else {
        MMLTTB_LAUNCH("lttb_chain_wide", s, launch_lttb_chain_wide(x, y, n, B, MX, MY, out_idx, s));
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
        MMLTTB_LAUNCH("iota", s, launch_iota(out_idx, n, nullptr, s));
        return ok();
    }
    const MmLayout L = mm_layout(n_out, r_ps);
    if (!ws)
        return fail(MMLTTB_EINVAL, "ws must not be NULL");
    if (ws_bytes < L.total)
        return fail(MMLTTB_ENOMEM, "workspace of %zu bytes is below the %zu required", ws_bytes, L.total);
    int64_t *P = at<int64_t>(ws, L.P), *XP = at<int64_t>(ws, L.XP), *m = at<int64_t>(ws, L.m);
    float *YP = at<float>(ws, L.YP);
    double *MX = at<double>(ws, L.MX), *MY = at<double>(ws, L.MY);
    rc = enqueue_preselect(x, y, n, n_out, r_ps, ws, L, P, XP, YP, m, s);
    if (rc)
        return rc;
    const int64_t B = n_out - 2;
    unsigned int *counter = at<unsigned int>(ws, L.counter);
    MMLTTB_LAUNCH("bucket_mean", s, launch_bucket_mean_small(XP, YP, m, 0, B, MX, MY, counter, s));
    // preselected points per bucket: at most ceil((m-2)/B) with m - 2 <= 2*nb
    const int64_t nb = n_out * (int64_t)r_ps / 2;
    const int64_t maxb_bound = (2 * nb + B - 1) / B;
    if (use_segmented_chain(maxb_bound)) {
        const SegChainArgs a = seg_args(ws, L.path, L.finals, L.start, L.counter, XP, YP, m, 0, B, MX, MY, maxb_bound);
        MMLTTB_LAUNCH("lttb_chain_seg", s, launch_lttb_chain_seg(a, P, out_idx, s));
    } else {
        MMLTTB_LAUNCH("lttb_chain", s, launch_lttb_chain(XP, YP, m, 0, B, MX, MY, P, out_idx, s));
    }
    return ok();
}

size_t mmlttb_batched_workspace_size(const mmlttb_segment_t *segs_host, int64_t n_segs)
{
    (void)segs_host;
    (void)n_segs;
    return 0;
}

int mmlttb_minmaxlttb_batched(int xk, const int64_t *x_base, const float *y_base, const mmlttb_segment_t *segs_host,
                              int64_t n_segs, int64_t *out_idx_base, void *ws, size_t ws_bytes, void *stream)
{
    (void)xk;
    (void)x_base;
    (void)y_base;
    (void)segs_host;
    (void)n_segs;
    (void)out_idx_base;
    (void)ws;
    (void)ws_bytes;
    (void)stream;
    return fail(MMLTTB_ENOTSUP, "batched mode is not built yet");
}

int mmlttb_set_tuning(int unroll, int64_t chunk, int chain)
{
    Tuning &t = tuning();
    if (unroll != 0 && unroll != 1 && unroll != 2 && unroll != 4 && unroll != 8)
        return fail(MMLTTB_EINVAL, "unroll must be 1, 2, 4 or 8");
    if (chunk != 0 && chunk < 256)
        return fail(MMLTTB_EINVAL, "chunk must be >= 256");
    if (chain < 0 || chain > 2)
        return fail(MMLTTB_EINVAL, "chain must be 0 (auto), 1 (sequential) or 2 (segmented)");
    if (unroll)
        t.unroll = unroll;
    if (chunk)
        t.chunk = chunk;
    if (chain)
        t.chain = chain;
    const int64_t q = 256 * (int64_t)t.unroll;
    t.chunk = ((t.chunk + q - 1) / q) * q;
    return ok();
}

int mmlttb_get_tuning(int *unroll, int64_t *chunk, int *chain)
{
    if (!unroll || !chunk || !chain)
        return fail(MMLTTB_EINVAL, "NULL argument");
    *unroll = tuning().unroll;
    *chunk = tuning().chunk;
    *chain = tuning().chain;
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

} // extern "C"
