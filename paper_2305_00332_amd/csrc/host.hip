// Host side of libmmlttb shared by its entry points: error reporting,
// tuning, launch timing, workspace layouts, argument checks and shared
// launch sequences (declared in host.hpp).
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "errors.hpp"
#include "host.hpp"

namespace mmlttb {
namespace host {

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

Tuning &tuning()
{
    static Tuning t = [] {
        Tuning r;
        if (const char *e = getenv("MMLTTB_UNROLL")) {
            if (valid_unroll(atoi(e)))
                r.unroll = atoi(e);
        }
        if (const char *e = getenv("MMLTTB_CHUNK")) {
            long long c = atoll(e);
            if (c >= 256)
                r.chunk = c;
        }
        if (const char *e = getenv("MMLTTB_TILE")) {
            if (valid_tile(atoi(e)))
                r.tile = atoi(e);
        }
        if (const char *e = getenv("MMLTTB_CHAIN")) {
            int c = atoi(e);
            if (c >= 1 && c <= 3)
                r.chain = c;
        }
        if (const char *e = getenv("MMLTTB_BATCH_UNROLL")) {
            if (valid_unroll(atoi(e)))
                r.batch_unroll = atoi(e);
        }
        if (const char *e = getenv("MMLTTB_BATCH_CHUNK")) {
            long long c = atoll(e);
            if (c >= 256)
                r.batch_chunk = c;
        }
        r.chunk = round_chunk(r.chunk, r.unroll);
        r.batch_chunk = round_chunk(r.batch_chunk, r.batch_unroll);
        return r;
    }();
    return t;
}

// ---------------------------------------------------------------- profiling

bool g_prof = false;
std::vector<Pending> g_pending;
std::vector<hipEvent_t> g_event_pool;
std::map<std::string, std::pair<double, int64_t>> g_totals;
std::map<std::string, std::vector<float>> g_samples; // per-launch durations, in launch order

// Timing-only events: no system-scope fence on record, so recording them
// neither writes back nor invalidates caches around the timed kernel.
hipEvent_t take_event()
{
    if (!g_event_pool.empty()) {
        hipEvent_t e = g_event_pool.back();
        g_event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess)
        return nullptr;
    return e;
}

// Timing events are recorded only on streams that are not being captured
// into a graph: a captured event would complete only when the graph runs, and
// reading the profile would wait for it.
bool capturing(hipStream_t s)
{
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    return hipStreamIsCapturing(s, &st) == hipSuccess && st != hipStreamCaptureStatusNone;
}

void drain_pending()
{
    for (auto &p : g_pending) {
        float ms = 0.f;
        if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            auto &t = g_totals[p.name];
            t.first += ms;
            t.second += 1;
            auto &v = g_samples[p.name];
            if (v.size() < kMaxSamples)
                v.push_back(ms);
        }
        g_event_pool.push_back(p.a);
        g_event_pool.push_back(p.b);
    }
    g_pending.clear();
}

// ---------------------------------------------------------------- layout

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
    L.start = take(seg_start_bytes(B));
    L.tiles = take(8 * (size_t)compact_tiles(nb)); // first slots of the tiled compaction
    L.total = off;
    return L;
}

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
    L.start = take(seg_start_bytes(B));
    const size_t tb = B <= kTableMaxBuckets ? (size_t)B : 0; // transition tables (wide buckets)
    L.yr = take(8 * tb);
    L.cand_cnt = take(4 * tb);
    L.cand = take(4 * tb * kCandMax);
    L.tab = take(8 * tb * kCandMax);
    L.slab_hi = take(8 * tb * kSlabsHost);
    L.slab_lo = take(8 * tb * kSlabsHost);
    L.delta = take(8 * tb);
    L.brk = take(16 * tb);
    L.total = off;
    return L;
}

// ---------------------------------------------------------------- checks

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

int check_rps(int64_t n, int64_t n_out, int32_t r_ps, int32_t min_rps)
{
    if (r_ps < min_rps)
        return fail(MMLTTB_EINVAL, "r_ps must be >= %d, got %d", min_rps, r_ps);
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

// Chunks per bin: enough for items of at most `chunk` points, and about
// kFillItems items in all (rounded to the nearest whole count per bin).
int64_t chunks_per_bin(int64_t maxbin, int64_t nb, int64_t chunk)
{
    int64_t cpb = (maxbin + chunk - 1) / chunk;
    const int64_t fill = (kFillItems + nb / 2) / nb;
    cpb = cpb > fill ? cpb : fill;
    cpb = cpb < maxbin ? cpb : maxbin;
    return cpb < 1 ? 1 : cpb;
}

// Bins over `len` points (the interior n-2 for MinMax, all n for M4).
MinMaxGeom minmax_geom(int64_t len, int64_t nb)
{
    const Tuning &t = tuning();
    MinMaxGeom g;
    g.bins = make_split(len, nb);
    const int64_t maxbin = g.bins.q + (g.bins.r ? 1 : 0);
    const int64_t gran = 256 * (int64_t)t.unroll; // points per batch of loads
    const int64_t cpb = chunks_per_bin(maxbin, nb, t.chunk);
    g.chunk = ((maxbin + cpb - 1) / cpb + gran - 1) / gran * gran;
    g.chunks_per_bin = (maxbin + g.chunk - 1) / g.chunk;
    g.n_items = nb * g.chunks_per_bin;
    return g;
}

// The MinMax stream of one float32 series into its bin keys: one work item
// per bin (or bin piece), or, for short bins, fixed chunks across bin ends.
// `ticket` (optional): cleared on the way for a k_preselect_tail launch.
int enqueue_minmax_stream(const float *y, const MinMaxGeom &g, unsigned long long *keys, hipStream_t s,
                          unsigned int *ticket)
{
    const int64_t maxbin = g.bins.q + (g.bins.r ? 1 : 0);
    if (maxbin < kShortBin && g.bins.len >= kShortBinChunk * kFillItems) { // and at least 2048 chunks
        if (!ticket && small_tile_bins(maxbin, g.bins.parts, tuning().tile) > 0) {
            // bins of at most a quarter tile: whole bins per tile, every key written
            MMLTTB_LAUNCH("minmax_bin_reduce", s, launch_minmax_small_tiles(y, g.bins, tuning().tile, keys, s));
            return MMLTTB_OK;
        }
        MMLTTB_LAUNCH("init_keys", s, launch_init_keys(keys, g.bins.parts, s, ticket));
        MMLTTB_LAUNCH("minmax_bin_reduce", s, launch_minmax_stream_chunks(y, g.bins, tuning().unroll, keys, s));
        return MMLTTB_OK;
    }
    if (keys_need_init(g))
        MMLTTB_LAUNCH("init_keys", s, launch_init_keys(keys, g.bins.parts, s, ticket));
    MMLTTB_LAUNCH("minmax_bin_reduce", s, launch_minmax_bin_reduce(y, g, tuning().unroll, keys, s, ticket));
    return MMLTTB_OK;
}

bool use_segmented_chain(int64_t maxb_bound)
{
    const int mode = tuning().chain;
    return mode != kChainSequential && maxb_bound <= kSegStarts;
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
    const MinMaxGeom g = minmax_geom(n - 2, nb);
    MMLTTB_TRY(enqueue_minmax_stream(y, g, keys, s));
    if (nb <= kFusedCompactBins) {
        MMLTTB_LAUNCH("preselect_compact", s, launch_preselect_compact(keys, g.bins, n, x, y, P, XP, YP, m_out, s));
    } else {
        MMLTTB_LAUNCH("preselect_compact", s,
                      launch_compact_tiled(keys, g.bins, n, x, y, P, XP, YP, m_out, at<int64_t>(ws, L.tiles), s));
    }
    return MMLTTB_OK;
}

// ---------------------------------------------------------------- x-width bins

XbLayout xb_layout(int64_t n_out, int32_t r_ps)
{
    XbLayout L;
    L.mm = mm_layout(n_out, r_ps);
    const int64_t nb = n_out * (int64_t)r_ps / 2;
    L.bounds = L.mm.total;
    L.m_eff = align_up(L.bounds + 8 * (size_t)(nb + 1));
    L.total = align_up(L.m_eff + 8);
    return L;
}

int check_xbins(const int64_t *x, const float *y, int64_t n, int64_t n_out, int32_t r_ps, int32_t min_rps)
{
    if (!x || !y)
        return fail(MMLTTB_EINVAL, "x and y must not be NULL");
    if (((uintptr_t)y & 3u) || ((uintptr_t)x & 7u))
        return fail(MMLTTB_EINVAL, "y must be 4-byte and x 8-byte aligned");
    if (n < 1 || n - 2 >= ((int64_t)1 << 32))
        return fail(MMLTTB_EINVAL, "n must be in [1, 2^32+1] with bins of equal x width, got %lld", (long long)n);
    if (n_out < 3 || n_out > kMaxI32)
        return fail(MMLTTB_EINVAL, "n_out must be in [3, 2^31-1], got %lld", (long long)n_out);
    if (r_ps < min_rps)
        return fail(MMLTTB_EINVAL, "r_ps must be >= %d, got %d", min_rps, r_ps);
    if (n_out * (int64_t)r_ps / 2 > kMaxI32)
        return fail(MMLTTB_EINVAL, "floor(n_out*r_ps/2) must be <= 2^31-1");
    return MMLTTB_OK;
}

// Bounds, keys and the stream over the interior; n > 2.
int enqueue_xbin_stream(const int64_t *x, const float *y, int64_t n, int64_t nb, void *ws, const XbLayout &L,
                        hipStream_t s)
{
    const Tuning &t = tuning();
    int64_t *bounds = at<int64_t>(ws, L.bounds);
    unsigned long long *keys = at<unsigned long long>(ws, L.mm.keys);
    const int64_t gran = 256 * (int64_t)t.unroll;
    const int64_t avg = (n - 2 + nb - 1) / nb;
    const int64_t cpb = chunks_per_bin(avg, nb, t.chunk);
    const int64_t chunk = ((avg + cpb - 1) / cpb + gran - 1) / gran * gran;
    MMLTTB_LAUNCH("xbin_bounds", s, launch_xbin_bounds(x, n, nb, bounds, s));
    MMLTTB_LAUNCH("init_keys", s, launch_init_keys(keys, nb, s));
    MMLTTB_LAUNCH("xbin_reduce", s, launch_xbin_reduce(y, bounds, n, nb, chunk, t.unroll, keys, s));
    return MMLTTB_OK;
}

// ---------------------------------------------------------------- other value types

// MinMax partials: at most max(nb, 2^16) work items, so the size depends on
// n_out and r_ps only.
TyLayout ty_layout(int64_t n_out, int32_t r_ps)
{
    const int64_t nb = n_out * (int64_t)r_ps / 2;
    const int64_t cap = 2 * nb + 2;
    const int64_t B = n_out - 2;
    TyLayout L;
    L.items_cap = nb > 65536 ? nb : 65536;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align_up(off + bytes);
        return o;
    };
    L.part = take(sizeof(TypedPartial) * (size_t)L.items_cap);
    L.pairs = take(16 * (size_t)nb);
    L.m = take(8);
    L.P = take(8 * (size_t)cap);
    L.XD = take(8 * (size_t)cap);
    L.YD = take(8 * (size_t)cap);
    L.MX = take(8 * (size_t)B);
    L.MY = take(8 * (size_t)B);
    L.path = take(seg_path_bytes(B));
    L.finals = take(seg_finals_bytes(B));
    L.start = take(seg_start_bytes(B));
    L.total = off;
    return L;
}

MinMaxGeom typed_geom(int64_t n, int64_t nb, int64_t items_cap, int yk)
{
    const Tuning &t = tuning();
    MinMaxGeom g;
    g.bins = make_split(n - 2, nb);
    const int64_t maxbin = g.bins.q + (g.bins.r ? 1 : 0);
    const int64_t gran = (yk == kYF64 ? 128 : 256) * (int64_t)t.unroll; // points per batch of loads
    const int64_t cap = items_cap / nb > 1 ? items_cap / nb : 1;
    int64_t cpb = chunks_per_bin(maxbin, nb, t.chunk);
    cpb = cpb > cap ? cap : cpb;
    int64_t chunk = (maxbin + cpb - 1) / cpb;
    chunk = (chunk + gran - 1) / gran * gran;
    g.chunk = chunk;
    g.chunks_per_bin = (maxbin + chunk - 1) / chunk;
    g.n_items = nb * g.chunks_per_bin;
    return g;
}

int check_typed(int xk, const void *x, int yk, const void *y, int64_t n, int64_t n_out, int32_t r_ps,
                int32_t min_rps)
{
    if (xk != MMLTTB_X_IMPLICIT && xk != MMLTTB_X_INT64 && xk != MMLTTB_X_F64)
        return fail(MMLTTB_EINVAL, "xk must be MMLTTB_X_IMPLICIT, MMLTTB_X_INT64 or MMLTTB_X_F64, got %d", xk);
    if ((xk == MMLTTB_X_IMPLICIT) != (x == nullptr))
        return fail(MMLTTB_EINVAL, "x must be NULL exactly when xk is MMLTTB_X_IMPLICIT");
    if (yk != MMLTTB_Y_F32 && yk != MMLTTB_Y_F64 && yk != MMLTTB_Y_I32)
        return fail(MMLTTB_EINVAL, "yk must be MMLTTB_Y_F32, MMLTTB_Y_F64 or MMLTTB_Y_I32, got %d", yk);
    const uintptr_t ysz = yk == MMLTTB_Y_F64 ? 8 : 4;
    if (!y || ((uintptr_t)y & (ysz - 1)) || ((uintptr_t)x & 7u))
        return fail(MMLTTB_EINVAL, "y must be non-NULL and aligned to its value size, x 8-byte aligned");
    if (n < 1 || n > kMaxN)
        return fail(MMLTTB_EINVAL, "n must be in [1, 2^62], got %lld", (long long)n);
    if (n_out < 3 || n_out > kMaxI32)
        return fail(MMLTTB_EINVAL, "n_out must be in [3, 2^31-1], got %lld", (long long)n_out);
    if (r_ps < min_rps)
        return fail(MMLTTB_EINVAL, "r_ps must be >= %d, got %d", min_rps, r_ps);
    if (n_out * (int64_t)r_ps / 2 > kMaxI32)
        return fail(MMLTTB_EINVAL, "floor(n_out*r_ps/2) must be <= 2^31-1");
    return MMLTTB_OK;
}

// P (with binary64 X_P, Y_P when XD != NULL) and m; n > 2.
int enqueue_typed_preselect(int xk, const void *x, int yk, const void *y, int64_t n, int64_t nb, void *ws,
                            const TyLayout &L, int64_t *P, double *XD, double *YD, int64_t *m, hipStream_t s)
{
    const MinMaxGeom g = typed_geom(n, nb, L.items_cap, yk);
    const bool all = nb >= n - 2; // every bin holds at most one point
    int64_t *pairs = at<int64_t>(ws, L.pairs);
    if (!all) {
        TypedPartial *part = at<TypedPartial>(ws, L.part);
        MMLTTB_LAUNCH("typed_bin_reduce", s, launch_typed_bin_reduce(yk, y, g, tuning().unroll, part, s));
        MMLTTB_LAUNCH("typed_bin_merge", s, launch_typed_bin_merge(part, nb, g.chunks_per_bin, pairs, s));
    }
    MMLTTB_LAUNCH("typed_compact", s, launch_typed_compact(xk, yk, pairs, g.bins, n, x, y, P, XD, YD, m, all, s));
    return MMLTTB_OK;
}

} // namespace host

int set_error(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    host::g_err = buf;
    return code;
}

} // namespace mmlttb
