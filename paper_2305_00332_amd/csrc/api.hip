// C ABI of libmmlttb: argument checks, workspace layout, launch sequences.
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <map>
#include <string>
#include <vector>

#include "errors.hpp"
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

} // namespace

namespace mmlttb {

int set_error(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

} // namespace mmlttb

namespace {

// ---------------------------------------------------------------- tuning

// Chain forms; 0 is reserved for "keep the current setting" in mmlttb_set_tuning.
enum ChainMode { kChainSequential = 1, kChainSegmented = 2, kChainAuto = 3 };

struct Tuning {
    // Defaults: the best settings the autotuner measured on MI355X (one
    // 1e9-point series; the 4096-series batch).
    int unroll = 4;              // float4 loads per lane per batch in the single-series MinMax streams
    int64_t chunk = 1 << 20;     // points per single-series MinMax work item (multiple of 256 * unroll)
    int chain = kChainAuto;
    int tile = 4096;             // batched small-bin tile points (bins of <= tile/4 points)
    int batch_unroll = 4;        // as unroll, for the batched large-bin stream
    int64_t batch_chunk = 65536; // points per batched large-bin work item (multiple of 256 * batch_unroll)
};

int64_t round_chunk(int64_t chunk, int unroll)
{
    const int64_t q = 256 * (int64_t)unroll;
    return ((chunk + q - 1) / q) * q;
}

bool valid_unroll(int u) { return u == 1 || u == 2 || u == 4 || u == 8; }

bool valid_tile(int t) { return t == 2048 || t == 4096 || t == 8192; }

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

struct Pending {
    std::string name;
    hipEvent_t a, b;
};
bool g_prof = false;
std::vector<Pending> g_pending;
std::vector<hipEvent_t> g_event_pool;
std::map<std::string, std::pair<double, int64_t>> g_totals;
std::map<std::string, std::vector<float>> g_samples; // per-launch durations, in launch order
constexpr size_t kMaxSamples = size_t(1) << 16;     // kept per name since the last reset

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

template <class F>
hipError_t timed(const char *name, hipStream_t s, F &&launch)
{
    if (!g_prof || capturing(s))
        return launch();
    hipEvent_t a = take_event(), b = take_event();
    if (!a || !b)
        return launch();
    (void)hipEventRecord(a, s);
    hipError_t e = launch();
    (void)hipEventRecord(b, s);
    g_pending.push_back({name, a, b});
    return e;
}

// Brackets a whole entry-point call with timing-only events while profiling is
// on: the span from before its first launch to after its last lands under
// `name` when close() runs (only on success; an early error return hands the
// opening event back to the pool unused).
struct CallSpan {
    const char *name;
    hipStream_t s;
    hipEvent_t a = nullptr;
    CallSpan(const char *nm, hipStream_t st) : name(nm), s(st)
    {
        if (g_prof && !capturing(s) && (a = take_event()))
            (void)hipEventRecord(a, s);
    }
    void close()
    {
        if (!a)
            return;
        hipEvent_t b = take_event();
        if (b) {
            (void)hipEventRecord(b, s);
            g_pending.push_back({name, a, b});
        } else {
            g_event_pool.push_back(a);
        }
        a = nullptr;
    }
    ~CallSpan()
    {
        if (a)
            g_event_pool.push_back(a);
    }
};

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

constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct MmLayout {
    size_t keys, m, P, XP, YP, MX, MY, path, finals, start, tiles, total;
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
    L.start = take(seg_start_bytes(B));
    L.tiles = take(8 * (size_t)compact_tiles(nb)); // first slots of the tiled compaction
    L.total = off;
    return L;
}

struct LtLayout {
    size_t MX, MY, path, finals, start, yr, cand_cnt, cand, tab, slab_hi, slab_lo, delta, brk, total;
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

int check_rps(int64_t n, int64_t n_out, int32_t r_ps, int32_t min_rps = 2)
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

#define MMLTTB_LAUNCH(name, stream, expr)                                                                              \
    do {                                                                                                               \
        hipError_t e_ = timed(name, stream, [&] { return (expr); });                                                   \
        if (e_ != hipSuccess)                                                                                          \
            return fail(MMLTTB_EDEVICE, "%s launch failed: %s", name, hipGetErrorString(e_));                          \
    } while (0)

#define MMLTTB_TRY(expr)                                                                                               \
    do {                                                                                                               \
        const int rc_ = (expr);                                                                                        \
        if (rc_ != MMLTTB_OK)                                                                                          \
            return rc_;                                                                                                \
    } while (0)

// Work items (one wave each) a stream launch should have to keep every CU
// busy: 8 waves per CU of the 256 on MI355X. Fewer, longer items leave CUs
// idle; many more add per-item reductions and merges.
constexpr int64_t kFillItems = 2048;

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

// Work items merge into their bin's keys with atomics only when bins are cut
// into several items; a single item per bin stores its keys.
bool keys_need_init(const MinMaxGeom &g) { return g.chunks_per_bin > 1; }

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
                          unsigned int *ticket = nullptr)
{
    const int64_t maxbin = g.bins.q + (g.bins.r ? 1 : 0);
    if (maxbin < kShortBin && g.bins.len >= kShortBinChunk * kFillItems) { // and at least 2048 chunks
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

template <class XT, class YT>
SegChainArgsT<XT, YT> seg_args(void *ws, size_t path, size_t finals, size_t start, const XT *XP, const YT *YP,
                               const int64_t *m_ptr, int64_t m_const, int64_t B, const double *MX, const double *MY,
                               int64_t maxb_bound)
{
    SegChainArgsT<XT, YT> a;
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

struct XbLayout {
    MmLayout mm;
    size_t bounds, m_eff, total;
};

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

struct TyLayout {
    size_t part, pairs, m, P, XD, YD, MX, MY, path, finals, start, total;
    int64_t items_cap;
};

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

// ---------------------------------------------------------------- batch plan

struct BatchPlan {
    BatchHeader h;
    std::vector<BatchSeg> segs;
    size_t total = 0;
    bool any_seq = false;
};

// Validate every segment and lay the batch out in the workspace. The layout
// depends on n_out, r_ps and the segment count only (not on lengths).
int plan_batch(int xk, const mmlttb_segment_t *in, int64_t n_segs, BatchPlan &plan)
{
    (void)xk;
    if (n_segs < 1)
        return fail(MMLTTB_EINVAL, "n_segs must be >= 1");
    if (!in)
        return fail(MMLTTB_EINVAL, "segs_host must not be NULL");
    const Tuning &tn = tuning();
    plan.segs.resize((size_t)n_segs);
    int64_t keys = 0, pslots = 0, bslots = 0, cslots = 0, large = 0, tiles = 0, cw = 0, max_stage = 0;
    for (int64_t i = 0; i < n_segs; ++i) {
        const mmlttb_segment_t &q = in[i];
        BatchSeg &g = plan.segs[(size_t)i];
        memset(&g, 0, sizeof(g));
        if (q.reserved != 0)
            return fail(MMLTTB_EINVAL, "segment %lld: reserved must be 0", (long long)i);
        if (q.offset < 0 || q.out_offset < 0)
            return fail(MMLTTB_EINVAL, "segment %lld: negative offset", (long long)i);
        if (q.n < 1 || q.n > kMaxN)
            return fail(MMLTTB_EINVAL, "segment %lld: n must be in [1, 2^62], got %lld", (long long)i, (long long)q.n);
        if (q.n_out < 3 || q.n_out > kMaxI32)
            return fail(MMLTTB_EINVAL, "segment %lld: n_out must be in [3, 2^31-1], got %lld", (long long)i,
                        (long long)q.n_out);
        int rc = check_rps(q.n, q.n_out, q.r_ps);
        if (rc) {
            std::string m = g_err;
            return fail(rc, "segment %lld: %s", (long long)i, m.c_str());
        }
        const int64_t nb = q.n_out * (int64_t)q.r_ps / 2;
        const int64_t B = q.n_out - 2;
        const int64_t S = seg_count(B);
        g.offset = q.offset;
        g.n = q.n;
        g.n_out = q.n_out;
        g.out_offset = q.out_offset;
        g.r_ps = q.r_ps;
        g.key0 = keys;
        keys += nb;
        g.p0 = pslots;
        pslots += 2 * nb + 2;
        g.B = B;
        g.b0 = bslots;
        bslots += B;
        g.c0 = cslots;
        cslots += S;
        g.mode = q.n <= q.n_out ? kSegIdentity : (nb >= q.n - 2 ? kSegAll : kSegMinMax);
        const int64_t maxb_bound = (2 * nb + B - 1) / B;
        g.seq = (tn.chain == kChainSequential || maxb_bound > kSegStarts) ? 1 : 0;
        g.cw0 = cw;
        g.cwn = 0;
        if (g.mode != kSegIdentity) {
            if (g.seq) {
                plan.any_seq = true;
            } else {
                g.cwn = S;
                cw += S;
                g.stage_cap = (int32_t)(kSegLen * maxb_bound);
                max_stage = g.stage_cap > max_stage ? g.stage_cap : max_stage;
            }
        }
        g.li0 = large;
        g.ti0 = tiles;
        if (g.mode == kSegMinMax) {
            g.bins = make_split(q.n - 2, nb);
            const int64_t maxbin = g.bins.q + (g.bins.r ? 1 : 0);
            if (maxbin <= tn.tile / 4 && nb < ((int64_t)1 << 26)) {
                int64_t G = 256;
                while (G * maxbin > tn.tile)
                    G >>= 1;
                g.small = 1;
                g.tile_bins = (int32_t)G;
                g.tn = (nb + G - 1) / G;
                tiles += g.tn;
            } else {
                g.chunk = tn.batch_chunk < kMaxStreamChunk ? tn.batch_chunk : kMaxStreamChunk;
                g.ln = (q.n - 2 + g.chunk - 1) / g.chunk;
                large += g.ln;
            }
        }
    }
    BatchHeader &h = plan.h;
    memset(&h, 0, sizeof(h));
    auto owner_table = [&](int32_t *table, int64_t total, auto start_of) {
        if (total <= 0)
            return;
        int64_t s = 0;
        for (int q = 0; q <= kOwnerTable; ++q) {
            int64_t unit = (int64_t)(((__int128)q * total) / kOwnerTable);
            unit = unit < total - 1 ? unit : total - 1;
            while (s + 1 < n_segs && start_of(plan.segs[(size_t)s + 1]) <= unit)
                ++s;
            table[q] = (int32_t)s;
        }
    };
    owner_table(h.own_large, large, [](const BatchSeg &g) { return g.li0; });
    owner_table(h.own_small, tiles, [](const BatchSeg &g) { return g.ti0; });
    owner_table(h.own_chain, cw, [](const BatchSeg &g) { return g.cw0; });
    h.n_segs = n_segs;
    h.n_keys = keys;
    h.n_large_items = large;
    h.n_small_tiles = tiles;
    h.n_chain_units = cw;
    h.max_stage_cap = max_stage;
    int64_t max_B = 0;
    for (const BatchSeg &g : plan.segs)
        if (g.mode != kSegIdentity && g.B > max_B)
            max_B = g.B;
    h.max_B = max_B;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align_up(off + bytes);
        return (int64_t)o;
    };
    take(sizeof(BatchHeader));
    h.off_segs = take((size_t)n_segs * sizeof(BatchSeg));
    h.off_keys = take(16 * (size_t)keys);
    h.off_P = take(8 * (size_t)pslots);
    h.off_XP = take(8 * (size_t)pslots);
    h.off_YP = take(4 * (size_t)pslots);
    h.off_m = take(8 * (size_t)n_segs);
    h.off_MX = take(8 * (size_t)bslots);
    h.off_MY = take(8 * (size_t)bslots);
    h.off_path = take((size_t)cslots * kSegStarts * kSegLen);
    h.off_finals = take((size_t)cslots * kSegStarts);
    h.off_start = take((size_t)cslots);
    plan.total = off;
    return MMLTTB_OK;
}

// ---------------------------------------------------------------- batch launch

void fill_table(char *dst, const BatchPlan &plan)
{
    const BatchHeader &h = plan.h;
    memset(dst, 0, (size_t)h.off_keys);
    memcpy(dst, &h, sizeof(h));
    memcpy(dst + h.off_segs, plan.segs.data(), plan.segs.size() * sizeof(BatchSeg));
}

// Enqueue the batched kernels; the header and segment table are already
// (being) copied into ws on stream s, or, when `table` is given, held there
// (device memory laid out as the start of ws).
int enqueue_batch(const BatchPlan &plan, int xk, const int64_t *x_base, const float *y_base, int64_t *out_idx_base,
                  void *ws, hipStream_t s, const void *table = nullptr)
{
    const BatchHeader &h = plan.h;
    BatchPtrs b;
    const void *tb = table ? table : ws;
    b.hdr = at<BatchHeader>(const_cast<void *>(tb), 0);
    b.segs = at<BatchSeg>(const_cast<void *>(tb), h.off_segs);
    b.n_segs = h.n_segs;
    b.xk = xk;
    b.x_base = x_base;
    b.y_base = y_base;
    b.out_base = out_idx_base;
    b.keys = at<unsigned long long>(ws, h.off_keys);
    b.P = at<int64_t>(ws, h.off_P);
    b.XP = at<int64_t>(ws, h.off_XP);
    b.YP = at<float>(ws, h.off_YP);
    b.m = at<int64_t>(ws, h.off_m);
    b.MX = at<double>(ws, h.off_MX);
    b.MY = at<double>(ws, h.off_MY);
    b.path = at<uint8_t>(ws, h.off_path);
    b.finals = at<uint8_t>(ws, h.off_finals);
    b.start = at<uint8_t>(ws, h.off_start);
    b.n_keys = h.n_keys;
    b.n_large_items = h.n_large_items;
    b.n_small_tiles = h.n_small_tiles;
    b.n_chain_units = h.n_chain_units;
    b.max_B = h.max_B;
    b.stage_cap_max = (int)(h.max_stage_cap > 0 ? h.max_stage_cap : kSegLen);
    if (h.n_large_items > 0) {
        MMLTTB_LAUNCH("batch_init", s, launch_batch_init(b, s));
        MMLTTB_LAUNCH("batch_minmax_large", s, launch_batch_large(b, tuning().batch_unroll, s));
    }
    if (h.n_small_tiles > 0) {
        MMLTTB_LAUNCH("batch_minmax_small", s, launch_batch_small(b, tuning().tile, s));
    }
    MMLTTB_LAUNCH("batch_compact", s, launch_batch_compact(b, s));
    MMLTTB_LAUNCH("batch_means", s, launch_batch_means(b, s));
    MMLTTB_LAUNCH("batch_chain", s, launch_batch_chain(b, s));
    if (plan.any_seq) {
        MMLTTB_LAUNCH("batch_chain_seq", s, launch_batch_chain_seq(b, s));
    }
    if (h.n_chain_units > 0) {
        MMLTTB_LAUNCH("batch_link_emit", s, launch_batch_link_emit(b, s));
    }
    return MMLTTB_OK;
}

// ---------------------------------------------------------------- graph cache
// Captured batched calls, keyed by everything that shapes the launch sequence
// and its arguments: pointers, stream, x kind, tuning and the segment table.

struct GraphEntry {
    uint64_t hash = 0;
    std::vector<char> key;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t done = nullptr; // recorded after the entry's latest launch
    void *table = nullptr;     // device copy of the header + segment table the captured kernels read
    uint64_t last_use = 0;
};

int g_graph_cap = 0;
std::vector<GraphEntry> g_graphs;
uint64_t g_graph_clock = 0;
int64_t g_graph_hits = 0, g_graph_captures = 0;

uint64_t fnv1a(const std::vector<char> &v)
{
    uint64_t h = 1469598103934665603ull;
    for (char c : v) {
        h ^= (unsigned char)c;
        h *= 1099511628211ull;
    }
    return h;
}

std::vector<char> graph_key(int xk, const int64_t *x_base, const float *y_base, const mmlttb_segment_t *segs,
                            int64_t n_segs, int64_t *out, void *ws, size_t ws_bytes, hipStream_t s)
{
    const Tuning &t = tuning();
    struct Head {
        int xk, unroll, chain, tile;
        int64_t chunk, n_segs;
        const void *x, *y, *out, *ws, *stream;
        size_t ws_bytes;
    } head{xk, t.batch_unroll, t.chain, t.tile, t.batch_chunk, n_segs, x_base, y_base, out, ws, (const void *)s, ws_bytes};
    std::vector<char> k(sizeof(head) + (size_t)n_segs * sizeof(mmlttb_segment_t));
    memcpy(k.data(), &head, sizeof(head));
    memcpy(k.data() + sizeof(head), segs, (size_t)n_segs * sizeof(mmlttb_segment_t));
    return k;
}

GraphEntry *graph_find(uint64_t hash, const std::vector<char> &key)
{
    for (auto &e : g_graphs) {
        if (e.hash == hash && e.key == key) {
            e.last_use = ++g_graph_clock;
            ++g_graph_hits;
            return &e;
        }
    }
    return nullptr;
}

void graph_release(GraphEntry &e)
{
    if (e.done)
        (void)hipEventSynchronize(e.done); // its last replay no longer reads the table
    if (e.exec)
        (void)hipGraphExecDestroy(e.exec);
    if (e.graph)
        (void)hipGraphDestroy(e.graph);
    if (e.done)
        (void)hipEventDestroy(e.done);
    if (e.table)
        (void)hipFree(e.table);
}

void graph_evict_oldest()
{
    if (g_graphs.empty())
        return;
    size_t oldest = 0;
    for (size_t i = 1; i < g_graphs.size(); ++i)
        if (g_graphs[i].last_use < g_graphs[oldest].last_use)
            oldest = i;
    graph_release(g_graphs[oldest]);
    g_graphs.erase(g_graphs.begin() + (long)oldest);
}

void graph_insert(GraphEntry &&e)
{
    while (!g_graphs.empty() && (int)g_graphs.size() >= g_graph_cap)
        graph_evict_oldest();
    e.last_use = ++g_graph_clock;
    ++g_graph_captures;
    g_graphs.push_back(std::move(e));
}

} // namespace

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
    const int64_t bytes = simplify_scratch_bytes(cap);
    int dev = 0, lds_max = 0, lds_optin = 0;
    if (hipGetDevice(&dev) == hipSuccess) {
        if (hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
            lds_max = 0;
        if (hipDeviceGetAttribute(&lds_optin, hipDeviceAttributeSharedMemPerBlockOptin, dev) != hipSuccess)
            lds_optin = 0;
        lds_max = lds_optin > lds_max ? lds_optin : lds_max;
    }
    bool in_lds = bytes <= (int64_t)lds_max;
    if (in_lds && bytes > 65536 && simplify_allow_lds((size_t)bytes) != hipSuccess)
        in_lds = false;
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

size_t mmlttb_batched_workspace_size(const mmlttb_segment_t *segs_host, int64_t n_segs)
{
    BatchPlan plan;
    if (plan_batch(MMLTTB_X_IMPLICIT, segs_host, n_segs, plan) != MMLTTB_OK)
        return 0;
    return plan.total;
}

int mmlttb_minmaxlttb_batched(int xk, const int64_t *x_base, const float *y_base, const mmlttb_segment_t *segs_host,
                              int64_t n_segs, int64_t *out_idx_base, void *ws, size_t ws_bytes, void *stream)
{
    if (xk != MMLTTB_X_IMPLICIT && xk != MMLTTB_X_INT64)
        return fail(MMLTTB_EINVAL, "xk must be MMLTTB_X_IMPLICIT (0) or MMLTTB_X_INT64 (1), got %d", xk);
    if (xk == MMLTTB_X_IMPLICIT && x_base)
        return fail(MMLTTB_EINVAL, "x_base must be NULL with MMLTTB_X_IMPLICIT");
    if (xk == MMLTTB_X_INT64 && !x_base)
        return fail(MMLTTB_EINVAL, "x_base must not be NULL with MMLTTB_X_INT64");
    if (!y_base || !out_idx_base)
        return fail(MMLTTB_EINVAL, "y_base and out_idx_base must not be NULL");
    if (((uintptr_t)y_base & 3u) || ((uintptr_t)x_base & 7u) || ((uintptr_t)out_idx_base & 7u))
        return fail(MMLTTB_EINVAL, "y_base must be 4-byte, x_base and out_idx_base 8-byte aligned");
    if (n_segs < 1 || !segs_host)
        return fail(MMLTTB_EINVAL, "n_segs must be >= 1 and segs_host not NULL");
    if (!ws)
        return fail(MMLTTB_EINVAL, "ws must not be NULL");
    hipStream_t s = (hipStream_t)stream;
    const bool use_graph = g_graph_cap > 0 && s != nullptr;
    std::vector<char> key;
    uint64_t hash = 0;
    if (use_graph) {
        key = graph_key(xk, x_base, y_base, segs_host, n_segs, out_idx_base, ws, ws_bytes, s);
        hash = fnv1a(key);
        if (GraphEntry *ge = graph_find(hash, key)) {
            hipError_t e = hipGraphLaunch(ge->exec, s);
            if (e == hipSuccess)
                e = hipEventRecord(ge->done, s);
            if (e != hipSuccess)
                return fail(MMLTTB_EDEVICE, "graph replay failed: %s", hipGetErrorString(e));
            return ok();
        }
    }
    BatchPlan plan;
    int rc = plan_batch(xk, segs_host, n_segs, plan);
    if (rc)
        return rc;
    if (ws_bytes < plan.total)
        return fail(MMLTTB_ENOMEM, "workspace of %zu bytes is below the %zu required", ws_bytes, plan.total);
    const BatchHeader &h = plan.h;
    const size_t table_bytes = (size_t)h.off_keys;
    if (!use_graph) {
        // header + segment table from pageable memory: copied before this call returns
        std::vector<char> staging(table_bytes);
        fill_table(staging.data(), plan);
        hipError_t e = hipMemcpyAsync(ws, staging.data(), table_bytes, hipMemcpyHostToDevice, s);
        if (e != hipSuccess)
            return fail(MMLTTB_EDEVICE, "segment table copy failed: %s", hipGetErrorString(e));
        rc = enqueue_batch(plan, xk, x_base, y_base, out_idx_base, ws, s);
        return rc ? rc : ok();
    }
    // capture: the kernels alone, reading the header and segment table from a
    // device copy owned by the graph entry (no upload node, so a replay does
    // not depend on what the workspace holds)
    GraphEntry ge;
    ge.hash = hash;
    ge.key = std::move(key);
    {
        std::vector<char> staging(table_bytes);
        fill_table(staging.data(), plan);
        if (hipMalloc(&ge.table, table_bytes) != hipSuccess) {
            ge.table = nullptr;
            return fail(MMLTTB_EDEVICE, "graph table allocation failed");
        }
        if (hipMemcpy(ge.table, staging.data(), table_bytes, hipMemcpyHostToDevice) != hipSuccess) {
            (void)hipFree(ge.table);
            return fail(MMLTTB_EDEVICE, "graph table copy failed");
        }
    }
    const bool prof = g_prof;
    g_prof = false; // no timing events inside a capture
    hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    rc = (e == hipSuccess) ? enqueue_batch(plan, xk, x_base, y_base, out_idx_base, ws, s, ge.table) : MMLTTB_EDEVICE;
    hipGraph_t graph = nullptr;
    hipError_t ec = hipStreamEndCapture(s, &graph);
    g_prof = prof;
    if (e != hipSuccess || rc != MMLTTB_OK || ec != hipSuccess || !graph) {
        if (graph)
            (void)hipGraphDestroy(graph);
        (void)hipFree(ge.table);
        return fail(MMLTTB_EDEVICE, "graph capture failed: %s", hipGetErrorString(e != hipSuccess ? e : ec));
    }
    ge.graph = graph;
    e = hipGraphInstantiate(&ge.exec, graph, nullptr, nullptr, 0);
    if (e == hipSuccess)
        e = hipEventCreateWithFlags(&ge.done, hipEventDisableTiming);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(graph);
        (void)hipFree(ge.table);
        return fail(MMLTTB_EDEVICE, "graph instantiation failed: %s", hipGetErrorString(e));
    }
    e = hipGraphLaunch(ge.exec, s);
    if (e == hipSuccess)
        e = hipEventRecord(ge.done, s);
    graph_insert(std::move(ge));
    if (e != hipSuccess)
        return fail(MMLTTB_EDEVICE, "graph launch failed: %s", hipGetErrorString(e));
    return ok();
}

int mmlttb_set_graph_cache(int max_graphs)
{
    if (max_graphs < 0)
        return fail(MMLTTB_EINVAL, "max_graphs must be >= 0");
    g_graph_cap = max_graphs;
    while ((int)g_graphs.size() > g_graph_cap)
        graph_evict_oldest();
    if (max_graphs == 0)
        g_graph_hits = g_graph_captures = 0;
    return ok();
}

int mmlttb_graph_cache_stats(int64_t *entries, int64_t *hits, int64_t *captures)
{
    if (!entries || !hits || !captures)
        return fail(MMLTTB_EINVAL, "NULL argument");
    *entries = (int64_t)g_graphs.size();
    *hits = g_graph_hits;
    *captures = g_graph_captures;
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
