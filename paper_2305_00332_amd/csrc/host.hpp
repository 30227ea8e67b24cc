// Host side of libmmlttb shared by its entry points (private to the
// library): error reporting, tuning, launch timing, workspace layouts,
// argument checks and the launch sequences several entry points share.
#pragma once

#include <stdint.h>

#include <map>
#include <string>
#include <utility>
#include <vector>

#include "kernels.hpp"
#include "libmmlttb.h"

namespace mmlttb {
namespace host {

// ---------------------------------------------------------------- errors

extern thread_local std::string g_err;
// Records the message of a failed call (printf format) and returns `code`.
int fail(int code, const char *fmt, ...);
// Clears the message; returns MMLTTB_OK.
int ok();

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

inline int64_t round_chunk(int64_t chunk, int unroll)
{
    const int64_t q = 256 * (int64_t)unroll;
    return ((chunk + q - 1) / q) * q;
}

inline bool valid_unroll(int u) { return u == 1 || u == 2 || u == 4 || u == 8; }

inline bool valid_tile(int t) { return t == 2048 || t == 4096 || t == 8192; }

// The process's tuning (compiled defaults, then the MMLTTB_* environment overrides).
Tuning &tuning();

// ---------------------------------------------------------------- profiling

struct Pending {
    std::string name;
    hipEvent_t a, b;
};

extern bool g_prof;
extern std::vector<Pending> g_pending;
extern std::vector<hipEvent_t> g_event_pool;
extern std::map<std::string, std::pair<double, int64_t>> g_totals;
extern std::map<std::string, std::vector<float>> g_samples;
constexpr size_t kMaxSamples = size_t(1) << 16; // kept per name since the last reset

hipEvent_t take_event();
bool capturing(hipStream_t s);
void drain_pending();

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

// ---------------------------------------------------------------- layout

constexpr size_t kAlign = 256;

inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct MmLayout {
    size_t keys, m, P, XP, YP, MX, MY, path, finals, start, tiles, total;
};

MmLayout mm_layout(int64_t n_out, int32_t r_ps);

struct LtLayout {
    size_t MX, MY, path, finals, start, yr, cand_cnt, cand, tab, slab_hi, slab_lo, delta, brk, total;
};

LtLayout lt_layout(int64_t n_out);

template <class T>
T *at(void *ws, size_t off)
{
    return reinterpret_cast<T *>(static_cast<char *>(ws) + off);
}

// ---------------------------------------------------------------- checks

constexpr int64_t kMaxN = (int64_t)1 << 62;
constexpr int64_t kMaxI32 = 0x7fffffff;

int check_series(int xk, const int64_t *x, const float *y, int64_t n, int64_t n_out);
int check_rps(int64_t n, int64_t n_out, int32_t r_ps, int32_t min_rps = 2);

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

// ---------------------------------------------------------------- MinMax stream and preselection

// Work items (one wave each) a stream launch should have to keep every CU
// busy: 8 waves per CU of the 256 on MI355X. Fewer, longer items leave CUs
// idle; many more add per-item reductions and merges.
constexpr int64_t kFillItems = 2048;

int64_t chunks_per_bin(int64_t maxbin, int64_t nb, int64_t chunk);
// Work items merge into their bin's keys with atomics only when bins are cut
// into several items; a single item per bin stores its keys.
inline bool keys_need_init(const MinMaxGeom &g) { return g.chunks_per_bin > 1; }

MinMaxGeom minmax_geom(int64_t len, int64_t nb);
// `ticket` (optional): cleared on the way for a k_preselect_tail launch.
int enqueue_minmax_stream(const float *y, const MinMaxGeom &g, unsigned long long *keys, hipStream_t s,
                          unsigned int *ticket = nullptr);
bool use_segmented_chain(int64_t maxb_bound);

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

int enqueue_preselect(const int64_t *x, const float *y, int64_t n, int64_t n_out, int32_t r_ps, void *ws,
                      const MmLayout &L, int64_t *P, int64_t *XP, float *YP, int64_t *m_out, hipStream_t s);

// ---------------------------------------------------------------- x-width bins

struct XbLayout {
    MmLayout mm;
    size_t bounds, m_eff, total;
};

XbLayout xb_layout(int64_t n_out, int32_t r_ps);
int check_xbins(const int64_t *x, const float *y, int64_t n, int64_t n_out, int32_t r_ps, int32_t min_rps);
int enqueue_xbin_stream(const int64_t *x, const float *y, int64_t n, int64_t nb, void *ws, const XbLayout &L,
                        hipStream_t s);

// ---------------------------------------------------------------- other value types

struct TyLayout {
    size_t part, pairs, m, P, XD, YD, MX, MY, path, finals, start, total;
    int64_t items_cap;
};

TyLayout ty_layout(int64_t n_out, int32_t r_ps);
MinMaxGeom typed_geom(int64_t n, int64_t nb, int64_t items_cap, int yk);
int check_typed(int xk, const void *x, int yk, const void *y, int64_t n, int64_t n_out, int32_t r_ps,
                int32_t min_rps);
int enqueue_typed_preselect(int xk, const void *x, int yk, const void *y, int64_t n, int64_t nb, void *ws,
                            const TyLayout &L, int64_t *P, double *XD, double *YD, int64_t *m, hipStream_t s);

} // namespace host
} // namespace mmlttb
