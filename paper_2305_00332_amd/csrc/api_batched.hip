// C ABI of libmmlttb, batched calls: the host planner (validation, flat work
// spaces, pooled workspace slots), the launch sequence and the graph cache.
#include <stdio.h>
#include <string.h>

#include <vector>

#include "host.hpp"

using namespace mmlttb;
using namespace mmlttb::host;

namespace {

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

} // extern "C"
