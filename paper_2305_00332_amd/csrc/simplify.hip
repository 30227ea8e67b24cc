// Other line simplifiers on the MinMax-preselected points (section 4 names
// them as future work): Visvalingam-Whyatt (VW), Douglas-Peucker with a point
// budget (DP) and Longest-Line-Bucket (LLB). Each runs on the m preselected
// points of one series in one wave, with the per-point state (binary64
// coordinates, areas / keys / path lengths, links) in LDS when it fits and in
// the caller's workspace otherwise (the same code through generic pointers).
//
// VW and DP are greedy: each step takes the extreme of a set that changes by
// a few entries. A 64-ary tournament tree of (key, index) minima finds it: a
// changed leaf costs one wave reduction per level, the root one more. VW's
// smallest area and DP's largest key (lowest index on ties) both map to a
// minimum of a 64-bit key. LLB is a dynamic program over LTTB's buckets
// (lanes over the current bucket's points), then a walk back along the
// recorded predecessors.
#include "device_common.hpp"
#include "kernels.hpp"

namespace mmlttb {

struct TNode {
    uint64_t k;
    int64_t i;
};

// One DPP step of a lexicographic (key, index) minimum.
template <int CTRL>
__device__ inline void argmin_step(uint64_t &k, int32_t &i)
{
    const uint32_t lo = (uint32_t)dpp_i32<CTRL>((int)(uint32_t)k);
    const uint32_t hi = (uint32_t)dpp_i32<CTRL>((int)(uint32_t)(k >> 32));
    const int32_t oi = dpp_i32<CTRL>(i);
    const uint64_t ok = ((uint64_t)hi << 32) | lo;
    if (ok < k || (ok == k && oi < i)) {
        k = ok;
        i = oi;
    }
}

// Levels l = 1..T above m leaves; level T holds at most 64 nodes. Every
// loop over levels is unrolled to kMaxLevels so the level arrays stay in
// registers (a runtime index would put them in private memory).
constexpr int kMaxLevels = 6; // 64^6 leaves
struct Tree {
    TNode *node;
    int64_t off[kMaxLevels + 1], cnt[kMaxLevels + 1];
    int T;
    int64_t top_off, top_cnt; // level T (the leaves when T = 0)
};

__host__ __device__ inline int64_t tree_nodes(int64_t m, Tree *t)
{
    int64_t c = m, total = 0;
    int T = 0;
    if (t) {
        t->cnt[0] = m;
        t->off[0] = 0;
        t->top_off = 0;
        t->top_cnt = m;
    }
#pragma unroll
    for (int l = 1; l <= kMaxLevels; ++l) {
        const bool more = c > 64;
        const int64_t cn = more ? (c + 63) / 64 : c;
        if (t) {
            t->off[l] = total;
            t->cnt[l] = cn;
            if (more) {
                t->top_off = total;
                t->top_cnt = cn;
            }
        }
        if (more) {
            total += cn;
            T = l;
        }
        c = cn;
    }
    if (t)
        t->T = T;
    return total;
}

// Per-point state: X, Y, F (binary64), A, N (int32) for `cap` points, then
// the tree nodes. Offsets are multiples of 16 bytes.
__host__ __device__ inline int64_t simplify_state_bytes(int64_t cap)
{
    const int64_t c16 = (cap + 1) / 2 * 2;
    return c16 * (8 * 3 + 4 * 2) + 16 * tree_nodes(cap, nullptr);
}

struct SimplifyState {
    double *X, *Y, *F;
    int32_t *A, *N;
    Tree t;
};

__device__ inline SimplifyState carve_state(unsigned char *base, int64_t cap, int64_t m)
{
    const int64_t c16 = (cap + 1) / 2 * 2;
    SimplifyState s;
    s.X = reinterpret_cast<double *>(base);
    s.Y = s.X + c16;
    s.F = s.Y + c16;
    s.A = reinterpret_cast<int32_t *>(s.F + c16);
    s.N = s.A + c16;
    tree_nodes(m, &s.t);
    s.t.node = reinterpret_cast<TNode *>(s.N + c16);
    return s;
}

// Smallest int32 over the wave; every lane active.
__device__ inline int32_t wave_min_i32(int32_t v)
{
    v = min(v, dpp_i32<0xB1>(v));
    v = min(v, dpp_i32<0x4E>(v));
    v = min(v, dpp_i32<0x141>(v));
    v = min(v, dpp_i32<0x140>(v));
    const int32_t a = min(__builtin_amdgcn_readlane(v, 0), __builtin_amdgcn_readlane(v, 16));
    const int32_t b = min(__builtin_amdgcn_readlane(v, 32), __builtin_amdgcn_readlane(v, 48));
    return min(a, b);
}

// Smallest key over the wave, lowest index on ties; every lane active. DPP
// within rows of 16 lanes, then the four row results through readlane.
__device__ inline void wave_argmin(uint64_t k, int64_t i64, uint64_t &ko, int64_t &io)
{
    int32_t i = i64 > INT32_MAX ? INT32_MAX : (int32_t)i64;
    argmin_step<0xB1>(k, i);
    argmin_step<0x4E>(k, i);
    argmin_step<0x141>(k, i);
    argmin_step<0x140>(k, i);
    uint64_t bk = (uint64_t)readlane_i64((int64_t)k, 0);
    int32_t bi = __builtin_amdgcn_readlane(i, 0);
#pragma unroll
    for (int r = 16; r < kWave; r += 16) {
        const uint64_t rk = (uint64_t)readlane_i64((int64_t)k, r);
        const int32_t ri = __builtin_amdgcn_readlane(i, r);
        if (rk < bk || (rk == bk && ri < bi)) {
            bk = rk;
            bi = ri;
        }
    }
    ko = bk;
    io = bi == INT32_MAX ? INT64_MAX : bi;
}

// Node (l, g) from its 64 children.
template <class LeafKey>
__device__ inline void tree_node(Tree &t, int l, int64_t g, LeafKey lk, int lane)
{
    const int64_t c = (g << 6) + lane;
    uint64_t k = ~0ull;
    int64_t i = INT64_MAX;
    if (c < t.cnt[l - 1]) {
        if (l == 1) {
            k = lk(c);
            i = c;
        } else {
            const TNode n = t.node[t.off[l - 1] + c];
            k = n.k;
            i = n.i;
        }
    }
    wave_argmin(k, i, k, i);
    if (lane == 0)
        t.node[t.off[l] + g] = TNode{k, i};
    __syncthreads(); // one-wave workgroup: the write is visible to every lane after this
}

template <class LeafKey>
__device__ inline void tree_build(Tree &t, LeafKey lk, int lane)
{
#pragma unroll
    for (int l = 1; l <= kMaxLevels; ++l) {
        if (l > t.T)
            break;
        for (int64_t g = 0; g < t.cnt[l]; ++g)
            tree_node(t, l, g, lk, lane);
    }
}

// The path from `leaf` to the top after its key (or a sibling's) changed.
template <class LeafKey>
__device__ inline void tree_fix(Tree &t, int64_t leaf, LeafKey lk, int lane)
{
#pragma unroll
    for (int l = 1; l <= kMaxLevels; ++l) {
        if (l > t.T)
            break;
        tree_node(t, l, leaf >> (6 * l), lk, lane);
    }
}

// Index of the smallest key (lowest index on ties), uniform across the wave.
template <class LeafKey>
__device__ inline int64_t tree_root(const Tree &t, LeafKey lk, int lane, uint64_t &key)
{
    uint64_t k = ~0ull;
    int64_t i = INT64_MAX;
    if (lane < t.top_cnt) {
        if (t.T == 0) {
            k = lk(lane);
            i = lane;
        } else {
            const TNode n = t.node[t.top_off + lane];
            k = n.k;
            i = n.i;
        }
    }
    wave_argmin(k, i, key, i);
    return i;
}

__device__ inline uint64_t f64_bits(double v) { return (uint64_t)__double_as_longlong(v); }

// Order key of a binary64 (unsigned integers ordered like the numbers).
__device__ inline uint64_t f64_okey(double v)
{
    uint64_t u = f64_bits(v);
    u = (u == 0x8000000000000000ull) ? 0ull : u;
    return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}

// Stage X, Y of the m points; returns false (identity output written) when
// m <= n_out.
__device__ inline bool simplify_begin(const SimplifyArgs &a, SimplifyState &s, int64_t m, int lane)
{
    if (m <= a.n_out) {
        for (int64_t i = lane; i < m; i += kWave)
            a.out[i] = a.Pmap[i];
        return false;
    }
    for (int64_t i = lane; i < m; i += kWave) {
        s.X[i] = (double)(a.XP ? a.XP[i] : i);
        s.Y[i] = (double)a.YP[i];
    }
    __syncthreads();
    return true;
}

// Output the kept points (keep(i) true) in index order, mapped through P.
template <class Keep>
__device__ inline void simplify_emit(const SimplifyArgs &a, int64_t m, Keep keep, int lane)
{
    int64_t count = 0;
    for (int64_t base = 0; base < m; base += kWave) {
        const int64_t i = base + lane;
        const bool k = i < m && keep(i);
        const unsigned long long mask = __builtin_amdgcn_ballot_w64(k);
        const unsigned long long below = lane ? (mask & ((1ull << lane) - 1ull)) : 0ull;
        if (k)
            a.out[count + __popcll(below)] = a.Pmap[i];
        count += __popcll(mask);
    }
}

// kLds: the state is the dynamic LDS array (native LDS addressing); else the
// workspace.
template <bool kLds>
__device__ inline unsigned char *state_base(const SimplifyArgs &a, unsigned char *lds)
{
    return kLds ? lds : a.scratch;
}

// ------------------------------------------------------------------ VW

__device__ inline double vw_area(const SimplifyState &s, int64_t p, int64_t j, int64_t q)
{
    return fabs((s.X[p] - s.X[q]) * (s.Y[j] - s.Y[p]) - (s.X[p] - s.X[j]) * (s.Y[q] - s.Y[p]));
}

template <bool kLds>
__global__ __launch_bounds__(64) void k_simplify_vw(SimplifyArgs a)
{
    extern __shared__ __align__(16) unsigned char lds[];
    const int lane = threadIdx.x;
    const int64_t m = *a.m_ptr;
    SimplifyState s = carve_state(state_base<kLds>(a, lds), a.cap, m);
    if (!simplify_begin(a, s, m, lane))
        return;
    // A = previous alive point (-2 once removed), N = next alive point, F = area
    for (int64_t i = lane; i < m; i += kWave) {
        s.A[i] = (int32_t)(i - 1);
        s.N[i] = (int32_t)(i + 1);
        s.F[i] = (i > 0 && i < m - 1) ? vw_area(s, i - 1, i, i + 1) : 0.0;
    }
    __syncthreads();
    auto lk = [&](int64_t i) -> uint64_t {
        return (i == 0 || i == m - 1 || s.A[i] == -2) ? ~0ull : f64_bits(s.F[i]); // areas are >= 0
    };
    tree_build(s.t, lk, lane);
    for (int64_t left = m; left > a.n_out; --left) {
        uint64_t key;
        const int64_t sel = tree_root(s.t, lk, lane, key);
        if (sel <= 0 || sel >= m - 1)
            break; // no interior point left (not reachable while left > n_out >= 3)
        const int64_t p = s.A[sel], q = s.N[sel];
        if (lane == 0) {
            s.N[p] = (int32_t)q;
            s.A[q] = (int32_t)p;
            s.A[sel] = -2;
        } else if (lane == 1 && p > 0) {
            s.F[p] = vw_area(s, s.A[p], p, q);
        } else if (lane == 2 && q < m - 1) {
            s.F[q] = vw_area(s, p, q, s.N[q]);
        }
        __syncthreads();
        tree_fix(s.t, sel, lk, lane);
        if ((p >> 6) != (sel >> 6))
            tree_fix(s.t, p, lk, lane);
        if ((q >> 6) != (sel >> 6))
            tree_fix(s.t, q, lk, lane);
    }
    simplify_emit(a, m, [&](int64_t i) { return s.A[i] != -2; }, lane);
}

// ------------------------------------------------------------------ DP

// Farthest interior point of segment (p, q) into A[p] (-1 if none) and its
// key into F[p]; the whole wave scans.
__device__ inline void dp_scan(SimplifyState &s, int64_t p, int64_t q, int lane)
{
    const double xp = s.X[p], yp = s.Y[p], dx = s.X[q] - xp, dy = s.Y[q] - yp;
    double best = -1.0;
    int32_t bj = INT32_MAX;
    for (int64_t j = p + 1 + lane; j < q; j += kWave) {
        const double c = fabs(dx * (s.Y[j] - yp) - (s.X[j] - xp) * dy);
        if (c > best) { // increasing j per lane: lowest index on ties
            best = c;
            bj = (int32_t)j;
        }
    }
    const double wb = wave_max_f64(best);
    const int32_t j = wave_min_i32(best == wb ? bj : INT32_MAX);
    if (lane == 0) {
        if (wb > -1.0) {
            double key = wb * wb / (dx * dx + dy * dy);
            s.F[p] = (key != key) ? -1.0 : key; // a zero-length chord counts as -1
            s.A[p] = (int32_t)j;
        } else {
            s.A[p] = -1;
        }
    }
    __syncthreads();
}

// ------------------------------------------------------------------ DP (split tree)
//
// The greedy loop above keeps, at every step, the farthest point of the
// segment with the largest key. Give each point that some segment would split
// at (recursing from the whole series down to segments with no interior
// point) a node in the split tree and the priority pi = (key, lower index
// first): the greedy loop is a best-first walk of that tree from the root. A
// best-first walk takes the nodes in decreasing order of their bottleneck,
// the node of lowest priority on the path from the root, and takes the nodes
// that share one bottleneck u (u's cluster) one after the other, u first.
// So the first n_out - 2 steps take every cluster whose bottleneck ranks
// above that of the cluster holding step n_out - 2, and a best-first walk of
// the rest inside that one cluster.
//
// One workgroup builds the tree a level at a time (each level: every
// interior point moves to the part of its segment it lies in and takes its
// distance into that segment's best by atomic maximum; the lowest index
// among the points reaching the best, by atomic minimum; the splits), ranks
// the clusters by a radix select over (bottleneck priority, bottleneck
// index), and walks the boundary cluster in one wave. The state (40 bytes a
// point) sits in LDS up to about 4000 points, else in the workspace. Trees
// deeper than kDpMaxLevels (below n_out - 2) and boundary walks longer than
// kDpMaxSteps steps or over more than kDpMaxCluster nodes are left to the
// greedy loop, which runs after this kernel only when the gate says so.
constexpr int kDpThreads = 1024;
constexpr int kDpWaves = kDpThreads / kWave;
constexpr int kDpMaxLevels = 512;
constexpr int kDpMaxSteps = 256;
constexpr int kDpMaxCluster = 512;
constexpr int kDpPerLane = kDpMaxCluster / kWave;
constexpr int kDpBatch = 4; // points a thread takes at once in the tree's passes

__host__ __device__ inline int64_t dp_c4(int64_t cap) { return (cap + 3) / 4 * 4; }
// X, F (binary64), Y (binary32: the points' y exactly), N, OWN, SP, bot, par (int32)
__host__ __device__ inline int64_t dp_state_bytes(int64_t cap) { return dp_c4(cap) * (8 * 2 + 4 * 6); }
// The boundary cluster's node list, in the workspace past the state.
__host__ __device__ inline int64_t dp_list_bytes() { return 16 * kDpMaxCluster; }
// The gate sits past both the greedy loop's state and the tree's, so neither overwrites it.
__host__ __device__ inline int64_t dp_gate_offset(int64_t cap)
{
    const int64_t t = dp_state_bytes(cap) + dp_list_bytes(), g = simplify_state_bytes(cap);
    return ((t > g ? t : g) + 15) / 16 * 16;
}
__device__ inline int32_t *dp_gate(const SimplifyArgs &a)
{
    return reinterpret_cast<int32_t *>(a.scratch + dp_gate_offset(a.cap));
}

struct DpState {
    // X: x. F: a node's key; for an interior point j, the best distance
    // (bits + 1, 0: none yet) of the segment that starts at j - 1.
    double *X, *F;
    float *Y;
    // N: next kept point (-1: not kept). OWN: for an interior point, the start
    // of its segment as of the last level (the segment may have split since);
    // for a kept point, the lowest farthest point of the segment it starts
    // (INT32_MAX outside the pass that finds it and the split that uses it).
    int32_t *N, *OWN;
    // SP: node whose split made the segment a kept point starts (-1: the whole
    // series); bot: the node's bottleneck; par: its parent node.
    int32_t *SP, *bot, *par;
    uint4 *list; // boundary cluster: (key bits lo, hi, node, list slot of its parent)
};

__device__ inline DpState dp_carve(unsigned char *base, unsigned char *scratch, int64_t cap)
{
    const int64_t c4 = dp_c4(cap);
    DpState s;
    s.X = reinterpret_cast<double *>(base);
    s.F = s.X + c4;
    s.Y = reinterpret_cast<float *>(s.F + c4);
    s.N = reinterpret_cast<int32_t *>(s.Y + c4);
    s.OWN = s.N + c4;
    s.SP = s.OWN + c4;
    s.bot = s.SP + c4;
    s.par = s.bot + c4;
    s.list = reinterpret_cast<uint4 *>(scratch + dp_state_bytes(cap));
    return s;
}

// Distance term of point j to the chord (p, q), as dp_scan computes it.
__device__ inline double dp_dist(const DpState &s, int p, int q, int j)
{
    const double xp = s.X[p], yp = (double)s.Y[p], dx = s.X[q] - xp, dy = (double)s.Y[q] - yp;
    return fabs(dx * ((double)s.Y[j] - yp) - (s.X[j] - xp) * dy);
}

// Add one to hist[dig] for every lane with `on`: one LDS atomic when every
// such lane of the wave has the same digit (the leading digits of nearby
// keys), else one per lane.
__device__ inline void dp_hist_add(uint32_t *hist, bool on, uint32_t dig, int lane)
{
    const unsigned long long act = __builtin_amdgcn_ballot_w64(on);
    if (act == 0)
        return;
    const int leader = __builtin_ctzll(act);
    const uint32_t d0 = (uint32_t)__builtin_amdgcn_readlane((int)dig, leader);
    if (__builtin_amdgcn_ballot_w64(on && dig != d0) == 0) {
        if (lane == leader)
            atomicAdd(&hist[d0], (uint32_t)__popcll(act));
    } else if (on) {
        atomicAdd(&hist[dig], 1u);
    }
}

struct DpShared {
    int32_t cnt[2];                // some split made at the current / next level (a flag); list slots
    uint32_t hist[2][256];         // radix select, one per digit parity
    uint32_t wc[2][kDpWaves];      // per-wave counts (node count, output)
    unsigned long long pick[2][3]; // radix select, one per digit parity: digit, rank left, count in digit
};

template <bool kLds>
__global__ __launch_bounds__(kDpThreads) void k_simplify_dp_tree(SimplifyArgs a)
{
    extern __shared__ __align__(16) unsigned char lds[];
    __shared__ DpShared sh;
    int32_t *s_cnt = sh.cnt;
    auto &s_wc = sh.wc;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    const int64_t m64 = *a.m_ptr;
    int32_t *gate = dp_gate(a);
    if (m64 <= a.n_out) {
        for (int64_t i = tid; i < m64; i += kDpThreads)
            a.out[i] = a.Pmap[i];
        if (tid == 0)
            *gate = 0;
        return;
    }
    const int m = (int)m64; // m <= cap < 2^31
    const int K = (int)(a.n_out - 2);
    DpState s = dp_carve(kLds ? lds : a.scratch, a.scratch, a.cap);
    unsigned long long *Fb = reinterpret_cast<unsigned long long *>(s.F);
    for (int i = tid; i < m; i += kDpThreads) {
        s.X[i] = (double)(a.XP ? a.XP[i] : i);
        s.Y[i] = a.YP[i];
        s.F[i] = 0.0;
        s.N[i] = i == 0 ? m - 1 : (i == m - 1 ? m : -1);
        s.OWN[i] = (i == 0 || i == m - 1) ? INT32_MAX : 0;
    }
    if (tid == 0) {
        s.SP[0] = -1;
        s_cnt[0] = s_cnt[1] = 0;
    }
    __syncthreads();

    // ---- the split tree, one level (one depth) at a time; nodes deeper than
    // K - 1 are never among the first K steps
    const int L = K < kDpMaxLevels ? K : kDpMaxLevels;
    bool split_last = true; // the last level built split some segment
    for (int level = 0; level < L; ++level) {
        // interior points move to the part of their segment they lie in (its
        // split, if any, is now N of its start) and take their distances into
        // the segment bests. Each thread takes kDpBatch points at once, every
        // round of loads issued for all of them before the next; a wave with
        // no interior point in the batch skips it.
        for (int i0 = 0; i0 < m; i0 += kDpBatch * kDpThreads) { // uniform trip count: whole waves aggregate
            int idx[kDpBatch], p[kDpBatch], q[kDpBatch];
            bool in[kDpBatch], moved[kDpBatch], any = false;
#pragma unroll
            for (int u = 0; u < kDpBatch; ++u) {
                idx[u] = i0 + u * kDpThreads + tid;
                in[u] = idx[u] < m && s.N[idx[u]] < 0;
                any = any || in[u];
            }
            if (__builtin_amdgcn_ballot_w64(any) == 0)
                continue;
#pragma unroll
            for (int u = 0; u < kDpBatch; ++u)
                p[u] = in[u] ? s.OWN[idx[u]] : 0;
#pragma unroll
            for (int u = 0; u < kDpBatch; ++u)
                q[u] = in[u] ? s.N[p[u]] : 0;
#pragma unroll
            for (int u = 0; u < kDpBatch; ++u) {
                moved[u] = in[u] && q[u] < idx[u]; // the segment split at q, left of the point
                p[u] = moved[u] ? q[u] : p[u];
            }
#pragma unroll
            for (int u = 0; u < kDpBatch; ++u)
                q[u] = moved[u] ? s.N[p[u]] : q[u];
            int seg[kDpBatch];
            unsigned long long kb[kDpBatch];
#pragma unroll
            for (int u = 0; u < kDpBatch; ++u) {
                const double c = in[u] ? dp_dist(s, p[u], q[u], idx[u]) : 0.0;
                const bool cand = in[u] && c == c; // a NaN distance never wins
                seg[u] = cand ? p[u] : -1;
                kb[u] = cand ? f64_bits(c) + 1 : 0; // c >= 0: the bits order like the values
            }
#pragma unroll
            for (int u = 0; u < kDpBatch; ++u) {
                if (moved[u])
                    s.OWN[idx[u]] = p[u];
            }
#pragma unroll
            for (int u = 0; u < kDpBatch; ++u) {
                const int seg0 = __builtin_amdgcn_readfirstlane(seg[u]);
                if (seg0 >= 0 && __builtin_amdgcn_ballot_w64(seg[u] == seg0 || seg[u] < 0) == ~0ull) {
                    // every candidate of the wave is in lane 0's segment: one atomic
                    unsigned long long dummy = ~0ull, best = kb[u];
                    wave_minmax_u64(dummy, best);
                    if (lane == 0)
                        atomicMax(&Fb[seg0 + 1], best);
                } else if (seg[u] >= 0) {
                    atomicMax(&Fb[seg[u] + 1], kb[u]);
                }
            }
        }
        __syncthreads();
        // the lowest index reaching its segment's best
        for (int i0 = 0; i0 < m; i0 += kDpBatch * kDpThreads) {
            int idx[kDpBatch], p[kDpBatch];
            bool in[kDpBatch], any = false;
#pragma unroll
            for (int u = 0; u < kDpBatch; ++u) {
                idx[u] = i0 + u * kDpThreads + tid;
                in[u] = idx[u] < m && s.N[idx[u]] < 0;
                any = any || in[u];
            }
            if (__builtin_amdgcn_ballot_w64(any) == 0)
                continue;
#pragma unroll
            for (int u = 0; u < kDpBatch; ++u)
                p[u] = in[u] ? s.OWN[idx[u]] : 0;
            unsigned long long best[kDpBatch];
            int q[kDpBatch];
#pragma unroll
            for (int u = 0; u < kDpBatch; ++u) {
                q[u] = in[u] ? s.N[p[u]] : 0;
                best[u] = in[u] ? Fb[p[u] + 1] : 0;
            }
#pragma unroll
            for (int u = 0; u < kDpBatch; ++u) {
                if (in[u]) {
                    const double c = dp_dist(s, p[u], q[u], idx[u]);
                    if (c == c && f64_bits(c) + 1 == best[u])
                        atomicMin(&s.OWN[p[u]], idx[u]);
                }
            }
        }
        __syncthreads();
        // the splits. A segment start made by this pass has a cleared best
        // (0) when another thread reads it, so it is skipped either way.
        for (int i = tid; i < m - 1; i += kDpThreads) {
            const int b = s.N[i];
            if (b < 0 || b - i < 2)
                continue;
            const unsigned long long kb = Fb[i + 1];
            if (kb == 0)
                continue; // no live interior point with a distance
            const int j = s.OWN[i];
            // both kept points' best-split slots start the next level cleared
            s.OWN[i] = INT32_MAX;
            s.OWN[j] = INT32_MAX;
            const double c = __longlong_as_double((long long)(kb - 1));
            const double dx = s.X[b] - s.X[i], dy = (double)s.Y[b] - (double)s.Y[i];
            double key = c * c / (dx * dx + dy * dy);
            key = (key != key) ? -1.0 : key; // a zero-length chord counts as -1
            const int p = s.SP[i];
            s.F[j] = key;
            s.par[j] = p;
            int bt = j;
            if (p >= 0) {
                // j is its own bottleneck when pi(j) < pi(the parent's
                // bottleneck): a smaller key, or the same key and a higher index
                const int bp = s.bot[p];
                const double fb = s.F[bp];
                bt = (key < fb || (key == fb && j > bp)) ? j : bp;
            }
            s.bot[j] = bt;
            s.N[i] = j;
            s.N[j] = b;
            s.SP[i] = j;
            s.SP[j] = j;
            if (j - i >= 2)
                Fb[i + 1] = 0;
            if (b - j >= 2)
                Fb[j + 1] = 0;
            s_cnt[level & 1] = 1; // a flag: every writer stores the same value
        }
        __syncthreads();
        const int made = s_cnt[level & 1];
        if (tid == 0)
            s_cnt[(level + 1) & 1] = 0; // last read before the previous level's final barrier
        split_last = made > 0;
        if (!split_last)
            break;
    }
    if (split_last && L < K) { // the tree may go deeper than kDpMaxLevels
        if (tid == 0)
            *gate = 1;
        return;
    }

    // ---- cluster keys: (bottleneck priority, bottleneck index) of every
    // node, larger first. X holds the priority's order key, N the index
    // part (m - 1 - bottleneck), OWN 1 for a node, 2 once kept.
    unsigned long long *Xk = reinterpret_cast<unsigned long long *>(s.X);
    uint32_t nodes_w = 0;
    for (int i0 = 0; i0 < m; i0 += kDpThreads) {
        const int i = i0 + tid;
        const bool node = i > 0 && i < m - 1 && s.N[i] >= 0;
        if (i < m) {
            if (node) {
                const int u = s.bot[i];
                Xk[i] = f64_okey(s.F[u]);
                s.N[i] = m - 1 - u;
            }
            s.OWN[i] = node ? 1 : 0;
        }
        nodes_w += (uint32_t)__popcll(__builtin_amdgcn_ballot_w64(node));
    }
    if (lane == 0)
        s_wc[0][wave] = nodes_w;
    __syncthreads();
    int nodes = 0;
    for (int w = 0; w < kDpWaves; ++w)
        nodes += (int)s_wc[0][w];
    __syncthreads(); // s_wc is rewritten below

    if (nodes > K) {
        // K-th largest cluster key: radix select, 8-bit digits, the
        // priority's 64 bits first, then as many of the index part as m needs
        const int lo_bits = 32 - __builtin_clz((unsigned)(m - 1) | 1u);
        const int lo_digits = (lo_bits + 7) / 8;
        unsigned long long pre_hi = 0, msk_hi = 0;
        uint32_t pre_lo = 0, msk_lo = 0;
        int k = K; // rank (from 1) of the sought key among those matching the prefix
        int in_digit = 0;
        if (tid < 256)
            sh.hist[0][tid] = 0;
        __syncthreads();
        for (int d = 0; d < 8 + lo_digits; ++d) {
            const bool on_hi = d < 8;
            const int shift = on_hi ? 56 - 8 * d : 8 * (lo_digits - 1 - (d - 8));
            uint32_t *s_hist = sh.hist[d & 1];
            unsigned long long *s_pick = sh.pick[d & 1];
            for (int i0 = 0; i0 < m; i0 += kDpThreads) {
                const int i = i0 + tid;
                bool on = false;
                uint32_t dig = 0;
                if (i < m && s.OWN[i] == 1) {
                    const unsigned long long h = Xk[i];
                    const uint32_t l = (uint32_t)s.N[i];
                    on = (h & msk_hi) == pre_hi && (l & msk_lo) == pre_lo;
                    dig = on_hi ? (uint32_t)(h >> shift) & 255u : (l >> shift) & 255u;
                }
                dp_hist_add(s_hist, on, dig, lane);
            }
            __syncthreads();
            if (wave == 0) {
                // lane l holds digits 255 - 4l .. 252 - 4l (largest first)
                uint32_t c[4], t = 0;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    c[e] = s_hist[255 - 4 * lane - e];
                    t += c[e];
                }
                uint32_t incl = t; // inclusive scan over lanes
#pragma unroll
                for (int off = 1; off < kWave; off <<= 1) {
                    const uint32_t o = (uint32_t)__shfl_up((int)incl, off);
                    if (lane >= off)
                        incl += o;
                }
                const uint32_t excl = incl - t;
                if (excl < (uint32_t)k && (uint32_t)k <= incl) { // one lane
                    uint32_t before = excl;
                    int e = 0;
                    while (before + c[e] < (uint32_t)k) {
                        before += c[e];
                        ++e;
                    }
                    s_pick[0] = (unsigned long long)(255 - 4 * lane - e);
                    s_pick[1] = (unsigned long long)((uint32_t)k - before);
                    s_pick[2] = (unsigned long long)c[e];
                }
                // the next digit's histogram: its last readers passed the barrier above
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    sh.hist[(d + 1) & 1][4 * lane + e] = 0;
            }
            __syncthreads();
            const unsigned long long dig = s_pick[0];
            k = (int)s_pick[1];
            in_digit = (int)s_pick[2];
            if (on_hi) {
                pre_hi |= dig << shift;
                msk_hi |= 255ull << shift;
            } else {
                pre_lo |= (uint32_t)dig << shift;
                msk_lo |= 255u << shift;
            }
            // this digit's pick and histogram are next written two digits on,
            // after the next digit's barriers
        }
        // clusters above the boundary cluster are kept whole; k nodes of the
        // boundary cluster (in_digit nodes) follow
        const int r = k, cs = in_digit;
        const int head = m - 1 - (int)pre_lo;
        for (int i = tid; i < m; i += kDpThreads) {
            if (s.OWN[i] == 1) {
                const unsigned long long h = Xk[i];
                const uint32_t l = (uint32_t)s.N[i];
                const bool above = h > pre_hi || (h == pre_hi && l > pre_lo);
                const bool same = h == pre_hi && l == pre_lo;
                if (above || (same && r == cs))
                    s.OWN[i] = 2;
            }
        }
        if (r < cs) {
            if (cs > kDpMaxCluster || r > kDpMaxSteps) {
                if (tid == 0)
                    *gate = 1;
                return;
            }
            // list the boundary cluster; SP (no longer needed) maps a node to its slot
            if (tid == 0)
                s_cnt[0] = 0;
            __syncthreads();
            for (int i = tid; i < m; i += kDpThreads) {
                if (s.OWN[i] == 1 && Xk[i] == pre_hi && (uint32_t)s.N[i] == pre_lo) {
                    const int slot = atomicAdd(&s_cnt[0], 1);
                    s.SP[i] = slot;
                    const unsigned long long ok = f64_okey(s.F[i]);
                    s.list[slot] = make_uint4((uint32_t)ok, (uint32_t)(ok >> 32), (uint32_t)i, 0u);
                }
            }
            __syncthreads();
            for (int e = tid; e < cs; e += kDpThreads) {
                const int v = (int)s.list[e].z;
                s.list[e].w = (uint32_t)(v == head ? -1 : s.SP[s.par[v]]);
            }
            __syncthreads();
            if (wave == 0) {
                // best-first inside the cluster from its head, in registers:
                // lane l holds slots l, l + 64, ...
                uint64_t ek[kDpPerLane];
                int ev[kDpPerLane], ep[kDpPerLane];
                bool avail[kDpPerLane], taken[kDpPerLane];
#pragma unroll
                for (int t = 0; t < kDpPerLane; ++t) {
                    const int e = lane + t * kWave;
                    const bool in = e < cs;
                    const uint4 q = in ? s.list[e] : make_uint4(0u, 0u, 0u, 0u);
                    ek[t] = ~(((unsigned long long)q.y << 32) | q.x); // larger key first
                    ev[t] = in ? (int)q.z : INT32_MAX;
                    ep[t] = (int)q.w;
                    avail[t] = in && (int)q.z == head;
                    taken[t] = false;
                }
                for (int step = 0; step < r; ++step) {
                    uint64_t bk = ~0ull;
                    int64_t bi = INT64_MAX;
                    int bslot = -1;
#pragma unroll
                    for (int t = 0; t < kDpPerLane; ++t) {
                        if (avail[t] && !taken[t] && (ek[t] < bk || (ek[t] == bk && ev[t] < bi))) {
                            bk = ek[t];
                            bi = ev[t];
                            bslot = lane + t * kWave;
                        }
                    }
                    uint64_t wk;
                    int64_t wi;
                    wave_argmin(bk, bi, wk, wi); // smallest ~key, lowest index on ties
                    const int pick = (int)wi;
#pragma unroll
                    for (int t = 0; t < kDpPerLane; ++t) {
                        if (ev[t] == pick)
                            taken[t] = true;
                    }
                    // the picked node's slot, from the lane that holds it
                    const unsigned long long own = __builtin_amdgcn_ballot_w64(bslot >= 0 && bi == wi);
                    const int holder = __builtin_ctzll(own);
                    const int pslot = __builtin_amdgcn_readlane(bslot, holder);
#pragma unroll
                    for (int t = 0; t < kDpPerLane; ++t) {
                        if (ep[t] == pslot && lane + t * kWave < cs)
                            avail[t] = true;
                    }
                }
#pragma unroll
                for (int t = 0; t < kDpPerLane; ++t) {
                    if (taken[t])
                        s.OWN[ev[t]] = 2;
                }
            }
        }
    } else {
        for (int i = tid; i < m; i += kDpThreads) {
            if (s.OWN[i] == 1)
                s.OWN[i] = 2;
        }
    }
    __syncthreads();

    // ---- output: first, last and the kept nodes in index order
    int base = 0, par = 0;
    for (int i0 = 0; i0 < m; i0 += kDpThreads) {
        const int i = i0 + tid;
        const bool keep = i < m && (i == 0 || i == m - 1 || s.OWN[i] == 2);
        const unsigned long long mask = __builtin_amdgcn_ballot_w64(keep);
        if (lane == 0)
            s_wc[par][wave] = (uint32_t)__popcll(mask);
        __syncthreads();
        int off = base, total = 0;
        for (int w = 0; w < kDpWaves; ++w) {
            const int c = (int)s_wc[par][w];
            off += w < wave ? c : 0;
            total += c;
        }
        if (keep) {
            const unsigned long long below = lane ? (mask & ((1ull << lane) - 1ull)) : 0ull;
            a.out[off + __popcll(below)] = a.Pmap[i];
        }
        base += total;
        par ^= 1;
    }
    if (tid == 0)
        *gate = 0;
}

template <bool kLds>
__global__ __launch_bounds__(64) void k_simplify_dp(SimplifyArgs a)
{
    extern __shared__ __align__(16) unsigned char lds[];
    if (*dp_gate(a) == 0)
        return; // the split tree gave the result
    const int lane = threadIdx.x;
    const int64_t m = *a.m_ptr;
    SimplifyState s = carve_state(state_base<kLds>(a, lds), a.cap, m);
    if (!simplify_begin(a, s, m, lane))
        return;
    // A[p] = farthest point of the segment starting at kept point p (-1: none
    // or p not a segment start), N[p] = next kept point (-1: p not kept)
    for (int64_t i = lane; i < m; i += kWave) {
        s.A[i] = -1;
        s.N[i] = -1;
    }
    __syncthreads();
    if (lane == 0)
        s.N[0] = (int32_t)(m - 1);
    __syncthreads();
    dp_scan(s, 0, m - 1, lane);
    auto lk = [&](int64_t i) -> uint64_t { return s.A[i] >= 0 ? ~f64_okey(s.F[i]) : ~0ull; };
    tree_build(s.t, lk, lane);
    for (int64_t kept = 2; kept < a.n_out; ++kept) {
        uint64_t key;
        const int64_t p = tree_root(s.t, lk, lane, key);
        if (p < 0 || p >= m - 1 || s.A[p] < 0)
            break; // no segment with an interior point (not reachable while kept < n_out < m)
        const int64_t j = s.A[p], q = s.N[p];
        __syncthreads();
        if (lane == 0) {
            s.N[p] = (int32_t)j;
            s.N[j] = (int32_t)q;
        }
        __syncthreads();
        dp_scan(s, p, j, lane);
        dp_scan(s, j, q, lane);
        tree_fix(s.t, p, lk, lane);
        if ((j >> 6) != (p >> 6))
            tree_fix(s.t, j, lk, lane);
    }
    simplify_emit(a, m, [&](int64_t i) { return i == m - 1 || s.N[i] >= 0; }, lane);
}

// ------------------------------------------------------------------ LLB

// Buckets of at most kLlbPair points take one lane per (point of the bucket,
// point of the previous bucket): lane 8 jj + q.
constexpr int kLlbPair = 8;

// One DPP step of the per-point best over its 8 lanes: the larger length,
// the lower previous-bucket position on ties.
template <int CTRL>
__device__ inline void llb_best_step(double &t, int &q)
{
    const double ot = dpp_f64<CTRL>(t);
    const int oq = dpp_i32<CTRL>(q);
    if (ot > t || (ot == t && oq < q)) {
        t = ot;
        q = oq;
    }
}

template <bool kLds>
__global__ __launch_bounds__(64) void k_simplify_llb(SimplifyArgs a)
{
    extern __shared__ __align__(16) unsigned char lds[];
    const int lane = threadIdx.x;
    const int64_t m = *a.m_ptr;
    SimplifyState s = carve_state(state_base<kLds>(a, lds), a.cap, m);
    if (!simplify_begin(a, s, m, lane))
        return;
    // F = longest total length ending at the point, A = its predecessor
    const int64_t B = a.n_out - 2;
    const Split bk = make_split(m - 2, B);
    if (lane == 0)
        s.F[0] = 0.0;
    __syncthreads();
    int64_t p0 = 0, p1 = 1;
    if (a.cap_bucket <= kLlbPair) {
        // every candidate length of a bucket at once: lane (jj, q) takes
        // point jj of this bucket after point q of the previous one; group q
        // of the previous step holds that point's longest length
        const int jj = lane >> 3, q = lane & (kLlbPair - 1);
        double pf = 0.0; // this group's point's longest length (the first point's: 0)
        SplitWalker w;
        w.init(bk, 0);
        for (int64_t k = 0; k <= B; ++k) {
            const int64_t s0 = k < B ? 1 + w.lo : m - 1;
            const int64_t s1 = k < B ? 1 + w.next_lo(bk) : m;
            if (k < B)
                w.advance(bk);
            const int np = (int)(p1 - p0), nc = (int)(s1 - s0);
            const bool on = jj < nc && q < np;
            const int64_t j = s0 + (jj < nc ? jj : 0), i = p0 + (q < np ? q : 0);
            const double xj = s.X[j], yj = s.Y[j], xi = s.X[i], yi = s.Y[i];
            const double fi = __shfl(pf, kLlbPair * q);
            const double dx = xj - xi, dy = yj - yi;
            const double t = fi + sqrt(dx * dx + dy * dy);
            // the loop below keeps t > best from best = -1, bi = 0: a NaN or a
            // length not above -1 never wins, and (-1, 0) stays when none does
            const bool win = on && t > -1.0;
            double bt = win ? t : -1.0;
            int bq = win ? q : 0;
            llb_best_step<0xB1>(bt, bq);  // lanes q ^ 1
            llb_best_step<0x4E>(bt, bq);  // lanes q ^ 2
            llb_best_step<0x141>(bt, bq); // lanes 7 - q: the other quad of the group
            if (q == 0 && jj < nc)
                s.A[s0 + jj] = (int32_t)(p0 + bq);
            pf = bt;
            p0 = s0;
            p1 = s1;
        }
        __syncthreads();
    } else if (a.cap_bucket <= kWave) {
        // every bucket fits the wave: lane l holds point l of the previous
        // bucket (x, y, longest length) in registers and reads the others'
        // through readlane
        double px = s.X[0], py = s.Y[0], pf = 0.0;
        SplitWalker w;
        w.init(bk, 0);
        for (int64_t k = 0; k <= B; ++k) {
            const int64_t s0 = k < B ? 1 + w.lo : m - 1;
            const int64_t s1 = k < B ? 1 + w.next_lo(bk) : m;
            if (k < B)
                w.advance(bk);
            const int64_t j = s0 + lane;
            const bool mine = j < s1;
            const double xj = mine ? s.X[j] : 0.0, yj = mine ? s.Y[j] : 0.0;
            double best = -1.0;
            int32_t bi = 0;
            const int np = (int)(p1 - p0);
            for (int q = 0; q < np; ++q) {
                const double xi = readlane_f64(px, q), yi = readlane_f64(py, q), fi = readlane_f64(pf, q);
                const double dx = xj - xi, dy = yj - yi;
                const double t = fi + sqrt(dx * dx + dy * dy);
                if (t > best) { // lowest index on ties
                    best = t;
                    bi = q;
                }
            }
            if (mine)
                s.A[j] = (int32_t)(p0 + bi);
            px = xj;
            py = yj;
            pf = best;
            p0 = s0;
            p1 = s1;
        }
        __syncthreads();
    } else {
    SplitWalker w;
    w.init(bk, 0);
    for (int64_t k = 0; k <= B; ++k) {
        const int64_t s0 = k < B ? 1 + w.lo : m - 1;
        const int64_t s1 = k < B ? 1 + w.next_lo(bk) : m;
        if (k < B)
            w.advance(bk);
        for (int64_t j = s0 + lane; j < s1; j += kWave) {
            double best = -1.0;
            int64_t bi = p0;
            for (int64_t i = p0; i < p1; ++i) {
                const double dx = s.X[j] - s.X[i], dy = s.Y[j] - s.Y[i];
                const double t = s.F[i] + sqrt(dx * dx + dy * dy);
                if (t > best) { // lowest index on ties
                    best = t;
                    bi = i;
                }
            }
            s.F[j] = best;
            s.A[j] = (int32_t)bi;
        }
        __syncthreads();
        p0 = s0;
        p1 = s1;
    }
    }
    if (lane == 0) {
        int64_t j = m - 1;
        for (int64_t k = a.n_out - 1; k >= 0; --k) {
            a.out[k] = a.Pmap[j];
            j = k > 0 ? s.A[j] : 0;
        }
    }
}

// ------------------------------------------------------------------ launch

int64_t simplify_scratch_bytes(int64_t cap) { return dp_gate_offset(cap) + 16; }
int64_t simplify_state_lds_bytes(int64_t cap) { return simplify_state_bytes(cap); }
int64_t simplify_tree_lds_bytes(int64_t cap) { return dp_state_bytes(cap); }
int64_t simplify_tree_static_lds() { return (int64_t)(sizeof(DpShared) + 255) / 256 * 256; }

hipError_t launch_simplify(int alg, const SimplifyArgs &a, hipStream_t s)
{
    const size_t lds = a.in_lds ? (size_t)simplify_state_bytes(a.cap) : 0;
    if (alg == 2) { // the split tree, then the greedy loop, which runs only when the tree's gate is set
        if (a.tree_in_lds)
            hipLaunchKernelGGL(k_simplify_dp_tree<true>, dim3(1), dim3(kDpThreads), (size_t)dp_state_bytes(a.cap), s, a);
        else
            hipLaunchKernelGGL(k_simplify_dp_tree<false>, dim3(1), dim3(kDpThreads), 0, s, a);
    }
    switch (alg * 2 + (a.in_lds ? 1 : 0)) {
    case 2:
        hipLaunchKernelGGL(k_simplify_vw<false>, dim3(1), dim3(kWave), 0, s, a);
        break;
    case 3:
        hipLaunchKernelGGL(k_simplify_vw<true>, dim3(1), dim3(kWave), lds, s, a);
        break;
    case 4:
        hipLaunchKernelGGL(k_simplify_dp<false>, dim3(1), dim3(kWave), 0, s, a);
        break;
    case 5:
        hipLaunchKernelGGL(k_simplify_dp<true>, dim3(1), dim3(kWave), lds, s, a);
        break;
    case 6:
        hipLaunchKernelGGL(k_simplify_llb<false>, dim3(1), dim3(kWave), 0, s, a);
        break;
    default:
        hipLaunchKernelGGL(k_simplify_llb<true>, dim3(1), dim3(kWave), lds, s, a);
        break;
    }
    return hipGetLastError();
}

hipError_t simplify_allow_lds(size_t state_bytes, size_t tree_bytes)
{
    // each kernel's limit is its own dynamic LDS: the limit plus the kernel's
    // static LDS must stay within the workgroup's
    hipError_t e = hipSuccess;
    if (state_bytes > 0) {
        for (auto f : {reinterpret_cast<const void *>(k_simplify_vw<true>),
                       reinterpret_cast<const void *>(k_simplify_dp<true>),
                       reinterpret_cast<const void *>(k_simplify_llb<true>)}) {
            hipError_t r = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)state_bytes);
            e = (e == hipSuccess) ? r : e;
        }
    }
    if (tree_bytes > 0) {
        hipError_t r = hipFuncSetAttribute(reinterpret_cast<const void *>(k_simplify_dp_tree<true>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)tree_bytes);
        e = (e == hipSuccess) ? r : e;
    }
    return e;
}

} // namespace mmlttb
