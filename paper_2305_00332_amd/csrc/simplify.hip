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

template <bool kLds>
__global__ __launch_bounds__(64) void k_simplify_dp(SimplifyArgs a)
{
    extern __shared__ __align__(16) unsigned char lds[];
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
    if (a.cap_bucket <= kWave) {
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

int64_t simplify_scratch_bytes(int64_t cap) { return simplify_state_bytes(cap); }

hipError_t launch_simplify(int alg, const SimplifyArgs &a, hipStream_t s)
{
    const size_t lds = a.in_lds ? (size_t)simplify_state_bytes(a.cap) : 0;
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

hipError_t simplify_allow_lds(size_t bytes)
{
    hipError_t e = hipSuccess;
    for (auto f : {reinterpret_cast<const void *>(k_simplify_vw<true>), reinterpret_cast<const void *>(k_simplify_dp<true>),
                   reinterpret_cast<const void *>(k_simplify_llb<true>)}) {
        hipError_t r = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
        e = (e == hipSuccess) ? r : e;
    }
    return e;
}

} // namespace mmlttb
