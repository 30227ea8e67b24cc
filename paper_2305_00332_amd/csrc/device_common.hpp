// Device helpers shared by the libmmlttb kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mmlttb {

constexpr int kWave = 64;

// Native 16-byte vector (usable with the nontemporal load builtin).
typedef float f32x4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// Equal-index partitions. Part k of `len` items cut into `parts` parts starts
// at floor(k * len / parts). With len = q * parts + r this is
// k * q + floor(k * r / parts); k * r < parts^2 <= 2^62 for parts < 2^31,
// so no 128-bit product or division is needed.
// ---------------------------------------------------------------------------
struct Split {
    int64_t len, parts, q, r;
};

__host__ __device__ inline Split make_split(int64_t len, int64_t parts)
{
    Split s;
    s.len = len;
    s.parts = parts;
    s.q = len / parts;
    s.r = len % parts;
    return s;
}

__host__ __device__ inline int64_t split_lo(const Split &s, int64_t k) { return k * s.q + (k * s.r) / s.parts; }

// Walks part starts in order without a division per step.
struct SplitWalker {
    int64_t lo;  // start of the current part
    int64_t rem; // (k * r) mod parts
    __device__ void init(const Split &s, int64_t k)
    {
        lo = split_lo(s, k);
        rem = (k * s.r) % s.parts;
    }
    // start of the next part
    __device__ int64_t next_lo(const Split &s) const
    {
        int64_t r2 = rem + s.r;
        return lo + s.q + (r2 >= s.parts ? 1 : 0);
    }
    __device__ void advance(const Split &s)
    {
        int64_t r2 = rem + s.r;
        int carry = r2 >= s.parts ? 1 : 0;
        lo += s.q + carry;
        rem = carry ? r2 - s.parts : r2;
    }
};

// ---------------------------------------------------------------------------
// float32 order key: unsigned integers ordered like the numbers, with -0.0
// and +0.0 mapped to one key (they compare equal as numbers).
// ---------------------------------------------------------------------------
__device__ inline uint32_t f32_order_key(float v)
{
    uint32_t u = __float_as_uint(v);
    u = (u == 0x80000000u) ? 0u : u;
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// ---------------------------------------------------------------------------
// Cross-lane moves. DPP controls (gfx9): quad_perm [1,0,3,2] = 0xB1,
// quad_perm [2,3,0,1] = 0x4E, row_half_mirror = 0x141, row_mirror = 0x140.
// After the four steps every lane of a 16-lane row holds the row's result.
// ---------------------------------------------------------------------------
template <int CTRL>
__device__ inline int dpp_i32(int v)
{
    return __builtin_amdgcn_update_dpp(v, v, CTRL, 0xF, 0xF, false);
}

template <int CTRL>
__device__ inline float dpp_f32(float v)
{
    return __int_as_float(dpp_i32<CTRL>(__float_as_int(v)));
}

template <int CTRL>
__device__ inline double dpp_f64(double v)
{
    int lo = __double2loint(v), hi = __double2hiint(v);
    return __hiloint2double(dpp_i32<CTRL>(hi), dpp_i32<CTRL>(lo));
}

// Packed-key min / max over a power-of-two group of tpb <= 64 lanes (aligned
// groups; every lane of the wave takes part). The DPP steps pair lanes within
// quads, half-rows and rows; shuffles by 16 and 32 lanes cross rows.
template <int CTRL>
__device__ inline unsigned long long dpp_u64(unsigned long long v)
{
    const int lo = dpp_i32<CTRL>((int)(uint32_t)v);
    const int hi = dpp_i32<CTRL>((int)(uint32_t)(v >> 32));
    return ((unsigned long long)(uint32_t)hi << 32) | (uint32_t)lo;
}

template <int CTRL>
__device__ inline void group_step(unsigned long long &kmin, unsigned long long &kmax)
{
    const unsigned long long a = dpp_u64<CTRL>(kmin), c = dpp_u64<CTRL>(kmax);
    kmin = a < kmin ? a : kmin;
    kmax = c > kmax ? c : kmax;
}

__device__ inline void group_minmax(int tpb, unsigned long long &kmin, unsigned long long &kmax)
{
    if (tpb >= 2)
        group_step<0xB1>(kmin, kmax);
    if (tpb >= 4)
        group_step<0x4E>(kmin, kmax);
    if (tpb >= 8)
        group_step<0x141>(kmin, kmax);
    if (tpb >= 16)
        group_step<0x140>(kmin, kmax);
    for (int off = 16; off < tpb; off <<= 1) {
        const unsigned long long a = __shfl_xor(kmin, off), c = __shfl_xor(kmax, off);
        kmin = a < kmin ? a : kmin;
        kmax = c > kmax ? c : kmax;
    }
}

__device__ inline unsigned long long readlane_u64(unsigned long long v, int lane)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, lane);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), lane);
    return ((unsigned long long)hi << 32) | lo;
}

// Packed-key min and max over the full wave (every lane active); the result
// is uniform across the wave.
__device__ inline void wave_minmax_u64(unsigned long long &kmin, unsigned long long &kmax)
{
    group_minmax(16, kmin, kmax); // every lane holds its row's result
    unsigned long long a = readlane_u64(kmin, 0), c = readlane_u64(kmax, 0);
#pragma unroll
    for (int row = 16; row < 64; row += 16) {
        const unsigned long long ra = readlane_u64(kmin, row), rc = readlane_u64(kmax, row);
        a = ra < a ? ra : a;
        c = rc > c ? rc : c;
    }
    kmin = a;
    kmax = c;
}

__device__ inline float readlane_f32(float v, int lane)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

__device__ inline double readlane_f64(double v, int lane)
{
    int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}

__device__ inline int64_t readlane_i64(int64_t v, int lane)
{
    uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, lane);
    uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)v >> 32), lane);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Min / max over the full wave; every lane must be active.
__device__ inline float wave_min_f32(float v)
{
    v = fminf(v, dpp_f32<0xB1>(v));
    v = fminf(v, dpp_f32<0x4E>(v));
    v = fminf(v, dpp_f32<0x141>(v));
    v = fminf(v, dpp_f32<0x140>(v));
    float a = fminf(readlane_f32(v, 0), readlane_f32(v, 16));
    float b = fminf(readlane_f32(v, 32), readlane_f32(v, 48));
    return fminf(a, b);
}

__device__ inline float wave_max_f32(float v)
{
    v = fmaxf(v, dpp_f32<0xB1>(v));
    v = fmaxf(v, dpp_f32<0x4E>(v));
    v = fmaxf(v, dpp_f32<0x141>(v));
    v = fmaxf(v, dpp_f32<0x140>(v));
    float a = fmaxf(readlane_f32(v, 0), readlane_f32(v, 16));
    float b = fmaxf(readlane_f32(v, 32), readlane_f32(v, 48));
    return fmaxf(a, b);
}

__device__ inline double dmax_sel(double a, double b) { return b > a ? b : a; }

__device__ inline double wave_max_f64(double v)
{
    v = dmax_sel(v, dpp_f64<0xB1>(v));
    v = dmax_sel(v, dpp_f64<0x4E>(v));
    v = dmax_sel(v, dpp_f64<0x141>(v));
    v = dmax_sel(v, dpp_f64<0x140>(v));
    double a = dmax_sel(readlane_f64(v, 0), readlane_f64(v, 16));
    double b = dmax_sel(readlane_f64(v, 32), readlane_f64(v, 48));
    return dmax_sel(a, b);
}

__device__ inline int64_t wave_min_i64(int64_t v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        int64_t o = __shfl_xor(v, off);
        v = o < v ? o : v;
    }
    return v;
}

__device__ inline int64_t wave_sum_i64(int64_t v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1)
        v += __shfl_xor(v, off);
    return v;
}

// ---------------------------------------------------------------------------
// Correct rounding of a non-negative multi-word integer to binary64.
// value = sum_i w[i] * 2^(32 i) * 2^scale_exp, rounded to nearest, ties to
// even. The top 64 significant bits are taken with every lower bit folded
// into bit 0 (a sticky bit below the rounding position), then converted by
// the hardware u64 -> f64 conversion (exact halves and one rounded add) and
// scaled exactly by ldexp. Callers keep the result in the normal range.
// Word indices are compile-time constants (no scratch memory).
// ---------------------------------------------------------------------------
template <int N>
__device__ inline double round_words_to_f64(const uint32_t (&w)[N], int scale_exp, bool negative)
{
    int t = -1;
#pragma unroll
    for (int i = 0; i < N; ++i)
        t = (w[i] != 0u) ? i : t;
    if (t < 0)
        return 0.0;
    uint32_t hi = 0u, mid = 0u, lo = 0u;
    bool sticky = false;
#pragma unroll
    for (int i = 0; i < N; ++i) {
        hi = (i == t) ? w[i] : hi;
        mid = (i == t - 1) ? w[i] : mid;
        lo = (i == t - 2) ? w[i] : lo;
        sticky = sticky || ((i < t - 2) && (w[i] != 0u));
    }
    int lz = __clz((int)hi);
    uint64_t H = ((uint64_t)hi << 32) | mid;
    uint64_t T = lz ? ((H << lz) | (uint64_t)(lo >> (32 - lz))) : H;
    uint32_t rest = lz ? (lo << lz) : lo;
    sticky = sticky || (rest != 0u);
    double d = (double)(T | (sticky ? 1ull : 0ull));
    double r = ldexp(d, 32 * (t - 2) + 32 - lz + scale_exp);
    return negative ? -r : r;
}

// Exact sum of int64 values (128-bit accumulation), rounded once.
struct I64ExactSum {
    __int128 s;
    __device__ void clear() { s = 0; }
    __device__ void add(int64_t v) { s += (__int128)v; }
    __device__ void merge(const I64ExactSum &o) { s += o.s; }
    __device__ double round() const
    {
        bool neg = s < 0;
        unsigned __int128 m = neg ? (unsigned __int128)(-s) : (unsigned __int128)s;
        uint32_t w[4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
            w[i] = (uint32_t)(m >> (32 * i));
        return round_words_to_f64<4>(w, 0, neg);
    }
};

// Exact sum of finite float32 values, rounded once to binary64.
// A finite float32 is mant * 2^(s - 149), mant < 2^24, s = max(E, 1) - 1 in
// [0, 253] (E: biased exponent). Limb k (k = s >> 5) gathers mant << (s & 31)
// < 2^55 with its sign, so 255 terms fit in an int64 limb; normalize()
// carries limbs 0..7 into [0, 2^32) and leaves the signed rest in limb 8.
struct F32ExactSum {
    int64_t limb[9];
    int pending;

    __device__ void clear()
    {
#pragma unroll
        for (int i = 0; i < 9; ++i)
            limb[i] = 0;
        pending = 0;
    }

    __device__ void normalize()
    {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            int64_t c = limb[i] >> 32; // floor division by 2^32
            limb[i] -= (int64_t)((uint64_t)c << 32);
            limb[i + 1] += c;
        }
        pending = 0;
    }

    __device__ void add(float v)
    {
        uint32_t u = __float_as_uint(v);
        uint32_t e = (u >> 23) & 0xffu;
        uint32_t mant = e ? ((u & 0x7fffffu) | 0x800000u) : (u & 0x7fffffu);
        uint32_t s = e ? e - 1u : 0u;
        uint32_t k = s >> 5;
        int64_t term = (int64_t)((uint64_t)mant << (s & 31u));
        term = (u >> 31) ? -term : term;
#pragma unroll
        for (int i = 0; i < 8; ++i)
            limb[i] += (k == (uint32_t)i) ? term : 0;
        if (++pending == 255)
            normalize();
    }

    // Adds a binary64 value that is an exact sum of float32 values (so a
    // multiple of 2^-149 below 2^129 in magnitude): its 53-bit significand,
    // placed at its bit position, spans at most three limbs.
    __device__ void add_exact_f64(double d)
    {
        if (d == 0.0)
            return;
        const uint64_t u = (uint64_t)__double_as_longlong(d);
        const int be = (int)((u >> 52) & 0x7ffu);
        uint64_t m = (u & 0xfffffffffffffull) | (be ? (1ull << 52) : 0ull);
        int shift = (be ? be : 1) - 1075 + 149; // bit position of m's lowest bit above 2^-149
        if (shift < 0) { // the bits below 2^-149 are zero (d is a multiple of it)
            m >>= -shift;
            shift = 0;
        }
        const int k = shift >> 5, r = shift & 31;
        const unsigned __int128 w = (unsigned __int128)m << r;
        const int64_t t[3] = {(int64_t)(uint64_t)(w & 0xffffffffu), (int64_t)(uint64_t)((w >> 32) & 0xffffffffu),
                              (int64_t)(uint64_t)(w >> 64)};
        const bool neg = (u >> 63) != 0;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const int64_t v = neg ? -t[j] : t[j];
#pragma unroll
            for (int i = 0; i < 8; ++i)
                limb[i] += (k + j == i) ? v : 0;
            limb[8] += (k + j == 8) ? v : ((k + j == 9) ? (int64_t)((uint64_t)v << 32) : 0);
        }
        if (++pending == 255)
            normalize();
    }

    // Merge a normalized accumulator into a normalized one.
    __device__ void merge_normalized(const F32ExactSum &o)
    {
#pragma unroll
        for (int i = 0; i < 9; ++i)
            limb[i] += o.limb[i];
        normalize();
    }

    __device__ double round()
    {
        normalize();
        bool neg = limb[8] < 0;
        uint32_t w[10];
        int64_t top;
        if (neg) {
            int64_t carry = 0;
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                int64_t t = -limb[i] + carry;
                w[i] = (uint32_t)(t & 0xffffffffll);
                carry = t >> 32;
            }
            top = -limb[8] + carry;
        } else {
#pragma unroll
            for (int i = 0; i < 8; ++i)
                w[i] = (uint32_t)limb[i];
            top = limb[8];
        }
        w[8] = (uint32_t)((uint64_t)top);
        w[9] = (uint32_t)((uint64_t)top >> 32);
        return round_words_to_f64<10>(w, -149, neg);
    }
};

// Doubled LTTB triangle area in binary64, one rounding per operation in this
// order, no contraction (the library is built with -ffp-contract=off):
// |(Xa - MX) * (Yj - Ya) - (Xa - Xj) * (MY - Ya)|.
__device__ inline double lttb_area2(double xa, double ya, double xj, double yj, double mx, double my)
{
    return fabs((xa - mx) * (yj - ya) - (xa - xj) * (my - ya));
}

} // namespace mmlttb
