// Device pieces of the path for other value types: float64 and int32 y,
// float64 x (float32 y takes it only together with float64 x).
//
// The stream compares values as numbers and hands each work item's extremes
// on as order keys (unsigned integers ordered like the numbers, -0.0 and +0.0
// on one key). 64-bit keys leave no room for an index next to them, so the
// MinMax stream writes one (key, index) partial per work item and a second
// kernel merges each bin's partials.
#pragma once

#include "device_common.hpp"

namespace mmlttb {

typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef int i32x4 __attribute__((ext_vector_type(4)));

template <class T>
struct ValueTraits;

template <>
struct ValueTraits<float> {
    using Key = uint32_t;
    using Vec = f32x4;
    static constexpr int kLanes = 4; // values per 16-byte load
    __device__ static Key key(float v) { return f32_order_key(v); }
    __device__ static float at(const Vec &v, int i) { return i == 0 ? v.x : i == 1 ? v.y : i == 2 ? v.z : v.w; }
    __device__ static double widen(float v) { return (double)v; }
    __device__ static float lo_id() { return __int_as_float(0x7f800000); }   // +inf
    __device__ static float hi_id() { return -__int_as_float(0x7f800000); }  // -inf
    __device__ static float vmin(float a, float b) { return fminf(a, b); }
    __device__ static float vmax(float a, float b) { return fmaxf(a, b); }
};

template <>
struct ValueTraits<int32_t> {
    using Key = uint32_t;
    using Vec = i32x4;
    static constexpr int kLanes = 4;
    __device__ static Key key(int32_t v) { return (uint32_t)v ^ 0x80000000u; }
    __device__ static int32_t at(const Vec &v, int i) { return i == 0 ? v.x : i == 1 ? v.y : i == 2 ? v.z : v.w; }
    __device__ static double widen(int32_t v) { return (double)v; }
    __device__ static int32_t lo_id() { return INT32_MAX; }
    __device__ static int32_t hi_id() { return INT32_MIN; }
    __device__ static int32_t vmin(int32_t a, int32_t b) { return a < b ? a : b; }
    __device__ static int32_t vmax(int32_t a, int32_t b) { return a > b ? a : b; }
};

template <>
struct ValueTraits<double> {
    using Key = uint64_t;
    using Vec = f64x2;
    static constexpr int kLanes = 2;
    __device__ static Key key(double v)
    {
        uint64_t u = (uint64_t)__double_as_longlong(v);
        u = (u == 0x8000000000000000ull) ? 0ull : u;
        return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
    }
    __device__ static double at(const Vec &v, int i) { return i == 0 ? v.x : v.y; }
    __device__ static double widen(double v) { return v; }
    __device__ static double lo_id() { return __longlong_as_double(0x7ff0000000000000ll); }  // +inf
    __device__ static double hi_id() { return -__longlong_as_double(0x7ff0000000000000ll); } // -inf
    __device__ static double vmin(double a, double b) { return fmin(a, b); }
    __device__ static double vmax(double a, double b) { return fmax(a, b); }
};

template <class K>
__device__ inline K wave_min_key(K v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        K o = __shfl_xor(v, off);
        v = o < v ? o : v;
    }
    return v;
}

template <class K>
__device__ inline K wave_max_key(K v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        K o = __shfl_xor(v, off);
        v = o > v ? o : v;
    }
    return v;
}

// Reduce y[lo, hi) (hi > lo) with one full wave: the order keys of the
// smallest and largest values and the lowest index holding each (uniform
// across the wave). Same scheme as the float32 stream: values are compared
// as numbers (finite inputs; -0.0 == +0.0), 16-byte nontemporal loads in
// batches of U per lane, the batch where each lane first reached its extreme,
// a wave reduction, then a re-read of only the winning batch.
template <class T, int U>
__device__ inline void wave_reduce_keys(const T *__restrict__ y, int64_t lo, int64_t hi, int lane,
                                        typename ValueTraits<T>::Key &o_kmin, int64_t &o_imin,
                                        typename ValueTraits<T>::Key &o_kmax, int64_t &o_imax)
{
    using Tr = ValueTraits<T>;
    using V = typename Tr::Vec;
    constexpr int W = Tr::kLanes;
    // head: values before the first 16-byte boundary; tail: after the last
    // full vector; fewer than W each, handled by lanes 0.. and 8..
    const uint64_t addr = (uint64_t)(uintptr_t)(y + lo);
    int64_t head = (int64_t)(((16u - (unsigned)(addr & 15u)) & 15u) / sizeof(T));
    head = head < hi - lo ? head : hi - lo;
    const int64_t body = lo + head;
    const int64_t nvec = (hi - body) / W;
    const int64_t body_end = body + nvec * W;
    const V *__restrict__ vv = reinterpret_cast<const V *>(y + body);

    T smin = Tr::lo_id(), smax = Tr::hi_id();
    int64_t sidx = INT64_MAX;
    if (lane < head) {
        sidx = lo + lane;
    } else if (lane >= 8 && lane < 8 + (hi - body_end)) {
        sidx = body_end + (lane - 8);
    }
    if (sidx != INT64_MAX)
        smin = smax = y[sidx];

    constexpr int64_t kPerBatch = (int64_t)kWave * U; // vectors per batch
    const int64_t nfull = nvec / kPerBatch;
    T mn = Tr::lo_id(), mx = Tr::hi_id();
    int64_t bmn = -1, bmx = -1;
    for (int64_t t = 0; t < nfull; ++t) {
        V d[U];
        const V *p = vv + t * kPerBatch + lane;
#pragma unroll
        for (int u = 0; u < U; ++u)
            d[u] = __builtin_nontemporal_load(p + u * kWave);
        T a = Tr::at(d[0], 0), b = a;
#pragma unroll
        for (int u = 0; u < U; ++u) {
#pragma unroll
            for (int i = (u == 0 ? 1 : 0); i < W; ++i) {
                a = Tr::vmin(a, Tr::at(d[u], i));
                b = Tr::vmax(b, Tr::at(d[u], i));
            }
        }
        if (a < mn) {
            mn = a;
            bmn = t;
        }
        if (b > mx) {
            mx = b;
            bmx = t;
        }
    }
    if (nfull * kPerBatch < nvec) { // last, partial batch
        const int64_t t = nfull;
        T a = Tr::lo_id(), b = Tr::hi_id();
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t q = t * kPerBatch + u * kWave + lane;
            if (q < nvec) {
                const V d = vv[q];
#pragma unroll
                for (int i = 0; i < W; ++i) {
                    a = Tr::vmin(a, Tr::at(d, i));
                    b = Tr::vmax(b, Tr::at(d, i));
                }
            }
        }
        if (a < mn) {
            mn = a;
            bmn = t;
        }
        if (b > mx) {
            mx = b;
            bmx = t;
        }
    }
    T wmin = Tr::vmin(mn, smin), wmax = Tr::vmax(mx, smax);
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        wmin = Tr::vmin(wmin, __shfl_xor(wmin, off));
        wmax = Tr::vmax(wmax, __shfl_xor(wmax, off));
    }

    // lowest index holding each extreme: the lane's scalar value, and the
    // first match inside the lane's winning batch
    int64_t cmin = (sidx != INT64_MAX && smin == wmin) ? sidx : INT64_MAX;
    int64_t cmax = (sidx != INT64_MAX && smax == wmax) ? sidx : INT64_MAX;
    if (bmn >= 0 && mn == wmin) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t q = bmn * kPerBatch + u * kWave + lane;
            if (q < nvec) {
                const V d = vv[q];
#pragma unroll
                for (int i = W - 1; i >= 0; --i)
                    if (Tr::at(d, i) == wmin)
                        cmin = (body + W * q + i) < cmin ? body + W * q + i : cmin;
            }
        }
    }
    if (bmx >= 0 && mx == wmax) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t q = bmx * kPerBatch + u * kWave + lane;
            if (q < nvec) {
                const V d = vv[q];
#pragma unroll
                for (int i = W - 1; i >= 0; --i)
                    if (Tr::at(d, i) == wmax)
                        cmax = (body + W * q + i) < cmax ? body + W * q + i : cmax;
            }
        }
    }
    o_kmin = Tr::key(wmin);
    o_kmax = Tr::key(wmax);
    o_imin = wave_min_i64(cmin);
    o_imax = wave_min_i64(cmax);
}

// Exact sum of finite binary64 values, rounded once to binary64.
// A finite binary64 is mant * 2^(s - 1074) with mant < 2^53 and
// s = max(E, 1) - 1 in [0, 2045]; mant << (s & 31) spans three 32-bit words
// starting at word s >> 5, each added with its sign to an int64 limb (so
// 2^31 terms fit before a carry pass). Rounding: the top 64 bits with a
// sticky bit, converted once; a sum below 2^53 units of 2^-1074 converts
// exactly (every subnormal result), a larger one is normal or overflows to
// an infinity as round-to-nearest does. The kLimbs limbs live in storage the
// caller provides (a row of LDS), since they are indexed by exponent.
struct F64ExactSum {
    static constexpr int kLimbs = 68; // 2176 bits >= 2098 + 64
    int64_t *limb;
    int64_t pending;

    __device__ explicit F64ExactSum(int64_t *storage) : limb(storage), pending(0) {}

    __device__ void clear()
    {
        for (int i = 0; i < kLimbs; ++i)
            limb[i] = 0;
        pending = 0;
    }

    __device__ void normalize()
    {
        for (int i = 0; i < kLimbs - 1; ++i) {
            const int64_t c = limb[i] >> 32; // floor division by 2^32
            limb[i] -= (int64_t)((uint64_t)c << 32);
            limb[i + 1] += c;
        }
        pending = 0;
    }

    __device__ void add(double v)
    {
        const uint64_t u = (uint64_t)__double_as_longlong(v);
        const uint32_t e = (uint32_t)((u >> 52) & 0x7ffu);
        const uint64_t mant = e ? ((u & 0xfffffffffffffull) | (1ull << 52)) : (u & 0xfffffffffffffull);
        const uint32_t s = e ? e - 1u : 0u;
        const int k = (int)(s >> 5);
        const unsigned __int128 w = (unsigned __int128)mant << (s & 31u); // < 2^85
        const int64_t w0 = (int64_t)(uint32_t)w, w1 = (int64_t)(uint32_t)(w >> 32), w2 = (int64_t)(uint32_t)(w >> 64);
        if (u >> 63) {
            limb[k] -= w0;
            limb[k + 1] -= w1;
            limb[k + 2] -= w2;
        } else {
            limb[k] += w0;
            limb[k + 1] += w1;
            limb[k + 2] += w2;
        }
        if (++pending == ((int64_t)1 << 30))
            normalize();
    }

    __device__ double round()
    {
        normalize();
        const bool neg = limb[kLimbs - 1] < 0;
        uint32_t w[kLimbs + 1];
        int64_t carry = 0;
#pragma unroll
        for (int i = 0; i < kLimbs - 1; ++i) {
            const int64_t t = (neg ? -limb[i] : limb[i]) + carry;
            w[i] = (uint32_t)(t & 0xffffffffll);
            carry = t >> 32;
        }
        const int64_t top = (neg ? -limb[kLimbs - 1] : limb[kLimbs - 1]) + carry;
        w[kLimbs - 1] = (uint32_t)(uint64_t)top;
        w[kLimbs] = (uint32_t)((uint64_t)top >> 32);
        return round_words_to_f64<kLimbs + 1>(w, -1074, neg);
    }
};

} // namespace mmlttb
