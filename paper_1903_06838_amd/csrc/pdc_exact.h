// Exact sums of binary32 values for the thresholded-mean common mode (Common
// Mode section, Fig. c): a region's sum is the exact sum of its noise pixels
// rounded once to binary32, ties to even, so that it depends on no order of
// summation.
//
// Window.  Every value a stage sums is an integer multiple of 2^lo and below
// 2^hi in magnitude.  For the first stage both come from the calibration
// (Frames1 = fl(fl(adc - dark) * k) is a multiple of 2^(min(0, lsb(dark)) +
// lsb(k)), because a rounding to binary32 keeps a multiple of a power of two
// that is not below 2^-149 a multiple of it; |Frames1| is at most its value at
// adc = 0 or 16383).  A later stage sums fl(v - c): a multiple of
// 2^min(lo, lsb(c)), at most 2^(max(hi, hi(c)) + 1) in magnitude.
//
// Limbs.  A value x becomes the integer t = x 2^-u (u <= lo), split into limbs
// of K bits: t = sum_i q_i 2^(K i), each q_i = trunc of the remaining part over
// 2^(K i), |q_i| < 2^K, every step exact in binary64 (the parts keep at most
// 24 significant bits).  Limb i of a lane (or of a group of lanes) adds its
// q_i: with at most 2^(53 - K) values per accumulator every partial sum is an
// integer below 2^53, so the binary64 additions are exact in any order.  The
// limb totals are then put together in a multiword integer and rounded once.
//
// Two ways are taken.  The fast one uses two limbs and u = lo: exact when
// hi - lo <= 2 K.  The general one uses u = -149 (every binary32 is a multiple
// of 2^-149) and NL limbs with NL K >= hi + 149; with the calibration ranges
// the library accepts (|dark| <= 2^24, k <= 2^24) hi <= 49 in the first stage
// and every stage adds at most 3 (|c| <= the largest |value| of its stage),
// so hi + 149 <= 204.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pdc {

// Lowest set bit of a nonzero finite binary32: c is an odd multiple of 2^lsb.
__host__ __device__ __forceinline__ int f32_lsb(float c)
{
    const uint32_t b = __builtin_bit_cast(uint32_t, c);
    const int E = (int)((b >> 23) & 0xFFu);
    const uint32_t M = E ? ((b & 0x7FFFFFu) | 0x800000u) : (b & 0x7FFFFFu);
    return (E ? E : 1) - 150 + __builtin_ctz(M);
}

// Smallest h with |c| < 2^h for finite c (zero gives -149).
__host__ __device__ __forceinline__ int f32_hi(float c)
{
    const uint32_t b = __builtin_bit_cast(uint32_t, c) & 0x7FFFFFFFu;
    if (!b) return -149;
    const int E = (int)(b >> 23);
    return E ? E - 126 : -149 + (32 - __builtin_clz(b));
}

struct SumWindow {
    int lo, hi;  // every value is a multiple of 2^lo and below 2^hi in magnitude
};

// The window of the values fl(v - c) of the next stage.
__host__ __device__ __forceinline__ SumWindow next_window(SumWindow w, float c)
{
    if (c == 0.0f) return w;  // v - 0 = v
    const int l = f32_lsb(c), h = f32_hi(c);
    return {w.lo < l ? w.lo : l, (w.hi > h ? w.hi : h) + 2};
}

// ceil(log2(n)) for n >= 1.
__host__ __device__ __forceinline__ int clog2(uint32_t n)
{
    return n <= 1 ? 0 : 32 - __builtin_clz(n - 1);
}

// Limbs of a general-way accumulator: K = 43 holds up to 2^10 values per
// accumulator (a bank of up to 1024 pixels), 5 limbs cover 215 >= 204 bits;
// K = 28 holds up to 2^25 values (one lane's share of a tile of up to 2^31
// pixels), 8 limbs cover 224 bits.
constexpr int kGenK10 = 43, kGenNL10 = 5;
constexpr int kGenK25 = 28, kGenNL25 = 8;

// Adds value x (an integer multiple of 2^u) to the limbs q[0..NL) of K bits;
// s = 2^-u, pw[i] = 2^(K i), ipw[i] = 2^-(K i).
template <int NL>
__host__ __device__ __forceinline__ void limbs_add(double (&q)[NL], float x, double s, const double (&pw)[NL],
                                          const double (&ipw)[NL])
{
    double t = (double)x * s;
#pragma unroll
    for (int i = NL - 1; i > 0; --i) {
        const double d = __builtin_trunc(t * ipw[i]);
        t = __builtin_fma(-d, pw[i], t);
        q[i] += d;
    }
    q[0] += t;
}

// The two-limb case of limbs_add with sk = 2^(-u-K) and p = 2^K.
__host__ __device__ __forceinline__ void limbs2_add(double &q0, double &q1, float x, double s, double sk, double p)
{
    const double xd = (double)x;
    const double d = __builtin_trunc(xd * sk);
    q1 += d;
    q0 += __builtin_fma(-d, p, xd * s);
}

// Multiword two's complement integer, least significant word first.
template <int NW>
struct Wide {
    uint64_t w[NW];
};

template <int NW>
__host__ __device__ __forceinline__ void wide_add(Wide<NW> &a, const Wide<NW> &b)
{
    uint64_t c = 0;
#pragma unroll
    for (int i = 0; i < NW; ++i) {
        const uint64_t s = a.w[i] + b.w[i];
        const uint64_t r = s + c;
        c = (uint64_t)(s < a.w[i]) | (uint64_t)(r < s);
        a.w[i] = r;
    }
}

// v 2^sh for 0 <= sh < 64 NW (bits above the top word are dropped).
template <int NW>
__host__ __device__ __forceinline__ Wide<NW> wide_from(int64_t v, int sh)
{
    const uint64_t ext = (uint64_t)(v >> 63);
    const int ws = sh >> 6, bs = sh & 63;
    Wide<NW> r;
#pragma unroll
    for (int i = 0; i < NW; ++i) {
        const uint64_t cur = i == ws ? (uint64_t)v : (i > ws ? ext : 0ull);
        const uint64_t prev = i - 1 == ws ? (uint64_t)v : (i - 1 > ws ? ext : 0ull);
        r.w[i] = bs ? (cur << bs) | (prev >> (64 - bs)) : cur;
    }
    return r;
}

// An integer-valued binary64 with |d| <= 2^53 as int64.
__host__ __device__ __forceinline__ int64_t d2i(double d)
{
    return (int64_t)d;
}

// The limb totals q[i] (weights 2^(K i)) as one integer.
template <int NW, int NL>
__host__ __device__ __forceinline__ Wide<NW> wide_from_limbs(const double (&q)[NL], int K)
{
    Wide<NW> s = wide_from<NW>(d2i(q[0]), 0);
#pragma unroll
    for (int i = 1; i < NL; ++i) wide_add(s, wide_from<NW>(d2i(q[i]), K * i));
    return s;
}

// 64 bits of a nonnegative s starting at bit b (0 <= b < 64 NW).
template <int NW>
__host__ __device__ __forceinline__ uint64_t wide_bits(const Wide<NW> &s, int b)
{
    const int ws = b >> 6, bs = b & 63;
    uint64_t lo = 0, hi = 0;
#pragma unroll
    for (int i = 0; i < NW; ++i) {
        lo = i == ws ? s.w[i] : lo;
        hi = i == ws + 1 ? s.w[i] : hi;
    }
    return bs ? (lo >> bs) | (hi << (64 - bs)) : lo;
}

// Whether any of the bits [0, b) of s is set (0 <= b).
template <int NW>
__host__ __device__ __forceinline__ bool wide_any_below(const Wide<NW> &s, int b)
{
    uint64_t acc = 0;
#pragma unroll
    for (int i = 0; i < NW; ++i) {
        const int n = b - 64 * i;  // bits of word i below b
        const uint64_t m = n >= 64 ? ~0ull : (n <= 0 ? 0ull : ((1ull << n) - 1));
        acc |= s.w[i] & m;
    }
    return acc != 0;
}

// s 2^u rounded to the nearest binary32, ties to even (u >= -149; the result
// is finite for the sums that occur: below 2^(204 + 31)).  Zero gives +0.
template <int NW>
__host__ __device__ __forceinline__ float wide_round(Wide<NW> s, int u)
{
    const bool neg = (int64_t)s.w[NW - 1] < 0;
    if (neg) {
        uint64_t c = 1;
#pragma unroll
        for (int i = 0; i < NW; ++i) {
            const uint64_t x = ~s.w[i] + c;
            c = (c && x == 0) ? 1 : 0;
            s.w[i] = x;
        }
    }
    int top = -1;
#pragma unroll
    for (int i = 0; i < NW; ++i)
        if (s.w[i]) top = 64 * i + 63 - __builtin_clzll(s.w[i]);
    if (top < 0) return 0.0f;
    float r;
    if (top < 24) {
        // s < 2^24 with u >= -149: s 2^u is a binary32 (normal or subnormal)
        r = __builtin_ldexpf((float)(uint32_t)s.w[0], u);
    } else {
        const int sh = top - 23;  // the result is normal: u + top >= -125
        const uint64_t win = wide_bits(s, sh - 1);
        uint32_t q = (uint32_t)(win >> 1) & 0xFFFFFFu;
        const bool half = win & 1u;
        if (half && ((q & 1u) || wide_any_below(s, sh - 1))) ++q;  // q may reach 2^24: still exact
        r = __builtin_ldexpf((float)q, u + sh);
    }
    return neg ? -r : r;
}

// Sum of x over aligned groups of L lanes (L a power of two <= 64); exact for
// the integer-valued limb totals.
template <int CTRL>
__device__ __forceinline__ double dpp_d(double x)
{
    const uint64_t b = (uint64_t)__double_as_longlong(x);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, CTRL, 0xF, 0xF, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

template <int L>
__device__ __forceinline__ double gsum_d(double x)
{
    x += dpp_d<0xB1>(x);                // quad_perm [1,0,3,2]
    if (L >= 4) x += dpp_d<0x4E>(x);    // quad_perm [2,3,0,1]
    if (L >= 8) x += dpp_d<0x141>(x);   // row_half_mirror
    if (L >= 16) x += dpp_d<0x140>(x);  // row_mirror
    if (L >= 32) x += __shfl_xor(x, 16, 64);
    if (L >= 64) x += __shfl_xor(x, 32, 64);
    return x;
}

template <int NW>
__device__ __forceinline__ void wave_sum_wide(Wide<NW> &s)
{
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        Wide<NW> o;
#pragma unroll
        for (int i = 0; i < NW; ++i)
            o.w[i] = (uint64_t)__shfl_xor((unsigned long long)s.w[i], d, 64);
        wide_add(s, o);
    }
}

// Exact sum, rounded once, of the values of x below t (the others add
// nothing) of a region held by a group of L lanes, NV values per lane, at most
// n values in all (n <= 1024), within window w; cnt receives the lane's number
// of values below t.  Every lane of the group returns the sum.  The general
// way forms one limb at a time, q_i = trunc(t 2^-(K i)) - 2^K trunc(t
// 2^-(K (i + 1))), which keeps one accumulator live.  Without GENERAL a window
// too wide for two limbs returns 0 with fits = false (the caller has the
// region summed elsewhere).
template <int L, int NV, bool GENERAL = true>
__device__ __forceinline__ float region_sum(const float (&x)[NV], float t, uint32_t n, SumWindow w, int &cnt,
                                            bool &fits)
{
    const int K = 53 - clog2(n);
    int c = 0;
#pragma unroll
    for (int v = 0; v < NV; ++v) c += x[v] < t;
    cnt = c;
    fits = w.hi - w.lo <= 2 * K;
    if (!GENERAL && !fits) return 0.0f;
    if (fits) {
        const double s = __builtin_ldexp(1.0, -w.lo), sk = __builtin_ldexp(1.0, -w.lo - K),
                     p = __builtin_ldexp(1.0, K);
        double q0 = 0.0, q1 = 0.0;
#pragma unroll
        for (int v = 0; v < NV; ++v) limbs2_add(q0, q1, x[v] < t ? x[v] : 0.0f, s, sk, p);
        const double q[2] = {gsum_d<L>(q0), gsum_d<L>(q1)};
        return wide_round(wide_from_limbs<2>(q, K), w.lo);
    }
    constexpr int NL = kGenNL10;
    constexpr int KG = kGenK10;
    const double p = __builtin_ldexp(1.0, KG);
    double q[NL];
#pragma unroll 1
    for (int i = 0; i < NL; ++i) {
        const double sa = __builtin_ldexp(1.0, 149 - KG * i), sb = __builtin_ldexp(1.0, 149 - KG * (i + 1));
        double acc = 0.0;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const double xd = (double)(x[v] < t ? x[v] : 0.0f);
            const double a = __builtin_trunc(xd * sa), b = __builtin_trunc(xd * sb);
            acc += __builtin_fma(-b, p, a);
        }
        q[i] = gsum_d<L>(acc);
    }
    return wide_round(wide_from_limbs<4>(q, KG), -149);
}

}  // namespace pdc
