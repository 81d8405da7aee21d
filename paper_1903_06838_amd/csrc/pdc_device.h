// Device helpers shared by the frame kernels.  Every operation is one IEEE
// binary32 operation rounded to nearest even (files including this are built
// with -ffp-contract=off and the pragma below).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#pragma clang fp contract(off)

namespace pdc {

// Photon counting: division by the single-photon signal, rounded to the
// nearest integer, ties to even (Photon Charge Summing section).  The quotient
// is the correctly rounded binary32 division; counts saturate at 2^32 - 1.
__device__ __forceinline__ uint32_t photon_count(float q, float photon_adu)
{
    float x = __fdiv_rn(q, photon_adu);
    if (x >= 4294967296.0f) return 0xFFFFFFFFu;
    return (uint32_t)__builtin_rintf(x);
}

// Frames1 for one pixel (Fig. b): (adc - dark) * (1 / gain), two roundings.
__device__ __forceinline__ float dark_gain(uint32_t raw, float ped, float k)
{
    float a = (float)(raw & 0x3FFFu);
    float t = __fsub_rn(a, ped);
    return __fmul_rn(t, k);
}

// Gain range reported by a raw word's bits 14-15 on an auto-ranging detector
// (Dark and Gain section: one dark and one gain plane per range), or -1 for
// an invalid code.  mode 1 (ePix10k-like): codes 0, 1, 2 -> ranges 0, 1, 2,
// code 3 invalid; mode 2 (Jungfrau-like): codes 0, 1, 3 -> ranges 0, 1, 2,
// code 2 invalid.
__device__ __forceinline__ int gain_range(uint32_t raw, int mode)
{
    const int c = (int)((raw >> 14) & 3u);
    if (mode == 1) return c == 3 ? -1 : c;
    return c == 2 ? -1 : (c == 3 ? 2 : c);
}

// Frames1 of one pixel of an auto-ranging detector: range 0 uses the given
// (resident) plane values, ranges 1 and 2 read their planes at p + r * stride;
// an invalid code gives +inf, which no valid value reaches.
__device__ __forceinline__ float dark_gain_ranged(uint32_t raw, int mode, float ped0, float k0, const float *ped,
                                                  const float *k, uint64_t stride, uint64_t p, bool &invalid)
{
    const int r = gain_range(raw, mode);
    invalid = r < 0;
    if (r == 0) return dark_gain(raw, ped0, k0);
    if (r < 0) return __builtin_inff();
    const uint64_t o = p + (uint64_t)r * stride;
    return dark_gain(raw, ped[o], k[o]);
}

// Order-preserving map of binary32 to int32 (-0 just below +0) and back.
__device__ __forceinline__ int32_t f2key(float x)
{
    int32_t b = __float_as_int(x);
    return b ^ ((b >> 31) & 0x7FFFFFFF);
}
__device__ __forceinline__ float key2f(int32_t k)
{
    return __int_as_float(k ^ ((k >> 31) & 0x7FFFFFFF));
}

}  // namespace pdc
