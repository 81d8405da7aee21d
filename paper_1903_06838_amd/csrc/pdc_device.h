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
