// Thresholded-mean common mode (Common Mode section, Fig. c), computed ahead
// of the frame kernels.  For each region (a bank: one row of B pixels of a
// tile; or a whole tile) and stage s:
//   noise pixels: v < t_cm;  N0 = their number;  S = their sum;
//   CM_s = S / max(N0, guard),  guard = sqrt(region size) in binary32;
//   v <- v - CM_s  (the next stage segments the corrected values).
// S is a binary32 sum in a fixed order: pixel i of the region (raster order)
// is added to partial sum i mod P (P = 64 for a bank, 256 for a tile) in
// increasing i from +0.0, then the partials are added in a balanced binary
// tree.  A lane owns one partial; a butterfly over lanes xor 1, 2, 4, ...
// forms the tree exactly, since each pair adds the same two values.
// The frame kernels then subtract CM_1, CM_2, CM_3 in turn (zeros for unused
// stages: x - 0 = x bit for bit).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pdc_device.h"
#include "pdc_internal.h"

#pragma clang fp contract(off)

namespace pdc {

namespace {

constexpr int kCmThreads = 256;

__device__ __forceinline__ float tree64(float p)
{
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) p = __fadd_rn(p, __shfl_xor(p, d, 64));
    return p;
}

__device__ __forceinline__ uint32_t sum64(uint32_t n)
{
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) n += (uint32_t)__shfl_xor((int)n, d, 64);
    return n;
}

// One wave per (frame, bank-row); lane j holds columns j + 64 k, k < KV.
template <int KV>
__global__ __launch_bounds__(kCmThreads) void cm_bank_kernel(CmArgs a)
{
    const int lane = threadIdx.x & 63;
    const uint64_t nreg = (uint64_t)a.T * a.H * a.nb;
    const uint64_t total = a.n_frames * nreg;
    const uint64_t npix = (uint64_t)a.T * a.H * a.W;
    const uint64_t nwaves = ((uint64_t)gridDim.x * kCmThreads) >> 6;
    for (uint64_t w = ((uint64_t)blockIdx.x * kCmThreads + threadIdx.x) >> 6; w < total; w += nwaves) {
        const uint64_t f = w / nreg;
        const uint32_t reg = (uint32_t)(w - f * nreg);
        const uint32_t rowi = reg / (uint32_t)a.nb;  // t * H + r
        const uint32_t bank = reg - rowi * (uint32_t)a.nb;
        const uint32_t p0 = rowi * (uint32_t)a.W + bank * (uint32_t)a.B;
        const uint16_t *fr = a.frames + f * npix + p0;
        float x[KV];
        bool ok[KV];
#pragma unroll
        for (int k = 0; k < KV; ++k) {
            const int c = lane + 64 * k;
            ok[k] = c < a.B;
            x[k] = ok[k] ? dark_gain(fr[c], a.ped[p0 + c], a.k[p0 + c]) : 0.0f;
        }
        float cs[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int s = 0; s < 3; ++s) {
            if (s >= a.stages) break;
            float part = 0.0f;
            uint32_t n0 = 0;
#pragma unroll
            for (int k = 0; k < KV; ++k)
                if (ok[k] && x[k] < a.t_cm) {
                    part = __fadd_rn(part, x[k]);
                    ++n0;
                }
            const float sum = tree64(part);
            const uint32_t n = sum64(n0);
            const float c = __fdiv_rn(sum, fmaxf((float)n, a.guard));
            cs[s] = c;
#pragma unroll
            for (int k = 0; k < KV; ++k) x[k] = __fsub_rn(x[k], c);
        }
        if (lane == 0) {
            float *o = a.cm + w * 3;
            o[0] = cs[0];
            o[1] = cs[1];
            o[2] = cs[2];
        }
    }
}

// Stage s of the tile regions: one workgroup per (frame, tile); thread j owns
// partial j (pixels p = j + 256 k of the tile); waves hold partials 64w..64w+63.
__global__ __launch_bounds__(kCmThreads) void cm_tile_kernel(CmArgs a, int s)
{
    __shared__ float s_part[kCmThreads / 64];
    __shared__ uint32_t s_cnt[kCmThreads / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint64_t items = a.n_frames * (uint64_t)a.T;
    const uint32_t HW = (uint32_t)a.H * (uint32_t)a.W;
    const uint64_t npix = (uint64_t)a.T * HW;
    for (uint64_t it = blockIdx.x; it < items; it += gridDim.x) {
        const uint64_t f = it / (uint64_t)a.T;
        const uint32_t t = (uint32_t)(it - f * (uint64_t)a.T);
        float *cv = a.cm + it * 3;
        const float c0 = s > 0 ? cv[0] : 0.0f;
        const float c1 = s > 1 ? cv[1] : 0.0f;
        const uint16_t *fr = a.frames + f * npix + (uint64_t)t * HW;
        const float *pd = a.ped + (uint64_t)t * HW;
        const float *kk = a.k + (uint64_t)t * HW;
        float part = 0.0f;
        uint32_t n0 = 0;
        for (uint32_t p = threadIdx.x; p < HW; p += kCmThreads) {
            float y = dark_gain(fr[p], pd[p], kk[p]);
            if (s > 0) y = __fsub_rn(y, c0);
            if (s > 1) y = __fsub_rn(y, c1);
            if (y < a.t_cm) {
                part = __fadd_rn(part, y);
                ++n0;
            }
        }
        part = tree64(part);
        n0 = sum64(n0);
        if (lane == 0) {
            s_part[wave] = part;
            s_cnt[wave] = n0;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            const float sum = __fadd_rn(__fadd_rn(s_part[0], s_part[1]), __fadd_rn(s_part[2], s_part[3]));
            const uint32_t n = s_cnt[0] + s_cnt[1] + s_cnt[2] + s_cnt[3];
            cv[s] = __fdiv_rn(sum, fmaxf((float)n, a.guard));
            if (s == 0) {
                cv[1] = 0.0f;
                cv[2] = 0.0f;
            }
        }
        __syncthreads();
    }
}

uint32_t cm_grid(uint64_t items, uint64_t per_block, uint32_t n_cu)
{
    const uint64_t want = (items + per_block - 1) / per_block;
    const uint64_t cap = 16ull * n_cu;
    return (uint32_t)(want < 1 ? 1 : (want > cap ? cap : want));
}

}  // namespace

hipError_t launch_cm_bank(const CmArgs &a, uint32_t n_cu, hipStream_t s)
{
    const uint64_t total = a.n_frames * (uint64_t)a.T * a.H * a.nb;
    if (total == 0) return hipSuccess;
    const uint32_t grid = cm_grid(total, kCmThreads / 64, n_cu);
    const int kv = (a.B + 63) / 64;
    if (kv <= 1) hipLaunchKernelGGL(cm_bank_kernel<1>, dim3(grid), dim3(kCmThreads), 0, s, a);
    else if (kv <= 2) hipLaunchKernelGGL(cm_bank_kernel<2>, dim3(grid), dim3(kCmThreads), 0, s, a);
    else if (kv <= 4) hipLaunchKernelGGL(cm_bank_kernel<4>, dim3(grid), dim3(kCmThreads), 0, s, a);
    else if (kv <= 8) hipLaunchKernelGGL(cm_bank_kernel<8>, dim3(grid), dim3(kCmThreads), 0, s, a);
    else if (kv <= 16) hipLaunchKernelGGL(cm_bank_kernel<16>, dim3(grid), dim3(kCmThreads), 0, s, a);
    else return hipErrorInvalidValue;  // bank_cols <= 1024
    return hipGetLastError();
}

hipError_t launch_cm_tile(const CmArgs &a, uint32_t n_cu, hipStream_t s)
{
    const uint64_t items = a.n_frames * (uint64_t)a.T;
    if (items == 0) return hipSuccess;
    const uint32_t grid = cm_grid(items, 1, n_cu);
    for (int st = 0; st < a.stages; ++st)
        hipLaunchKernelGGL(cm_tile_kernel, dim3(grid), dim3(kCmThreads), 0, s, a, st);
    return hipGetLastError();
}

}  // namespace pdc
