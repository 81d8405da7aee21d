// Thresholded-mean common mode (Common Mode section, Fig. c), computed ahead
// of the frame kernels.  For each region (a bank: one row of B pixels of a
// tile; or a whole tile) and stage s:
//   noise pixels: v < t_cm;  N0 = their number;  S = their sum;
//   CM_s = S / max(N0, guard),  guard = sqrt(region size) in binary32;
//   v <- v - CM_s  (the next stage segments the corrected values).
// S is the exact sum of the noise values rounded once to binary32 (ties to
// even), so no order of summation enters: each lane adds its values into
// binary64 limbs exactly, and the lanes' limbs are put together in a
// multiword integer (pdc_exact.h).
// The frame kernels then subtract CM_1, CM_2, CM_3 in turn (zeros for unused
// stages: x - 0 = x bit for bit).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pdc_device.h"
#include "pdc_exact.h"
#include "pdc_internal.h"

#pragma clang fp contract(off)

namespace pdc {

namespace {

constexpr int kCmThreads = 256;

__device__ __forceinline__ uint32_t sum64(uint32_t n)
{
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) n += (uint32_t)__shfl_xor((int)n, d, 64);
    return n;
}

// One wave per (bank-row, group of F consecutive frames); lane j holds columns
// j + 64 k, k < KV, of the bank-row in each of the F frames.  The bank-row's
// dark and 1/gain are loaded once for the F frames.
template <int KV, int F>
__global__ __launch_bounds__(kCmThreads) void cm_bank_kernel(CmArgs a)
{
    const int lane = threadIdx.x & 63;
    const uint64_t nreg = (uint64_t)a.T * a.H * a.nb;
    const uint64_t nfg = (a.n_frames + F - 1) / F;
    const uint64_t total = nfg * nreg;
    const uint64_t npix = (uint64_t)a.T * a.H * a.W;
    const uint64_t nwaves = ((uint64_t)gridDim.x * kCmThreads) >> 6;
    for (uint64_t w = ((uint64_t)blockIdx.x * kCmThreads + threadIdx.x) >> 6; w < total; w += nwaves) {
        const uint64_t fg = w / nreg;
        const uint32_t reg = (uint32_t)(w - fg * nreg);
        const uint32_t rowi = reg / (uint32_t)a.nb;  // t * H + r
        const uint32_t bank = reg - rowi * (uint32_t)a.nb;
        const uint32_t p0 = rowi * (uint32_t)a.W + bank * (uint32_t)a.B;
        const uint64_t f0 = fg * F;
        const int nf = (int)(a.n_frames - f0 < (uint64_t)F ? a.n_frames - f0 : (uint64_t)F);
        float pd[KV], kk[KV];
        bool ok[KV];
#pragma unroll
        for (int k = 0; k < KV; ++k) {
            const int c = lane + 64 * k;
            ok[k] = c < a.B;
            pd[k] = ok[k] ? a.ped[p0 + c] : 0.0f;
            kk[k] = ok[k] ? a.k[p0 + c] : 0.0f;
        }
        float x[F][KV];
#pragma unroll
        for (int j = 0; j < F; ++j) {
            const uint16_t *fr = a.frames + (f0 + j) * npix + p0;
#pragma unroll
            for (int k = 0; k < KV; ++k) {
                x[j][k] = __builtin_inff();  // absent column or frame: never noise
                if (j < nf && ok[k]) {
                    const uint32_t w = fr[lane + 64 * k];
                    bool bad;
                    x[j][k] = a.gain_mode ? dark_gain_ranged(w, a.gain_mode, pd[k], kk[k], a.ped, a.k, npix,
                                                             p0 + lane + 64 * k, bad)
                                          : dark_gain(w, pd[k], kk[k]);
                }
            }
        }
        float cs[F][3];
        SumWindow win[F];
#pragma unroll
        for (int j = 0; j < F; ++j) {
            cs[j][0] = cs[j][1] = cs[j][2] = 0.0f;
            win[j] = {a.sum_lo, a.sum_hi};
        }
#pragma unroll
        for (int s = 0; s < 3; ++s) {
            if (s >= a.stages) break;
#pragma unroll
            for (int j = 0; j < F; ++j) {
                int n0;
                bool fits;
                const float sum = region_sum<64, KV>(x[j], a.t_cm, (uint32_t)a.B, win[j], n0, fits);
                const uint32_t n = sum64((uint32_t)n0);
                const float c = __fdiv_rn(sum, fmaxf((float)n, a.guard));
                cs[j][s] = c;
                win[j] = next_window(win[j], c);
#pragma unroll
                for (int k = 0; k < KV; ++k) x[j][k] = __fsub_rn(x[j][k], c);
            }
        }
        if (lane < F && lane < nf) {
            float c0 = 0.0f, c1 = 0.0f, c2 = 0.0f;
#pragma unroll
            for (int j = 0; j < F; ++j)
                if (j == lane) {
                    c0 = cs[j][0];
                    c1 = cs[j][1];
                    c2 = cs[j][2];
                }
            float *o = a.cm + ((f0 + lane) * nreg + reg) * 3;
            o[0] = c0;
            o[1] = c1;
            o[2] = c2;
        }
    }
}

// Window of stage s of a tile item (F frames from f0, nf of them): the union
// of the frames' windows.  Returns false when the two-limb way cannot hold
// it with K-bit limbs.
template <int F>
__device__ __forceinline__ bool tile_window(const CmArgs &a, int s, uint64_t f0, uint32_t t, int nf, int K,
                                            float (&c0)[F], float (&c1)[F], int &lo)
{
    int l = a.sum_lo, h = a.sum_hi;
#pragma unroll
    for (int j = 0; j < F; ++j) {
        const float *cv = a.cm + ((f0 + j) * a.T + t) * 3;
        c0[j] = (s > 0 && j < nf) ? cv[0] : 0.0f;
        c1[j] = (s > 1 && j < nf) ? cv[1] : 0.0f;
        SumWindow w = next_window(next_window({a.sum_lo, a.sum_hi}, c0[j]), c1[j]);
        l = w.lo < l ? w.lo : l;
        h = w.hi > h ? w.hi : h;
    }
    lo = l;
    return h - l <= 2 * K;
}

// One pixel of a tile at stage s: Frames1 less the earlier stages' values.
__device__ __forceinline__ float tile_value(const CmArgs &a, int s, uint32_t w, float pp, float kp, uint64_t p,
                                            uint64_t npix, float c0, float c1)
{
    bool bad;
    // an invalid pixel is +inf: never below t_cm, and stays +inf
    float y = a.gain_mode ? dark_gain_ranged(w, a.gain_mode, pp, kp, a.ped, a.k, npix, p, bad) : dark_gain(w, pp, kp);
    if (s > 0) y = __fsub_rn(y, c0);
    if (s > 1) y = __fsub_rn(y, c1);
    return y;
}

// General-way sum of stage s over one tile and frame f (values beyond the
// two-limb window): the lanes of the workgroup (or wave, with nt = 64) add
// pixels tid, tid + nt, ... in eight 28-bit limbs of unit 2^-149.
__device__ __forceinline__ Wide<4> tile_sum_general(const CmArgs &a, int s, uint64_t f, uint32_t t, float c0, float c1,
                                                    uint32_t tid, uint32_t nt, uint32_t &n0)
{
    constexpr int NL = kGenNL25, KG = kGenK25;
    const uint32_t HW = (uint32_t)a.H * (uint32_t)a.W;
    const uint64_t npix = (uint64_t)a.T * HW;
    double pw[NL], ipw[NL], q[NL];
#pragma unroll
    for (int i = 0; i < NL; ++i) {
        pw[i] = __builtin_ldexp(1.0, KG * i);
        ipw[i] = __builtin_ldexp(1.0, -KG * i);
        q[i] = 0.0;
    }
    const double sc = __builtin_ldexp(1.0, 149);
    const uint16_t *fr = a.frames + f * npix + (uint64_t)t * HW;
    const uint64_t pbase = (uint64_t)t * HW;
    n0 = 0;
    for (uint32_t p = tid; p < HW; p += nt) {
        const float y = tile_value(a, s, fr[p], a.ped[pbase + p], a.k[pbase + p], pbase + p, npix, c0, c1);
        const bool nz = y < a.t_cm;
        n0 += nz;
        limbs_add<NL>(q, nz ? y : 0.0f, sc, pw, ipw);
    }
    return wide_from_limbs<4>(q, KG);
}

// Stage s of the tile regions: one workgroup per (tile, group of F frames);
// thread j adds pixels j + 256 k of the tile in each frame; dark and 1/gain
// are read once per F frames.
template <int F>
__global__ __launch_bounds__(kCmThreads) void cm_tile_kernel(CmArgs a, int s)
{
    __shared__ Wide<4> s_part[kCmThreads / 64][F];
    __shared__ uint32_t s_cnt[kCmThreads / 64][F];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint64_t nfg = (a.n_frames + F - 1) / F;
    const uint64_t items = nfg * (uint64_t)a.T;
    const uint32_t HW = (uint32_t)a.H * (uint32_t)a.W;
    const uint64_t npix = (uint64_t)a.T * HW;
    const int K = 53 - clog2((HW + kCmThreads - 1) / kCmThreads);  // values one thread adds per frame
    for (uint64_t it = blockIdx.x; it < items; it += gridDim.x) {
        const uint64_t fg = it / (uint64_t)a.T;
        const uint32_t t = (uint32_t)(it - fg * (uint64_t)a.T);
        const uint64_t f0 = fg * F;
        const int nf = (int)(a.n_frames - f0 < (uint64_t)F ? a.n_frames - f0 : (uint64_t)F);
        float c0[F], c1[F];
        int lo;
        const bool fast = tile_window<F>(a, s, f0, t, nf, K, c0, c1, lo);
        Wide<4> S[F];
        uint32_t n0[F];
        if (fast) {
            const double sc = __builtin_ldexp(1.0, -lo), sk = __builtin_ldexp(1.0, -lo - K),
                         pk = __builtin_ldexp(1.0, K);
            double q0[F], q1[F];
#pragma unroll
            for (int j = 0; j < F; ++j) {
                q0[j] = q1[j] = 0.0;
                n0[j] = 0;
            }
            const uint16_t *fr = a.frames + f0 * npix + (uint64_t)t * HW;
            const float *pd = a.ped + (uint64_t)t * HW;
            const float *kk = a.k + (uint64_t)t * HW;
#pragma unroll 2
            for (uint32_t p = threadIdx.x; p < HW; p += kCmThreads) {
                const float pp = pd[p], kp = kk[p];
#pragma unroll
                for (int j = 0; j < F; ++j) {
                    if (j >= nf) break;
                    const float y = tile_value(a, s, fr[j * npix + p], pp, kp, (uint64_t)t * HW + p, npix, c0[j], c1[j]);
                    const bool nz = y < a.t_cm;
                    n0[j] += nz;
                    limbs2_add(q0[j], q1[j], nz ? y : 0.0f, sc, sk, pk);
                }
            }
#pragma unroll
            for (int j = 0; j < F; ++j) {
                const double q[2] = {q0[j], q1[j]};
                S[j] = wide_from_limbs<4>(q, K);
            }
        } else {
            lo = -149;
#pragma unroll
            for (int j = 0; j < F; ++j) {
                n0[j] = 0;
                S[j] = Wide<4>{{0, 0, 0, 0}};
                if (j < nf) S[j] = tile_sum_general(a, s, f0 + j, t, c0[j], c1[j], threadIdx.x, kCmThreads, n0[j]);
            }
        }
#pragma unroll
        for (int j = 0; j < F; ++j) {
            wave_sum_wide(S[j]);
            const uint32_t ns = sum64(n0[j]);
            if (lane == 0) {
                s_part[wave][j] = S[j];
                s_cnt[wave][j] = ns;
            }
        }
        __syncthreads();
        if (threadIdx.x < nf) {
            const int j = threadIdx.x;
            Wide<4> sum = s_part[0][j];
            uint32_t n = s_cnt[0][j];
#pragma unroll
            for (int w = 1; w < kCmThreads / 64; ++w) {
                wide_add(sum, s_part[w][j]);
                n += s_cnt[w][j];
            }
            float *cv = a.cm + ((f0 + j) * a.T + t) * 3;
            cv[s] = __fdiv_rn(wide_round(sum, lo), fmaxf((float)n, a.guard));
            if (s == 0) {
                cv[1] = 0.0f;
                cv[2] = 0.0f;
            }
        }
        __syncthreads();
    }
}

// Stage s of the tile regions when every tile and frame starts on a 4-pixel
// boundary (single gain range): one wave per (tile, group of F frames); lane
// l adds pixels 256 k + 4 l + i, which it reads as one 8-byte group of raw
// words and one 16-byte group of dark and 1/gain values per k.
template <int F>
__global__ __launch_bounds__(kCmThreads) void cm_tile_wide_kernel(CmArgs a, int s)
{
    const int lane = threadIdx.x & 63;
    const uint64_t nfg = (a.n_frames + F - 1) / F;
    const uint64_t items = nfg * (uint64_t)a.T;
    const uint32_t HW = (uint32_t)a.H * (uint32_t)a.W;
    const uint64_t npix = (uint64_t)a.T * HW;
    const uint64_t nwaves = ((uint64_t)gridDim.x * kCmThreads) >> 6;
    const int K = 53 - clog2(4u * ((HW + 255u) / 256u));  // values one lane adds per frame
    for (uint64_t it = ((uint64_t)blockIdx.x * kCmThreads + threadIdx.x) >> 6; it < items; it += nwaves) {
        const uint64_t fg = it / (uint64_t)a.T;
        const uint32_t t = (uint32_t)(it - fg * (uint64_t)a.T);
        const uint64_t f0 = fg * F;
        const int nf = (int)(a.n_frames - f0 < (uint64_t)F ? a.n_frames - f0 : (uint64_t)F);
        float c0[F], c1[F];
        int lo;
        const bool fast = tile_window<F>(a, s, f0, t, nf, K, c0, c1, lo);
        if (fast) {
            const double sc = __builtin_ldexp(1.0, -lo), sk = __builtin_ldexp(1.0, -lo - K),
                         pk = __builtin_ldexp(1.0, K);
            double q0[F], q1[F];
            uint32_t n0[F];
#pragma unroll
            for (int j = 0; j < F; ++j) {
                q0[j] = q1[j] = 0.0;
                n0[j] = 0;
            }
            const uint16_t *fr = a.frames + f0 * npix + (uint64_t)t * HW;
            const float *pd = a.ped + (uint64_t)t * HW;
            const float *kk = a.k + (uint64_t)t * HW;
            for (uint32_t p = 4u * (uint32_t)lane; p < HW; p += 256u) {  // HW is a multiple of 4
                const float4 pp = *reinterpret_cast<const float4 *>(pd + p);
                const float4 kp = *reinterpret_cast<const float4 *>(kk + p);
                const float pv[4] = {pp.x, pp.y, pp.z, pp.w}, kv[4] = {kp.x, kp.y, kp.z, kp.w};
#pragma unroll
                for (int j = 0; j < F; ++j) {
                    if (j >= nf) break;
                    const uint2 w = *reinterpret_cast<const uint2 *>(fr + (uint64_t)j * npix + p);
                    const uint32_t r[4] = {w.x & 0xFFFFu, w.x >> 16, w.y & 0xFFFFu, w.y >> 16};
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        float y = dark_gain(r[i], pv[i], kv[i]);
                        if (s > 0) y = __fsub_rn(y, c0[j]);
                        if (s > 1) y = __fsub_rn(y, c1[j]);
                        const bool nz = y < a.t_cm;
                        n0[j] += nz;
                        limbs2_add(q0[j], q1[j], nz ? y : 0.0f, sc, sk, pk);
                    }
                }
            }
#pragma unroll
            for (int j = 0; j < F; ++j) {
                const double q[2] = {q0[j], q1[j]};
                Wide<2> S = wide_from_limbs<2>(q, K);
                wave_sum_wide(S);
                const uint32_t n = sum64(n0[j]);
                if (lane == 0 && j < nf) {
                    float *cv = a.cm + ((f0 + j) * a.T + t) * 3;
                    cv[s] = __fdiv_rn(wide_round(S, lo), fmaxf((float)n, a.guard));
                    if (s == 0) {
                        cv[1] = 0.0f;
                        cv[2] = 0.0f;
                    }
                }
            }
        } else {
            for (int j = 0; j < nf; ++j) {
                uint32_t n0;
                Wide<4> S = tile_sum_general(a, s, f0 + j, t, c0[j], c1[j], (uint32_t)lane, 64u, n0);
                wave_sum_wide(S);
                const uint32_t n = sum64(n0);
                if (lane == 0) {
                    float *cv = a.cm + ((f0 + j) * a.T + t) * 3;
                    cv[s] = __fdiv_rn(wide_round(S, -149), fmaxf((float)n, a.guard));
                    if (s == 0) {
                        cv[1] = 0.0f;
                        cv[2] = 0.0f;
                    }
                }
            }
        }
    }
}

uint32_t cm_grid(uint64_t items, uint64_t per_block, uint32_t n_cu)
{
    const uint64_t want = (items + per_block - 1) / per_block;
    const uint64_t cap = 64ull * n_cu;
    return (uint32_t)(want < 1 ? 1 : (want > cap ? cap : want));
}

}  // namespace

template <int KV, int F>
static void launch_bank_t(const CmArgs &a, uint32_t n_cu, hipStream_t s)
{
    const uint64_t total = (a.n_frames + F - 1) / F * (uint64_t)a.T * a.H * a.nb;
    const uint32_t grid = cm_grid(total, kCmThreads / 64, n_cu);
    hipLaunchKernelGGL((cm_bank_kernel<KV, F>), dim3(grid), dim3(kCmThreads), 0, s, a);
}

// Frames per wave: as many as keep F * KV values per lane at 32.
hipError_t launch_cm_bank(const CmArgs &a, uint32_t n_cu, hipStream_t s)
{
    if (a.n_frames == 0 || (uint64_t)a.T * a.H * a.nb == 0) return hipSuccess;
    const int kv = (a.B + 63) / 64;
    if (kv <= 1) launch_bank_t<1, 16>(a, n_cu, s);
    else if (kv <= 2) launch_bank_t<2, 16>(a, n_cu, s);
    else if (kv <= 4) launch_bank_t<4, 8>(a, n_cu, s);
    else if (kv <= 8) launch_bank_t<8, 4>(a, n_cu, s);
    else if (kv <= 16) launch_bank_t<16, 2>(a, n_cu, s);
    else return hipErrorInvalidValue;  // bank_cols <= 1024
    return hipGetLastError();
}

hipError_t launch_cm_tile(const CmArgs &a, uint32_t n_cu, hipStream_t s)
{
    constexpr int F = 8;
    const uint64_t items = (a.n_frames + F - 1) / F * (uint64_t)a.T;
    if (items == 0) return hipSuccess;
    // wide loads need every tile and frame on a 4-pixel (8-byte) boundary
    const uint64_t hw = (uint64_t)a.H * a.W;
    const bool wide = a.gain_mode == 0 && hw % 4 == 0 && ((uintptr_t)a.frames & 7u) == 0 &&
                      ((uintptr_t)a.ped & 15u) == 0 && ((uintptr_t)a.k & 15u) == 0;
    if (wide) {
        const uint32_t grid = cm_grid(items, kCmThreads / 64, n_cu);
        for (int st = 0; st < a.stages; ++st)
            hipLaunchKernelGGL(cm_tile_wide_kernel<F>, dim3(grid), dim3(kCmThreads), 0, s, a, st);
    } else {
        const uint32_t grid = cm_grid(items, 1, n_cu);
        for (int st = 0; st < a.stages; ++st)
            hipLaunchKernelGGL(cm_tile_kernel<F>, dim3(grid), dim3(kCmThreads), 0, s, a, st);
    }
    return hipGetLastError();
}

}  // namespace pdc
