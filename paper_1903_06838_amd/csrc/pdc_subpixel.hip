// Subpixel position of photon hits (Photon Subpixel Resolution section and
// its figure of centroid versus learned positions): the classical masked 3x3
// centroid with eta linearization, and a small learned estimator (a
// 25-64-64-2 ReLU network on the 5x5 patch of corrected values around a hit)
// trained and evaluated with bfloat16 MFMA (v_mfma_f32_16x16x32_bf16) and
// float32 accumulation.
//
// MFMA 16x16x32 bf16 operand layout (wave64): lane l holds
//   A[l % 16][8 (l / 16) + j]  and  B[8 (l / 16) + j][l % 16],  j = 0..7,
// and receives C[4 (l / 16) + i][l % 16], i = 0..3.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <atomic>

#include "pdc_device.h"
#include "pdc_subpixel.h"

#pragma clang fp contract(off)

namespace pdc {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(2))) __bf16 bf16x2;
typedef __attribute__((ext_vector_type(2))) float f32x2;
typedef __attribute__((ext_vector_type(4))) float f32x4;
typedef __attribute__((ext_vector_type(4))) unsigned int u32x4;
typedef __attribute__((ext_vector_type(8))) short i16x8;

namespace {

// float32 -> bfloat16 bits, round to nearest even (finite inputs).
__device__ __forceinline__ uint16_t f2bf(float f)
{
    uint32_t b = __float_as_uint(f);
    b += 0x7FFFu + ((b >> 16) & 1u);
    return (uint16_t)(b >> 16);
}

// Two float32 -> bfloat16 (a in the low half), round to nearest even: one
// v_cvt_pk_bf16_f32, the same values as f2bf for finite inputs.
__device__ __forceinline__ uint32_t pk_bf16(float a, float b)
{
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2{a, b}, bf16x2));
}

// Operand fragment: 8 bf16 values base[o * SO + (k + j) * SK], j = 0..7.
// With SK == 1 one 16-byte load (o * SO + k is a multiple of 8 at every call).
template <int SO, int SK>
__device__ __forceinline__ bf16x8 frag(const uint16_t *base, int o, int k)
{
    if constexpr (SK == 1) {
        return __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4 *>(base + o * SO + k));
    } else {
        bf16x8 r;
#pragma unroll
        for (int j = 0; j < 8; ++j) r[j] = __builtin_bit_cast(__bf16, base[o * SO + (k + j) * SK]);
        return r;
    }
}

__device__ __forceinline__ f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ f32x4 zero4() { return f32x4{0.f, 0.f, 0.f, 0.f}; }

// Orders this wave's LDS accesses (all lanes) before the ones that follow.
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// The same for a wave whose global loads must stay in flight: waits for its
// LDS accesses only (a workgroup fence would also wait for the loads).
__device__ __forceinline__ void wave_lds_wait() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

}  // namespace

__global__ void fill_zero_kernel(float *p, uint64_t n)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0f;
}

hipError_t launch_fill_zero(float *p, uint64_t n, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(fill_zero_kernel, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// classical estimator
// ---------------------------------------------------------------------------
// Masked 3x3 centroid of a 5x5 patch: pixels not above t_nb count as 0; the
// sums run over rows top to bottom and columns left to right;
// (dy, dx) = (sum s*dr, sum s*dc) / sum s, and (0, 0) when sum s is 0.
__device__ __forceinline__ void centroid3(const float *p, float t_nb, float &cy, float &cx)
{
    float s = 0.0f, sy = 0.0f, sx = 0.0f;
#pragma unroll
    for (int dr = -1; dr <= 1; ++dr)
#pragma unroll
        for (int dc = -1; dc <= 1; ++dc) {
            const float v = p[(2 + dr) * 5 + 2 + dc];
            const float m = v > t_nb ? v : 0.0f;
            s = __fadd_rn(s, m);
            sy = __fadd_rn(sy, __fmul_rn(m, (float)dr));
            sx = __fadd_rn(sx, __fmul_rn(m, (float)dc));
        }
    cy = s > 0.0f ? __fdiv_rn(sy, s) : 0.0f;
    cx = s > 0.0f ? __fdiv_rn(sx, s) : 0.0f;
}

// Position of a centroid coordinate on [-1, 1] in units of bins (nbins bins).
__device__ __forceinline__ float eta_pos(float c, int nbins)
{
    return (fminf(fmaxf(c, -1.0f), 1.0f) + 1.0f) * 0.5f * (float)nbins;
}

// Eta linearization: position = CDF(c) - 1/2, linear between table edges
// (tab holds the CDF at the nbins + 1 bin edges).
__device__ __forceinline__ float eta_map(const float *tab, int nbins, float c)
{
    const float t = eta_pos(c, nbins);
    const int i = min((int)floorf(t), nbins - 1);
    const float f = t - (float)i;
    return tab[i] * (1.0f - f) + tab[i + 1] * f - 0.5f;
}

__global__ void centroid_eta_kernel(const float *patches, uint64_t n, float t_nb, const float *eta, int nbins,
                                    float *out)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float cy, cx;
    centroid3(patches + i * 25, t_nb, cy, cx);
    if (eta) {
        cy = eta_map(eta, nbins, cy);
        cx = eta_map(eta + nbins + 1, nbins, cx);
    }
    out[2 * i] = cy;
    out[2 * i + 1] = cx;
}

hipError_t launch_centroid_eta(const float *patches, uint64_t n, float t_nb, const float *eta, int nbins,
                               float *out, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(centroid_eta_kernel, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, s, patches, n, t_nb,
                       eta, nbins, out);
    return hipGetLastError();
}

__global__ void zero_u32_kernel(uint32_t *p, uint64_t n)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

// Per-axis histogram of centroids over [-1, 1] in nbins bins.
__global__ void eta_hist_kernel(const float *patches, uint64_t n, float t_nb, int nbins, uint32_t *hist)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float c[2];
    centroid3(patches + i * 25, t_nb, c[0], c[1]);
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        const int b = min((int)floorf(eta_pos(c[a], nbins)), nbins - 1);
        atomicAdd(&hist[a * nbins + b], 1u);
    }
}

// Empirical CDF at the bin edges, one thread per axis (nbins is small).
__global__ void eta_cdf_kernel(const uint32_t *hist, int nbins, uint64_t n, float *table)
{
    const int a = blockIdx.x;
    if (threadIdx.x != 0) return;
    const uint32_t *h = hist + (uint64_t)a * nbins;
    float *t = table + (uint64_t)a * (nbins + 1);
    uint64_t acc = 0;
    t[0] = 0.0f;
    for (int b = 0; b < nbins; ++b) {
        acc += h[b];
        t[b + 1] = (float)((double)acc / (double)n);
    }
}

hipError_t launch_eta_table(const float *patches, uint64_t n, float t_nb, int nbins, uint32_t *hist,
                            float *table, hipStream_t s)
{
    const uint64_t nh = 2 * (uint64_t)nbins;
    hipLaunchKernelGGL(zero_u32_kernel, dim3((uint32_t)((nh + 255) / 256)), dim3(256), 0, s, hist, nh);
    if (n)
        hipLaunchKernelGGL(eta_hist_kernel, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, s, patches, n, t_nb,
                           nbins, hist);
    hipLaunchKernelGGL(eta_cdf_kernel, dim3(2), dim3(64), 0, s, hist, nbins, n ? n : (uint64_t)1, table);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// learned estimator
// ---------------------------------------------------------------------------
constexpr int kTile = 32;          // hits per wave tile
constexpr int kWaves = 4;          // waves per workgroup

__global__ void mlp_pack_kernel(const float *theta, uint16_t *pk)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < 64 * 32) {  // w1t[c][k] = W1[k][c]
        const int c = t / 32, k = t % 32;
        pk[kPackW1t + t] = k < 25 ? f2bf(theta[kOffW1 + k * 64 + c]) : (uint16_t)0;
    }
    if (t < 64 * 64) {
        const int c = t / 64, k = t % 64;
        pk[kPackW2t + t] = f2bf(theta[kOffW2 + k * 64 + c]);  // w2t[c][k] = W2[k][c]
        pk[kPackW2 + t] = f2bf(theta[kOffW2 + t]);            // w2 = W2
    }
    if (t < 16 * 64) {  // w3t[c][k] = W3[k][c]
        const int c = t / 64, k = t % 64;
        pk[kPackW3t + t] = c < 2 ? f2bf(theta[kOffW3 + k * 2 + c]) : (uint16_t)0;
    }
    if (t < 64 * 32) {  // w3p[r][k] = W3[r][k]
        const int r = t / 32, k = t % 32;
        pk[kPackW3p + t] = k < 2 ? f2bf(theta[kOffW3 + r * 2 + k]) : (uint16_t)0;
    }
}

hipError_t launch_mlp_pack(const float *theta, uint16_t *packed, hipStream_t s)
{
    hipLaunchKernelGGL(mlp_pack_kernel, dim3(16), dim3(256), 0, s, theta, packed);
    return hipGetLastError();
}

struct alignas(16) WeightLds {
    uint16_t w[kPackElems];
    float b1[64], b2[64], b3[4];
};

struct alignas(16) FwdLds {
    uint16_t X[kTile * 32];   // [hit][input], inputs 25..31 zero
    uint16_t H1[kTile * 64];  // [hit][unit]
    uint16_t H2[kTile * 64];
};

struct alignas(16) BwdLds {
    uint16_t D[kTile * 64];   // dH2 (bf16)
    uint16_t DY[kTile * 32];  // dY, columns 2..31 zero
};

// Copy the packed weights and biases into the workgroup's LDS.
__device__ __forceinline__ void stage_weights(WeightLds &W, const float *theta, const uint16_t *packed)
{
    const u32x4 *src = reinterpret_cast<const u32x4 *>(packed);
    u32x4 *dst = reinterpret_cast<u32x4 *>(W.w);
    for (int i = threadIdx.x; i < kPackElems / 8; i += blockDim.x) dst[i] = src[i];
    for (int i = threadIdx.x; i < 64; i += blockDim.x) {
        W.b1[i] = theta[kOffB1 + i];
        W.b2[i] = theta[kOffB2 + i];
    }
    if (threadIdx.x < 4) W.b3[threadIdx.x] = threadIdx.x < 2 ? theta[kOffB3 + threadIdx.x] : 0.0f;
}

// Forward pass of the tile of hits [h0, h0 + 32): X, H1, H2 in LDS (bf16),
// ReLU activity bits pos1/pos2 (bit i of [rt][nt] for C-layout row i), and
// the outputs y[rt] in C layout (columns 0 and 1 valid).  Rows past n hold
// zero inputs.
__device__ __forceinline__ void tile_forward(const float *patches, uint64_t n, uint64_t h0, float inv_adu,
                                             const WeightLds &W, FwdLds &F, int lane, f32x4 (&y)[2],
                                             uint32_t (&pos1)[2][4], uint32_t (&pos2)[2][4])
{
    const uint64_t nv = n - h0 < (uint64_t)kTile ? n - h0 : (uint64_t)kTile;
    const float *src = patches + h0 * 25;
    // every element of the tile is written, the padding columns 25..31 and
    // rows past n as zeros: LDS left over from earlier kernels may hold
    // bit patterns that read as bf16 inf or NaN, and inf * 0 is NaN
    for (int e = lane; e < kTile * 32; e += 64) {
        const int r = e >> 5, k = e & 31;
        const float v = (k < 25 && (uint64_t)r < nv) ? src[r * 25 + k] * inv_adu : 0.0f;
        F.X[e] = f2bf(v);
    }
    wave_lds_sync();
    const int lo = lane & 15, kq = 8 * (lane >> 4), rq = 4 * (lane >> 4);
    // layer 1: X[32 x 32] W1[32 x 64]
#pragma unroll
    for (int rt = 0; rt < 2; ++rt) {
        const bf16x8 a = frag<32, 1>(F.X, 16 * rt + lo, kq);
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            const f32x4 acc = mfma(a, frag<32, 1>(W.w + kPackW1t, 16 * nt + lo, kq), zero4());
            const int col = 16 * nt + lo;
            const float bias = W.b1[col];
            uint32_t pm = 0;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float z = acc[i] + bias;
                F.H1[(16 * rt + rq + i) * 64 + col] = f2bf(z > 0.0f ? z : 0.0f);
                pm |= (uint32_t)(z > 0.0f) << i;
            }
            pos1[rt][nt] = pm;
        }
    }
    wave_lds_sync();
    // layer 2: H1[32 x 64] W2[64 x 64]
#pragma unroll
    for (int rt = 0; rt < 2; ++rt) {
        const bf16x8 a0 = frag<64, 1>(F.H1, 16 * rt + lo, kq);
        const bf16x8 a1 = frag<64, 1>(F.H1, 16 * rt + lo, 32 + kq);
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            f32x4 acc = mfma(a0, frag<64, 1>(W.w + kPackW2t, 16 * nt + lo, kq), zero4());
            acc = mfma(a1, frag<64, 1>(W.w + kPackW2t, 16 * nt + lo, 32 + kq), acc);
            const int col = 16 * nt + lo;
            const float bias = W.b2[col];
            uint32_t pm = 0;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float z = acc[i] + bias;
                F.H2[(16 * rt + rq + i) * 64 + col] = f2bf(z > 0.0f ? z : 0.0f);
                pm |= (uint32_t)(z > 0.0f) << i;
            }
            pos2[rt][nt] = pm;
        }
    }
    wave_lds_sync();
    // layer 3: H2[32 x 64] W3[64 x 16] (output columns 2..15 zero)
    const float b3 = W.b3[lo < 2 ? lo : 3];
#pragma unroll
    for (int rt = 0; rt < 2; ++rt) {
        f32x4 acc = mfma(frag<64, 1>(F.H2, 16 * rt + lo, kq), frag<64, 1>(W.w + kPackW3t, lo, kq), zero4());
        acc = mfma(frag<64, 1>(F.H2, 16 * rt + lo, 32 + kq), frag<64, 1>(W.w + kPackW3t, lo, 32 + kq), acc);
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[i] = acc[i] + b3;
        y[rt] = acc;
    }
}

// Inference: out[2h], out[2h + 1] = (dy, dx) of hit h, with every activation
// kept in registers.  Each layer is computed transposed, Z^T = W^T H^T: the
// weights are the A operand (rows = output units) and a 16-hit tile the B
// operand (columns = hits), so the result fragment of lane (n, g) holds units
// 16 m + 4 g + i of hit n.  After bias, ReLU and rounding to bf16 those values
// are the next layer's B operand as they stand, once the contraction index is
// permuted: slot (g, j) of K-chunk c stands for unit 16 (2 c + j / 4) + 4 g +
// j % 4, which lane group g holds, and the weight fragments are loaded in the
// same order.  The first layer's B operand comes straight from the patches
// (lane (n, g) takes inputs 8 g .. 8 g + 7 of hit n), the next tile's values
// loaded while the current one is in the MFMAs.  The weights (the bf16 copies training uses)
// and biases stay in registers for the whole run.
// Products use the training forward pass's bf16 operands; the float32 sums
// differ from it in order only (the bias starts the accumulator here, where
// training adds it to the finished sum).
constexpr int kInferWaves = 4;

// The 32-hit tile's 800 patch words as 200 16-byte groups, lane l taking
// groups l + 64 k, through a buffer resource that covers the tile only if
// all its hits exist (else nothing: every group reads as 0).  The same four
// loads whatever the tile, so that the wait counts of the loop below are
// the same on every path.
constexpr int kXWords = kTile * 25, kXGroups = kXWords / 4;
__device__ __forceinline__ void load_x_full(const float *patches, uint64_t n, uint64_t h0, int lane, u32x4 (&xv)[4])
{
    const int bytes = h0 + kTile <= n ? kXWords * 4 : 0;
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<float *>(patches + h0 * 25), 0, bytes, 0x00020000);
#pragma unroll
    for (int k = 0; k < 4; ++k)
        xv[k] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(rs, 16 * (lane + 64 * k), 0, 0));
}

// A partial last tile (h0 < n < h0 + 32), word by word, each word range-
// checked on its own, so that words past the last hit read as 0.
__device__ __forceinline__ void load_x_part(const float *patches, uint64_t n, uint64_t h0, int lane, u32x4 (&xv)[4])
{
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<float *>(patches + h0 * 25), 0, (int)((n - h0) * 100), 0x00020000);
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int i = 0; i < 4; ++i) xv[k][i] = __builtin_amdgcn_raw_buffer_load_b32(rs, 16 * (lane + 64 * k) + 4 * i, 0, 0);
}

// ReLU and bf16 of the result fragments d[2c], d[2c + 1] (bias included):
// K-chunk c.  Rounding keeps the sign, so ReLU is applied to the bf16 values,
// two per instruction, as a signed 16-bit max with 0 (negative values and -0
// have the sign bit set).
__device__ __forceinline__ bf16x8 relu_chunk(const f32x4 &d0, const f32x4 &d1)
{
    const u32x4 w = {pk_bf16(d0[0], d0[1]), pk_bf16(d0[2], d0[3]), pk_bf16(d1[0], d1[1]), pk_bf16(d1[2], d1[3])};
    const i16x8 v = __builtin_elementwise_max(__builtin_bit_cast(i16x8, w), i16x8{0, 0, 0, 0, 0, 0, 0, 0});
    return __builtin_bit_cast(bf16x8, v);
}

// The first layer's B operand of a 32-hit tile of network inputs (IN16):
// lane (n, g) loads words 8 g .. 8 g + 7 of hits n and 16 + n, one 16-byte
// load each, through a resource that covers the tile's own hits.  Two loads
// whatever the tile, as for the patches.
__device__ __forceinline__ void load_in_tile(const uint16_t *inputs, uint64_t n, uint64_t h0, int lane, u32x4 (&xq)[2])
{
    // hits past n (a whole tile past the end too) read as 0: each lane's
    // 16 bytes lie wholly inside or outside the resource
    const uint64_t nv = h0 >= n ? 0 : (n - h0 < (uint64_t)kTile ? n - h0 : (uint64_t)kTile);
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<uint16_t *>(inputs + h0 * kMlpInWords), 0, (int)(nv * 2 * kMlpInWords), 0x00020000);
    const int lo = lane & 15, g = lane >> 4;
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
        xq[rt] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(
                                               rs, (16 * rt + lo) * 2 * kMlpInWords + 16 * g, 0, 0));
}

// IN16: src holds the network's inputs (uint16 [n][kMlpInWords], inv_adu
// unused), else float32 patches [n][25].
template <bool IN16>
__device__ __forceinline__ void mlp_infer_body(const void *src, uint64_t n, float inv_adu, const float *theta,
                                               const uint16_t *packed, float *out)
{
    const int lane = threadIdx.x & 63;
    const int r = lane & 15, g = lane >> 4;
    // weight fragments from the packed bf16 copies: lane (r, g) takes row
    // 16 m + r of w1t (columns 8 g .. 8 g + 7) and of w2t, and row r of w3t,
    // the latter two at the permuted columns (two runs of 4)
    bf16x8 w1[4], w2[4][2], w3[2];
    // biases in LDS (registers are kept for the weights): lane group g reads
    // the 4 of units 16 m + 4 g .. + 3 as an accumulator start
    __shared__ __align__(16) float s_b[128];
    for (int i = threadIdx.x; i < 128; i += blockDim.x) s_b[i] = theta[i < 64 ? kOffB1 + i : kOffB2 + i - 64];
    float b3[2];
    typedef __attribute__((ext_vector_type(2))) unsigned int u32x2v;
    auto runs = [&](const uint16_t *row, int c) {
        const u32x2v p0 = *reinterpret_cast<const u32x2v *>(row + 32 * c + 4 * g);
        const u32x2v p1 = *reinterpret_cast<const u32x2v *>(row + 32 * c + 16 + 4 * g);
        return __builtin_bit_cast(bf16x8, u32x4{p0[0], p0[1], p1[0], p1[1]});
    };
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        w1[m] = frag<32, 1>(packed + kPackW1t, 16 * m + r, 8 * g);
#pragma unroll
        for (int c = 0; c < 2; ++c) w2[m][c] = runs(packed + kPackW2t + (16 * m + r) * 64, c);
    }
#pragma unroll
    for (int c = 0; c < 2; ++c) w3[c] = runs(packed + kPackW3t + r * 64, c);
    b3[0] = theta[kOffB3];
    b3[1] = theta[kOffB3 + 1];
    // wait for these loads here: a first use inside the loop below would wait
    // for every load in flight there, the next tile's included (vmcnt 0)
    __builtin_amdgcn_s_waitcnt(0x0F70);
    __syncthreads();  // the biases in LDS

    // inputs 25..31 (lane group 3, slots 1..7) are zero (also for network
    // inputs, whose padding words a caller may have left unset)
    const u32x4 xmask = g < 3 ? u32x4{~0u, ~0u, ~0u, ~0u} : u32x4{0xFFFFu, 0u, 0u, 0u};
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint64_t tiles = (n + kTile - 1) / kTile;
    const uint64_t stride = (uint64_t)gridDim.x * kInferWaves;
    uint64_t t = (uint64_t)blockIdx.x * kInferWaves + wv;
    // float32 patches: the wave's tile, staged in LDS so that the loads stay
    // coalesced; lane (n, g) then reads inputs 8 g .. 8 g + 7 of hits n and
    // 16 + n (lane group 3 also reads the words after input 24, which the mask
    // clears)
    __shared__ float s_x[IN16 ? 1 : kInferWaves][kXWords + 32];
    float *xs = s_x[IN16 ? 0 : wv];
    const float *patches = static_cast<const float *>(src);
    const uint16_t *inputs = static_cast<const uint16_t *>(src);
    // tiles are loaded kDepth ahead of their use (kDepth register buffers,
    // the loop unrolled over them; the patches' larger buffers leave room for
    // one).  Loads are issued for tiles past the end too (they read
    // nothing), so that every path waits for the same counts.  Float32 patches:
    // the loop takes the whole tiles, a partial last tile comes after it.
    constexpr int kDepth = 1;
    const uint64_t full = IN16 ? tiles : n / kTile;
    u32x4 xv[kDepth][4];
    auto load = [&](uint64_t tile, auto &buf) {
        if constexpr (IN16)
            load_in_tile(inputs, n, tile * kTile, lane, buf);
        else
            load_x_full(patches, n, tile * kTile, lane, buf);
    };
    // float32 patches of the tile in buf, staged in LDS, as B operands
    auto stage = [&](const u32x4 (&buf)[4], bf16x8 (&x)[2]) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (lane + 64 * q < kXGroups) *reinterpret_cast<u32x4 *>(xs + 4 * (lane + 64 * q)) = buf[q];
        wave_lds_wait();
#pragma unroll
        for (int rt = 0; rt < 2; ++rt) {
            const float *sp = xs + (16 * rt + r) * 25 + 8 * g;
            u32x4 xw;
#pragma unroll
            for (int j = 0; j < 4; ++j) xw[j] = pk_bf16(sp[2 * j] * inv_adu, sp[2 * j + 1] * inv_adu);
            x[rt] = __builtin_bit_cast(bf16x8, xw & xmask);
        }
        wave_lds_wait();
    };
    auto forward = [&](uint64_t tk, const bf16x8 (&x)[2]) {
        // the bias reads stay in the loop (an opaque offset each tile): kept
        // in registers they would cost the waves per SIMD they save
        int go = g;
        asm volatile("" : "+v"(go));
        const f32x4 *b1 = reinterpret_cast<const f32x4 *>(s_b) + go, *b2 = b1 + 16;
        f32x4 y[2];
#pragma unroll
        for (int rt = 0; rt < 2; ++rt) {
            f32x4 d[4];
#pragma unroll
            for (int m = 0; m < 4; ++m) d[m] = mfma(w1[m], x[rt], b1[4 * m]);
            const bf16x8 h1a = relu_chunk(d[0], d[1]), h1b = relu_chunk(d[2], d[3]);
#pragma unroll
            for (int m = 0; m < 4; ++m) d[m] = mfma(w2[m][1], h1b, mfma(w2[m][0], h1a, b2[4 * m]));
            const bf16x8 h2a = relu_chunk(d[0], d[1]), h2b = relu_chunk(d[2], d[3]);
            y[rt] = mfma(w3[1], h2b, mfma(w3[0], h2a, zero4()));
        }
        if (g == 0) {
            const uint64_t h0 = tk * kTile;
#pragma unroll
            for (int rt = 0; rt < 2; ++rt) {
                const uint64_t h = h0 + 16 * rt + r;
                if (h < n)
                    *reinterpret_cast<float2 *>(out + 2 * h) = make_float2(y[rt][0] + b3[0], y[rt][1] + b3[1]);
            }
        }
    };
    if constexpr (IN16) {
        // two sets of kSet tiles, each loaded while the other is computed: the
        // set in use was issued before the other on every path, so the waits
        // for it leave the other's loads in flight
        constexpr int kSet = 2;
        u32x4 sa[kSet][2], sb[kSet][2];
#pragma unroll
        for (int k = 0; k < kSet; ++k) load(t + k * stride, sa[k]);
        for (; t < full; t += 2 * kSet * stride) {
#pragma unroll
            for (int k = 0; k < kSet; ++k) load(t + (kSet + k) * stride, sb[k]);
#pragma unroll
            for (int k = 0; k < kSet; ++k) {
                const uint64_t tk = t + k * stride;
                if (tk < full) {
                    const bf16x8 x[2] = {__builtin_bit_cast(bf16x8, sa[k][0] & xmask),
                                         __builtin_bit_cast(bf16x8, sa[k][1] & xmask)};
                    forward(tk, x);
                }
            }
#pragma unroll
            for (int k = 0; k < kSet; ++k) load(t + (2 * kSet + k) * stride, sa[k]);
#pragma unroll
            for (int k = 0; k < kSet; ++k) {
                const uint64_t tk = t + (kSet + k) * stride;
                if (tk < full) {
                    const bf16x8 x[2] = {__builtin_bit_cast(bf16x8, sb[k][0] & xmask),
                                         __builtin_bit_cast(bf16x8, sb[k][1] & xmask)};
                    forward(tk, x);
                }
            }
        }
    } else {
#pragma unroll
        for (int k = 0; k < kDepth; ++k) load(t + k * stride, xv[k]);
        for (; t < full; t += kDepth * stride)
#pragma unroll
            for (int k = 0; k < kDepth; ++k) {
                const uint64_t tk = t + k * stride;
                if (tk >= full) break;
                bf16x8 x[2];
                stage(xv[k], x);
                load(tk + kDepth * stride, xv[k]);
                forward(tk, x);
            }
    }
    if (!IN16 && full < tiles && (uint64_t)blockIdx.x * kInferWaves + wv == full % stride) {
        u32x4 buf[4];
        load_x_part(patches, n, full * kTile, lane, buf);
        bf16x8 x[2];
        stage(buf, x);
        forward(full, x);
    }
}

__global__ void __launch_bounds__(64 * kInferWaves) mlp_infer_kernel(const void *src, uint64_t n, float inv_adu,
                                                                     const float *theta, const uint16_t *packed,
                                                                     float *out)
{
    mlp_infer_body<false>(src, n, inv_adu, theta, packed, out);
}

__global__ void __launch_bounds__(64 * kInferWaves) mlp_infer_inputs_kernel(const void *src, uint64_t n, float inv_adu, const float *theta, const uint16_t *packed,
                        float *out)
{
    mlp_infer_body<true>(src, n, inv_adu, theta, packed, out);
}

// At most the workgroups that are resident at once: every wave loads the
// weights once and then takes tiles until none are left.
template <bool IN16>
static hipError_t launch_infer(const void *src, uint64_t n, float inv_adu, const float *theta,
                               const uint16_t *packed, float *out, uint32_t max_grid, hipStream_t s)
{
    const auto kernel = IN16 ? mlp_infer_inputs_kernel : mlp_infer_kernel;
    if (n == 0) return hipSuccess;
    static std::atomic<int> resident[64];
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    int res = dev < 64 ? resident[dev].load(std::memory_order_relaxed) : 0;
    if (res <= 0) {
        int per_cu = 0, n_cu = 0;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void *>(kernel),
                                                         64 * kInferWaves, 0);
        if (e != hipSuccess) return e;
        e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return e;
        res = (per_cu > 0 ? per_cu : 1) * (n_cu > 0 ? n_cu : 1);
        if (dev < 64) resident[dev].store(res, std::memory_order_relaxed);
    }
    const uint64_t tiles = (n + kTile - 1) / kTile;
    uint64_t grid = (tiles + kInferWaves - 1) / kInferWaves;
    if (grid > max_grid) grid = max_grid;
    if (grid > (uint64_t)res) grid = (uint64_t)res;
    hipLaunchKernelGGL(kernel, dim3((uint32_t)grid), dim3(64 * kInferWaves), 0, s, src, n, inv_adu, theta, packed,
                       out);
    return hipGetLastError();
}

hipError_t launch_mlp_infer(const float *patches, uint64_t n, float inv_adu, const float *theta,
                            const uint16_t *packed, float *out, uint32_t max_grid, hipStream_t s)
{
    return launch_infer<false>(patches, n, inv_adu, theta, packed, out, max_grid, s);
}

hipError_t launch_mlp_infer_inputs(const uint16_t *inputs, uint64_t n, const float *theta, const uint16_t *packed,
                                   float *out, uint32_t max_grid, hipStream_t s)
{
    return launch_infer<true>(inputs, n, 0.0f, theta, packed, out, max_grid, s);
}

// Sum over the 4 lane groups that share l % 16 (the rows of a C tile).
__device__ __forceinline__ float col_sum(float v)
{
    v += __shfl_xor(v, 16, 64);
    v += __shfl_xor(v, 32, 64);
    return v;
}

// Per-wave gradient of L = sum((y - t)^2) / (2 n) over its tiles, written to
// the wave's slot (kMlpSlotStride floats: parameters in packed order, then
// sum((y - t)^2)).  Products take bf16 operands (X, H1, H2, dY, dH2, dH1 and
// the weights) with float32 accumulation; bias gradients sum float32 values.
__global__ void __launch_bounds__(256) mlp_grad_kernel(const float *patches, const float *target, uint64_t n,
                                                       float inv_adu, float inv_n, const float *theta,
                                                       const uint16_t *packed, float *slots)
{
    __shared__ WeightLds W;
    __shared__ FwdLds Fs[kWaves];
    __shared__ BwdLds Bs[kWaves];
    stage_weights(W, theta, packed);
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    FwdLds &F = Fs[wv];
    BwdLds &Bk = Bs[wv];
    for (int i = lane; i < kTile * 32; i += 64) Bk.DY[i] = 0;
    __syncthreads();
    const int lo = lane & 15, kq = 8 * (lane >> 4), rq = 4 * (lane >> 4);

    f32x4 gW1[2][4], gW2[4][4], gW3[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        gW3[a] = zero4();
#pragma unroll
        for (int b = 0; b < 4; ++b) gW2[a][b] = zero4();
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) gW1[a][b] = zero4();
    float gb1[4] = {0.f, 0.f, 0.f, 0.f}, gb2[4] = {0.f, 0.f, 0.f, 0.f}, gb3 = 0.f, lsum = 0.f;

    const uint64_t tiles = (n + kTile - 1) / kTile;
    for (uint64_t t = (uint64_t)blockIdx.x * kWaves + wv; t < tiles; t += (uint64_t)gridDim.x * kWaves) {
        const uint64_t h0 = t * kTile;
        f32x4 y[2];
        uint32_t p1[2][4], p2[2][4];
        tile_forward(patches, n, h0, inv_adu, W, F, lane, y, p1, p2);
        // dY = (y - t) / n, zero for columns >= 2 and rows past n
#pragma unroll
        for (int rt = 0; rt < 2; ++rt)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int row = 16 * rt + rq + i;
                const uint64_t h = h0 + row;
                float d = 0.0f;
                if (lo < 2 && h < n) {
                    const float e = y[rt][i] - target[2 * h + lo];
                    lsum += e * e;
                    d = e * inv_n;
                }
                gb3 += d;
                Bk.DY[row * 32 + lo] = f2bf(d);
            }
        wave_lds_sync();
        // dW3[64 x 16] += H2^T[64 x 32] dY[32 x 16]
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
            gW3[mt] = mfma(frag<1, 64>(F.H2, 16 * mt + lo, kq), frag<1, 32>(Bk.DY, lo, kq), gW3[mt]);
        // dH2[32 x 64] = (dY[32 x 32] W3^T[32 x 64]) * relu'(z2)
#pragma unroll
        for (int rt = 0; rt < 2; ++rt) {
            const bf16x8 a = frag<32, 1>(Bk.DY, 16 * rt + lo, kq);
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) {
                const f32x4 acc = mfma(a, frag<32, 1>(W.w + kPackW3p, 16 * nt + lo, kq), zero4());
                const int col = 16 * nt + lo;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const float g = ((p2[rt][nt] >> i) & 1u) ? acc[i] : 0.0f;
                    gb2[nt] += g;
                    Bk.D[(16 * rt + rq + i) * 64 + col] = f2bf(g);
                }
            }
        }
        wave_lds_sync();
        // dW2[64 x 64] += H1^T[64 x 32] dH2[32 x 64]
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            const bf16x8 a = frag<1, 64>(F.H1, 16 * mt + lo, kq);
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) gW2[mt][nt] = mfma(a, frag<1, 64>(Bk.D, 16 * nt + lo, kq), gW2[mt][nt]);
        }
        // dH1[32 x 64] = (dH2[32 x 64] W2^T[64 x 64]) * relu'(z1), into H2's space
#pragma unroll
        for (int rt = 0; rt < 2; ++rt) {
            const bf16x8 a0 = frag<64, 1>(Bk.D, 16 * rt + lo, kq);
            const bf16x8 a1 = frag<64, 1>(Bk.D, 16 * rt + lo, 32 + kq);
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) {
                f32x4 acc = mfma(a0, frag<64, 1>(W.w + kPackW2, 16 * nt + lo, kq), zero4());
                acc = mfma(a1, frag<64, 1>(W.w + kPackW2, 16 * nt + lo, 32 + kq), acc);
                const int col = 16 * nt + lo;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const float g = ((p1[rt][nt] >> i) & 1u) ? acc[i] : 0.0f;
                    gb1[nt] += g;
                    F.H2[(16 * rt + rq + i) * 64 + col] = f2bf(g);
                }
            }
        }
        wave_lds_sync();
        // dW1[32 x 64] += X^T[32 x 32] dH1[32 x 64]
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) {
            const bf16x8 a = frag<1, 32>(F.X, 16 * mt + lo, kq);
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) gW1[mt][nt] = mfma(a, frag<1, 64>(F.H2, 16 * nt + lo, kq), gW1[mt][nt]);
        }
        wave_lds_sync();
    }

    float *slot = slots + ((uint64_t)blockIdx.x * kWaves + wv) * kMlpSlotStride;
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int k = 16 * mt + rq + i;
                if (k < 25) slot[kOffW1 + k * 64 + 16 * nt + lo] = gW1[mt][nt][i];
            }
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
            for (int i = 0; i < 4; ++i) slot[kOffW2 + (16 * mt + rq + i) * 64 + 16 * nt + lo] = gW2[mt][nt][i];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int i = 0; i < 4; ++i)
            if (lo < 2) slot[kOffW3 + (16 * mt + rq + i) * 2 + lo] = gW3[mt][i];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        const float s1 = col_sum(gb1[nt]);
        const float s2 = col_sum(gb2[nt]);
        if (lane < 16) {
            slot[kOffB1 + 16 * nt + lane] = s1;
            slot[kOffB2 + 16 * nt + lane] = s2;
        }
    }
    const float s3 = col_sum(gb3);
    if (lane < 2) slot[kOffB3 + lane] = s3;
    for (int d = 32; d >= 1; d >>= 1) lsum += __shfl_xor(lsum, d, 64);
    if (lane == 0) slot[kMlpParams] = lsum;
}

// out[p] = sum over the slots in index order (deterministic), p <= kMlpParams.
__global__ void slot_reduce_kernel(const float *slots, uint32_t n_slots, float *out)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p > kMlpParams) return;
    float s = 0.0f;
    for (uint32_t i = 0; i < n_slots; ++i) s += slots[(uint64_t)i * kMlpSlotStride + p];
    out[p] = s;
}

uint32_t mlp_grad_grid(uint64_t n, uint32_t max_grid)
{
    const uint64_t tiles = (n + kTile - 1) / kTile;
    uint64_t grid = (tiles + kWaves - 1) / kWaves;
    if (grid > max_grid) grid = max_grid;
    return grid ? (uint32_t)grid : 1u;
}

hipError_t launch_mlp_grad(const float *patches, const float *target, uint64_t n, float inv_adu,
                           const float *theta, const uint16_t *packed, float *out, float *slots, uint32_t max_grid,
                           hipStream_t s)
{
    if (n == 0) return launch_fill_zero(out, kMlpParams + 1, s);
    const uint32_t grid = mlp_grad_grid(n, max_grid);
    hipLaunchKernelGGL(mlp_grad_kernel, dim3(grid), dim3(64 * kWaves), 0, s, patches, target, n, inv_adu,
                       (float)(1.0 / (double)n), theta, packed, slots);
    hipLaunchKernelGGL(slot_reduce_kernel, dim3((kMlpParams + 256) / 256), dim3(256), 0, s, slots,
                       grid * (uint32_t)kWaves, out);
    return hipGetLastError();
}

// Adam in float32, every operation rounded to nearest even:
//   m = b1 m + (1 - b1) g;  v = b2 v + ((1 - b2) g) g;
//   theta -= (lr (m / c1)) / (sqrt(v / c2) + eps),  c1 = 1 - b1^t, c2 = 1 - b2^t.
// sqrtf is correctly rounded under -fhip-fp32-correctly-rounded-divide-sqrt;
// __fsqrt_rn is not used: it maps to the native approximation.
// One training step's update after mlp_grad_kernel, in one kernel: each
// parameter's gradient summed over the slots in index order (the additions
// of slot_reduce_kernel, with the loads issued eight ahead), then Adam as
// above, then the bf16 copies of the new value in every packed layout
// (the packing's zero padding is never written).  grad also receives the
// sums (the loss term at kMlpParams).
__global__ void mlp_update_kernel(const float *slots, uint32_t n_slots, float *grad, float *theta, float *m, float *v,
                                  float lr, float b1, float omb1, float b2, float omb2, float eps, float c1, float c2,
                                  uint16_t *pk)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p > kMlpParams) return;
    float s = 0.0f;
    uint32_t i = 0;
    for (; i + 8 <= n_slots; i += 8) {
        float t[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) t[j] = slots[(uint64_t)(i + j) * kMlpSlotStride + p];
#pragma unroll
        for (int j = 0; j < 8; ++j) s += t[j];
    }
    for (; i < n_slots; ++i) s += slots[(uint64_t)i * kMlpSlotStride + p];
    grad[p] = s;
    if (p == kMlpParams) return;
    const float g = s;
    const float mi = __fadd_rn(__fmul_rn(b1, m[p]), __fmul_rn(omb1, g));
    const float vi = __fadd_rn(__fmul_rn(b2, v[p]), __fmul_rn(__fmul_rn(omb2, g), g));
    m[p] = mi;
    v[p] = vi;
    const float step = __fdiv_rn(__fmul_rn(lr, __fdiv_rn(mi, c1)), __fadd_rn(sqrtf(__fdiv_rn(vi, c2)), eps));
    const float th = __fsub_rn(theta[p], step);
    theta[p] = th;
    const uint16_t b = f2bf(th);
    if (p < kOffB1) {  // W1[k][c]
        const int k = p / 64, c = p % 64;
        pk[kPackW1t + c * 32 + k] = b;
    } else if (p >= kOffW2 && p < kOffB2) {  // W2[k][c]
        const int q = p - kOffW2, k = q / 64, c = q % 64;
        pk[kPackW2t + c * 64 + k] = b;
        pk[kPackW2 + q] = b;
    } else if (p >= kOffW3 && p < kOffB3) {  // W3[k][c]
        const int q = p - kOffW3, k = q / 2, c = q % 2;
        pk[kPackW3t + c * 64 + k] = b;
        pk[kPackW3p + k * 32 + c] = b;
    }
}

hipError_t launch_mlp_train(const float *patches, const float *target, uint64_t n, float inv_adu, float *theta,
                            float *m, float *v, uint16_t *packed, float *grad, float *slots, uint32_t max_grid,
                            float lr, int64_t step, hipStream_t s)
{
    if (n == 0) return hipErrorInvalidValue;
    const uint32_t grid = mlp_grad_grid(n, max_grid);
    hipLaunchKernelGGL(mlp_grad_kernel, dim3(grid), dim3(64 * kWaves), 0, s, patches, target, n, inv_adu,
                       (float)(1.0 / (double)n), theta, packed, slots);
    const double b1 = 0.9, b2 = 0.999;
    const float c1 = (float)(1.0 - pow(b1, (double)step)), c2 = (float)(1.0 - pow(b2, (double)step));
    hipLaunchKernelGGL(mlp_update_kernel, dim3((kMlpParams + 256) / 256), dim3(256), 0, s, slots,
                       grid * (uint32_t)kWaves, grad, theta, m, v, lr, (float)b1, (float)(1.0 - b1), (float)b2,
                       (float)(1.0 - b2), 1e-8f, c1, c2, packed);
    return hipGetLastError();
}

// 5x5 neighbourhood of each hit in the corrected frames (zero outside the
// tile).  hits[i] = {pixel, charge bits} of the raster-order list; its frame
// is the largest f with frame_offset[f] <= i.
// A captured patch goes out as 25 float32 values (patches[i][25]) or as the
// network's input (inputs != nullptr): bf16(fl(v * inv_adu)) of each value,
// then 7 zero words, 64 bytes per hit (inputs[i][32]).
__device__ __forceinline__ void store_patch(const float (&v)[25], uint64_t i, float *patches, uint16_t *inputs,
                                            float inv_adu)
{
    if (inputs) {
        u32x4 *dst = reinterpret_cast<u32x4 *>(inputs + i * kMlpInWords);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            u32x4 w;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int e = 8 * q + 2 * j;
                w[j] = pk_bf16(e < 25 ? v[e] * inv_adu : 0.0f, e + 1 < 25 ? v[e + 1] * inv_adu : 0.0f);
            }
            dst[q] = w;
        }
    } else {
#pragma unroll
        for (int e = 0; e < 25; ++e) patches[i * 25 + e] = v[e];
    }
}

// Frame of hit i: the last frame whose first hit is at most i.
__device__ __forceinline__ uint64_t hit_frame(const unsigned long long *frame_offset, uint64_t n_frames, uint64_t i)
{
    uint64_t lo = 0, hi = n_frames;
    while (hi - lo > 1) {
        const uint64_t mid = (lo + hi) / 2;
        if (frame_offset[mid] <= i) lo = mid;
        else hi = mid;
    }
    return lo;
}

__global__ void capture_patches_kernel(const float *corrected, const uint2 *hits,
                                       const unsigned long long *frame_offset, uint64_t n_frames, uint64_t n, int T,
                                       int H, int W, float *patches, uint16_t *inputs, float inv_adu)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint64_t lo = hit_frame(frame_offset, n_frames, i);
    const uint32_t p = hits[i].x;
    const int c = (int)(p % (uint32_t)W);
    const int rt = (int)(p / (uint32_t)W);
    const int t = rt / H, r = rt - t * H;
    const float *fr = corrected + (lo * (uint64_t)T + (uint64_t)t) * (uint64_t)H * W;
    float v[25];
#pragma unroll
    for (int dr = -2; dr <= 2; ++dr)
#pragma unroll
        for (int dc = -2; dc <= 2; ++dc) {
            const int rr = r + dr, cc = c + dc;
            v[(dr + 2) * 5 + dc + 2] = (rr >= 0 && rr < H && cc >= 0 && cc < W) ? fr[(uint64_t)rr * W + cc] : 0.0f;
        }
    store_patch(v, i, patches, inputs, inv_adu);
}

hipError_t launch_capture_patches(const float *corrected, const uint2 *hits, const unsigned long long *frame_offset,
                                  uint64_t n_frames, uint64_t n, int T, int H, int W, float *patches,
                                  uint16_t *inputs, float inv_adu, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(capture_patches_kernel, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, s, corrected, hits,
                       frame_offset, n_frames, n, T, H, W, patches, inputs, inv_adu);
    return hipGetLastError();
}

// Frames2 of pixel (rr, cc) of tile t of frame lo, formed again from its raw
// word, the calibration and the kept common-mode values by the frame
// kernels' operations (an invalid gain code gives +0).
__device__ __forceinline__ float frames2_at(const PatchSrc &a, uint64_t lo, int t, int rr, int cc)
{
    const int H = a.H, W = a.W;
    const uint64_t HW = (uint64_t)H * W, npix = (uint64_t)a.T * HW;
    const uint64_t q = (uint64_t)t * HW + (uint64_t)rr * W + cc;
    const uint32_t w = a.frames[lo * npix + q];
    bool bad = false;
    const float u = a.gain_mode ? dark_gain_ranged(w, a.gain_mode, a.ped[q], a.k[q], a.ped, a.k, npix, q, bad)
                                : dark_gain(w, a.ped[q], a.k[q]);
    const uint32_t grow = (uint32_t)(t * H + rr);
    if (a.meds) {
        const float m = a.meds[lo * (uint64_t)a.T * H * a.nb + (uint64_t)grow * a.nb + cc / a.B];
        return bad ? 0.0f : __fsub_rn(u, m);  // invalid: fl(m - m) = +0
    }
    const uint32_t reg = a.cm_tile ? (uint32_t)t : grow * (uint32_t)a.nb + (uint32_t)(cc / a.B);
    const float *cv = a.cm + (lo * a.cm_regions + reg) * 3;
    return bad ? 0.0f : __fsub_rn(__fsub_rn(__fsub_rn(u, cv[0]), cv[1]), cv[2]);
}

// The same patches without Frames2: each window pixel's Frames2 value formed
// again (frames2_at).
__global__ void patches_from_frames_kernel(PatchSrc a, const uint2 *hits, const unsigned long long *frame_offset,
                                           uint64_t n_frames, uint64_t n, float *patches, uint16_t *inputs,
                                           float inv_adu)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint64_t lo = hit_frame(frame_offset, n_frames, i);
    const int H = a.H, W = a.W;
    const uint32_t p = hits[i].x;
    const int c = (int)(p % (uint32_t)W);
    const int rt = (int)(p / (uint32_t)W);
    const int t = rt / H, r = rt - t * H;
    float out[25];
#pragma unroll
    for (int dr = -2; dr <= 2; ++dr)
#pragma unroll
        for (int dc = -2; dc <= 2; ++dc) {
            const int rr = r + dr, cc = c + dc;
            out[(dr + 2) * 5 + dc + 2] = (rr >= 0 && rr < H && cc >= 0 && cc < W) ? frames2_at(a, lo, t, rr, cc) : 0.0f;
        }
    store_patch(out, i, patches, inputs, inv_adu);
}

// Classical positions straight from a batch: the masked 3x3 centroid of each
// hit (eta-corrected when eta is not NULL) from its Frames2 values, read from
// corrected when Frames2 was kept, else formed again (frames2_at); the same
// arithmetic as centroid_eta_kernel on the hit's patch.  only_bad: pos holds
// positions already (the learned estimator's) and only those that are not
// finite or outside [-1, 1] in a coordinate are replaced.
__global__ void centroids_kernel(PatchSrc a, const float *corrected, const uint2 *hits,
                                 const unsigned long long *frame_offset, uint64_t n_frames, uint64_t n, float t_nb,
                                 const float *eta, int nbins, int only_bad, float *pos)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (only_bad && fabsf(pos[2 * i]) <= 1.0f && fabsf(pos[2 * i + 1]) <= 1.0f) return;  // NaN is replaced
    const uint64_t lo = hit_frame(frame_offset, n_frames, i);
    const int H = a.H, W = a.W;
    const uint32_t p = hits[i].x;
    const int c = (int)(p % (uint32_t)W);
    const int rt = (int)(p / (uint32_t)W);
    const int t = rt / H, r = rt - t * H;
    float v[25];
#pragma unroll
    for (int e = 0; e < 25; ++e) v[e] = 0.0f;
#pragma unroll
    for (int dr = -1; dr <= 1; ++dr)
#pragma unroll
        for (int dc = -1; dc <= 1; ++dc) {
            const int rr = r + dr, cc = c + dc;
            if (rr >= 0 && rr < H && cc >= 0 && cc < W)
                v[(dr + 2) * 5 + dc + 2] = corrected ? corrected[((lo * a.T + t) * H + rr) * (uint64_t)W + cc]
                                                     : frames2_at(a, lo, t, rr, cc);
        }
    float cy, cx;
    centroid3(v, t_nb, cy, cx);
    if (eta) {
        cy = eta_map(eta, nbins, cy);
        cx = eta_map(eta + nbins + 1, nbins, cx);
    }
    pos[2 * i] = cy;
    pos[2 * i + 1] = cx;
}

hipError_t launch_centroids(const PatchSrc &a, const float *corrected, const uint2 *hits,
                            const unsigned long long *frame_offset, uint64_t n_frames, uint64_t n, float t_nb,
                            const float *eta, int nbins, int only_bad, float *pos, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(centroids_kernel, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, s, a, corrected, hits,
                       frame_offset, n_frames, n, t_nb, eta, nbins, only_bad, pos);
    return hipGetLastError();
}

hipError_t launch_patches_from_frames(const PatchSrc &a, const uint2 *hits, const unsigned long long *frame_offset,
                                      uint64_t n_frames, uint64_t n, float *patches, uint16_t *inputs, float inv_adu,
                                      hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(patches_from_frames_kernel, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, s, a, hits,
                       frame_offset, n_frames, n, patches, inputs, inv_adu);
    return hipGetLastError();
}

// Network inputs of n float32 patches: thread 4 h + q writes words 8 q .. 8 q
// + 7 of hit h (16 bytes; consecutive threads write consecutive groups).
__global__ void make_inputs_kernel(const float *patches, uint64_t n, float inv_adu, uint16_t *inputs)
{
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 4 * n) return;
    const uint64_t h = t >> 2;
    const int q = (int)(t & 3);
    const float *src = patches + h * 25 + 8 * q;
    u32x4 w;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int e = 8 * q + 2 * j;
        w[j] = pk_bf16(e < 25 ? src[2 * j] * inv_adu : 0.0f, e + 1 < 25 ? src[2 * j + 1] * inv_adu : 0.0f);
    }
    reinterpret_cast<u32x4 *>(inputs + h * kMlpInWords)[q] = w;
}

hipError_t launch_make_inputs(const float *patches, uint64_t n, float inv_adu, uint16_t *inputs, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(make_inputs_kernel, dim3((uint32_t)((4 * n + 255) / 256)), dim3(256), 0, s, patches, n,
                       inv_adu, inputs);
    return hipGetLastError();
}

// One 16x32 by 32x16 bf16 product D = A B (A, B, D row-major) through the
// same fragment loads as the network kernels: checks the operand layout.
__global__ void mfma_probe_kernel(const uint16_t *A, const uint16_t *B, float *D)
{
    __shared__ alignas(16) uint16_t a[16 * 32];
    __shared__ alignas(16) uint16_t bt[16 * 32];  // B^T: [col][k]
    const int lane = threadIdx.x;
    for (int e = lane; e < 16 * 32; e += 64) {
        a[e] = A[e];
        const int k = e / 16, c = e % 16;
        bt[c * 32 + k] = B[e];
    }
    __syncthreads();
    const int lo = lane & 15, kq = 8 * (lane >> 4);
    const f32x4 acc = mfma(frag<32, 1>(a, lo, kq), frag<32, 1>(bt, lo, kq), zero4());
#pragma unroll
    for (int i = 0; i < 4; ++i) D[(4 * (lane >> 4) + i) * 16 + lo] = acc[i];
}

hipError_t launch_mfma_probe(const uint16_t *A, const uint16_t *B, float *D, hipStream_t s)
{
    hipLaunchKernelGGL(mfma_probe_kernel, dim3(1), dim3(64), 0, s, A, B, D);
    return hipGetLastError();
}

}  // namespace pdc
