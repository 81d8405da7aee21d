// Summaries (Summarization section; Fig. g spectra; Dark and Gain section):
// accumulated photon-counting maps, charge spectra of hits (optionally split
// by the number of pixels the charge was summed over), histograms of Frames2,
// and exact per-pixel sums over dark frames for pedestal and noise.
//
// All counts are integers added with device atomics, so every result is
// independent of the order in which threads run.  Bins follow one rule on
// every path (x a binary32 value, s = nbins / (hi - lo) formed in binary32):
//   bin 0            if not (x >= lo)
//   1 + floor(t)     if t < nbins, with t = fl(fl(x - lo) * s)
//   nbins + 1        otherwise.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pdc_device.h"
#include "pdc_summary.h"

#pragma clang fp contract(off)

namespace pdc {

namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ uint32_t hist_bin(float x, float lo, float s, uint32_t nbins)
{
    if (!(x >= lo)) return 0;
    const float t = __fmul_rn(__fsub_rn(x, lo), s);
    if (!(t < (float)nbins)) return nbins + 1;
    return 1u + (uint32_t)t;  // t in [0, nbins): truncation is floor
}

__global__ void fill_u32_kernel(uint32_t *p, uint64_t n)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

__global__ void fill_u64_kernel(unsigned long long *p, uint64_t n)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

// Bins held in LDS by one workgroup before they are added to memory; larger
// histograms go straight to device memory.
__device__ __forceinline__ void lds_clear(uint32_t *h, uint32_t n)
{
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) h[i] = 0u;
}
__device__ __forceinline__ void lds_flush(const uint32_t *h, uint32_t n, uint32_t *dst)
{
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
        const uint32_t c = h[i];
        if (c) atomicAdd(dst + i, c);
    }
}

// Frame of hit i: the largest f < n_frames with frame_offset[f] <= i, given
// f0 <= that frame.  Gallops forward from f0, then bisects, so hits visited in
// increasing order cost O(log(frames skipped)) loads each.
__device__ __forceinline__ uint64_t frame_from(const unsigned long long *frame_offset, uint64_t n_frames, uint64_t i,
                                               uint64_t f0)
{
    uint64_t lo = f0, step = 1;
    uint64_t hi = n_frames;  // frame_offset[n_frames] = total > i is never read
    while (lo + step < n_frames) {
        if (frame_offset[lo + step] <= i) {
            lo += step;
            step *= 2;
        } else {
            hi = lo + step;
            break;
        }
    }
    while (hi - lo > 1) {
        const uint64_t mid = (lo + hi) / 2;
        if (frame_offset[mid] <= i) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Each workgroup takes a contiguous range of hits, 256 consecutive hits per
// step (coalesced), so each thread meets its hits in increasing order.
// count_map[pixel] += nphot;
// spectrum[bin(charge)] += 1; size_spectra[(size - 1) * (nbins + 2) +
// bin(charge)] += 1 where size counts the pixels of the hit's in-tile 3x3
// window whose Frames2 value is above t_nb.
template <bool MAP, bool SPEC, bool SIZES, bool PRIV>
__global__ __launch_bounds__(kThreads) void accumulate_hits_kernel(AccumulateArgs a)
{
    extern __shared__ uint32_t s_h[];
    const uint32_t nb2 = a.nbins + 2u;
    uint32_t *h_spec = s_h;
    uint32_t *h_size = s_h + (SPEC ? nb2 : 0u);
    if (PRIV) {
        lds_clear(s_h, (SPEC ? nb2 : 0u) + (SIZES ? 9u * nb2 : 0u));
        __syncthreads();
    }
    const uint64_t per = ((a.n + gridDim.x - 1) / gridDim.x + blockDim.x - 1) / blockDim.x * blockDim.x;
    const uint64_t i_end = (blockIdx.x + 1) * per < a.n ? (blockIdx.x + 1) * per : a.n;
    uint64_t f = 0;
    for (uint64_t i = blockIdx.x * per + threadIdx.x; i < i_end; i += blockDim.x) {
        const uint2 hit = a.hits[i];
        const float q = __uint_as_float(hit.y);
        if (MAP) {
            const uint32_t k = photon_count(q, a.photon_adu);
            if (k) atomicAdd(a.count_map + hit.x, k);
        }
        if (!SPEC && !SIZES) continue;
        const uint32_t b = hist_bin(q, a.lo, a.scale, a.nbins);
        if (SPEC) {
            if (PRIV) atomicAdd(h_spec + b, 1u);
            else atomicAdd(a.spectrum + b, 1u);
        }
        if (SIZES) {
            f = frame_from(a.frame_offset, a.n_frames, i, f);
            const uint32_t W = (uint32_t)a.W, H = (uint32_t)a.H;
            const int c = (int)(hit.x % W);
            const uint32_t rt = hit.x / W;
            const int t = (int)(rt / H), r = (int)(rt - (uint32_t)t * H);
            const float *fr = a.corrected + (f * (uint64_t)a.T + (uint64_t)t) * (uint64_t)H * W;
            uint32_t size = 0;
#pragma unroll
            for (int dr = -1; dr <= 1; ++dr)
#pragma unroll
                for (int dc = -1; dc <= 1; ++dc) {
                    const int rr = r + dr, cc = c + dc;
                    if (rr >= 0 && rr < a.H && cc >= 0 && cc < a.W && fr[(uint64_t)rr * W + cc] > a.t_nb) ++size;
                }
            // the hit pixel itself is above T_seed >= T_nb, so size >= 1
            if (size == 0) continue;
            const uint32_t idx = (size - 1u) * nb2 + b;
            if (PRIV) atomicAdd(h_size + idx, 1u);
            else atomicAdd(a.size_spectra + idx, 1u);
        }
    }
    if (PRIV) {
        __syncthreads();
        if (SPEC) lds_flush(h_spec, nb2, a.spectrum);
        if (SIZES) lds_flush(h_size, 9u * nb2, a.size_spectra);
    }
}

// Histogram of n binary32 values (Frames2), 4 per thread per step.
template <bool PRIV>
__global__ __launch_bounds__(kThreads) void histogram_kernel(const float *x, uint64_t n, float lo, float s,
                                                             uint32_t nbins, uint32_t *hist)
{
    extern __shared__ uint32_t s_h[];
    uint32_t *h = PRIV ? s_h : hist;
    if (PRIV) {
        lds_clear(s_h, nbins + 2u);
        __syncthreads();
    }
    const uint64_t n4 = n / 4;
    const float4 *x4 = reinterpret_cast<const float4 *>(x);
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride) {
        const float4 v = x4[i];
        atomicAdd(h + hist_bin(v.x, lo, s, nbins), 1u);
        atomicAdd(h + hist_bin(v.y, lo, s, nbins), 1u);
        atomicAdd(h + hist_bin(v.z, lo, s, nbins), 1u);
        atomicAdd(h + hist_bin(v.w, lo, s, nbins), 1u);
    }
    if (blockIdx.x == 0)
        for (uint64_t i = 4 * n4 + threadIdx.x; i < n; i += blockDim.x) atomicAdd(h + hist_bin(x[i], lo, s, nbins), 1u);
    if (PRIV) {
        __syncthreads();
        lds_flush(s_h, nbins + 2u, hist);
    }
}

// Exact sums over dark frames: s1[p] += sum adc, s2[p] += sum adc^2 with
// adc = raw & 0x3FFF, over frames [f0, f0 + chunk) of blockIdx.y's chunk.
// VEC pixels per thread (VEC = 4 needs pixels % 4 == 0 for aligned loads).
template <int VEC>
__global__ __launch_bounds__(kThreads) void dark_sums_kernel(const uint16_t *d, uint64_t n_frames, uint64_t px,
                                                             uint64_t chunk, unsigned long long *s1,
                                                             unsigned long long *s2)
{
    const uint64_t p0 = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) * VEC;
    if (p0 >= px) return;
    const uint64_t f0 = (uint64_t)blockIdx.y * chunk;
    const uint64_t f1 = f0 + chunk < n_frames ? f0 + chunk : n_frames;
    uint32_t a1[VEC];
    uint64_t a2[VEC];
#pragma unroll
    for (int j = 0; j < VEC; ++j) {
        a1[j] = 0u;
        a2[j] = 0ull;
    }
    for (uint64_t f = f0; f < f1; ++f) {
        const uint16_t *row = d + f * px + p0;
        uint32_t v[VEC];
        if constexpr (VEC == 4) {
            const ushort4 w = *reinterpret_cast<const ushort4 *>(row);
            v[0] = w.x;
            v[1] = w.y;
            v[2] = w.z;
            v[3] = w.w;
        } else {
#pragma unroll
            for (int j = 0; j < VEC; ++j) v[j] = row[j];
        }
#pragma unroll
        for (int j = 0; j < VEC; ++j) {
            const uint32_t adc = v[j] & 0x3FFFu;
            a1[j] += adc;                      // chunk <= 2^18: no wrap
            a2[j] += (uint64_t)(adc * adc);    // adc^2 < 2^28
        }
    }
#pragma unroll
    for (int j = 0; j < VEC; ++j) {
        atomicAdd(s1 + p0 + j, (unsigned long long)a1[j]);
        atomicAdd(s2 + p0 + j, (unsigned long long)a2[j]);
    }
}

uint32_t stride_grid(uint64_t items, uint32_t cap)
{
    const uint64_t g = (items + kThreads - 1) / kThreads;
    return (uint32_t)(g < 1 ? 1 : (g > cap ? cap : g));
}

}  // namespace

// Plain streaming read of n16 16-byte words: four independent loads per
// thread and step, grid-stride; each wave folds what it read into one XOR and
// adds it to *out with one atomic, so no load can be dropped.
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint32_t fold4(u32x4 a) { return (a.x ^ a.y) ^ (a.z ^ a.w); }

__global__ void __launch_bounds__(kThreads) stream_read_kernel(const u32x4 *src, uint64_t n16, uint32_t *out)
{
    const uint64_t stride = (uint64_t)gridDim.x * kThreads;
    uint64_t i = (uint64_t)blockIdx.x * kThreads + threadIdx.x;
    uint32_t acc = 0;
    for (; i + 3 * stride < n16; i += 4 * stride) {
        const u32x4 a = __builtin_nontemporal_load(src + i);
        const u32x4 b = __builtin_nontemporal_load(src + i + stride);
        const u32x4 c = __builtin_nontemporal_load(src + i + 2 * stride);
        const u32x4 d = __builtin_nontemporal_load(src + i + 3 * stride);
        acc ^= (fold4(a) ^ fold4(b)) ^ (fold4(c) ^ fold4(d));
    }
    for (; i < n16; i += stride) acc ^= fold4(__builtin_nontemporal_load(src + i));
    for (int o = 32; o > 0; o >>= 1) acc ^= (uint32_t)__shfl_xor((int)acc, o);
    if ((threadIdx.x & 63) == 0) atomicXor(out, acc);
}

hipError_t launch_stream_read(const void *src, uint64_t bytes, uint32_t *out, uint32_t n_cu, hipStream_t s)
{
    const uint64_t n16 = bytes / 16;
    if (n16 == 0) return hipSuccess;
    const uint32_t grid = stride_grid(n16, 16u * (n_cu ? n_cu : 256u));
    hipLaunchKernelGGL(stream_read_kernel, dim3(grid), dim3(kThreads), 0, s, reinterpret_cast<const u32x4 *>(src),
                       n16, out);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t *p, uint64_t n, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(fill_u32_kernel, dim3((uint32_t)((n + kThreads - 1) / kThreads)), dim3(kThreads), 0, s, p, n);
    return hipGetLastError();
}

bool accumulate_uses_lds(const AccumulateArgs &a)
{
    const uint64_t bins = (a.spectrum ? a.nbins + 2ull : 0ull) + (a.size_spectra ? 9ull * (a.nbins + 2ull) : 0ull);
    return bins > 0 && bins <= kLdsBins;
}

hipError_t launch_accumulate_hits(const AccumulateArgs &a, uint32_t max_grid, hipStream_t s)
{
    if (a.n == 0) return hipSuccess;
    const bool map = a.count_map != nullptr, spec = a.spectrum != nullptr, sizes = a.size_spectra != nullptr;
    const bool priv = accumulate_uses_lds(a);
    const size_t lds = priv ? ((spec ? a.nbins + 2u : 0u) + (sizes ? 9u * (a.nbins + 2u) : 0u)) * sizeof(uint32_t) : 0;
    const uint32_t grid = stride_grid(a.n, max_grid);
#define PDC_ACC(M, S, Z, P) \
    hipLaunchKernelGGL((accumulate_hits_kernel<M, S, Z, P>), dim3(grid), dim3(kThreads), lds, s, a)
    const int key = (map ? 8 : 0) | (spec ? 4 : 0) | (sizes ? 2 : 0) | (priv ? 1 : 0);
    switch (key) {
    case 8: PDC_ACC(true, false, false, false); break;
    case 12: PDC_ACC(true, true, false, false); break;
    case 13: PDC_ACC(true, true, false, true); break;
    case 10: PDC_ACC(true, false, true, false); break;
    case 11: PDC_ACC(true, false, true, true); break;
    case 14: PDC_ACC(true, true, true, false); break;
    case 15: PDC_ACC(true, true, true, true); break;
    case 4: PDC_ACC(false, true, false, false); break;
    case 5: PDC_ACC(false, true, false, true); break;
    case 2: PDC_ACC(false, false, true, false); break;
    case 3: PDC_ACC(false, false, true, true); break;
    case 6: PDC_ACC(false, true, true, false); break;
    case 7: PDC_ACC(false, true, true, true); break;
    default: return hipSuccess;  // nothing requested
    }
#undef PDC_ACC
    return hipGetLastError();
}

hipError_t launch_histogram(const float *x, uint64_t n, float lo, float scale, uint32_t nbins, uint32_t *hist,
                            uint32_t max_grid, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    const uint32_t grid = stride_grid(n / 4 + 1, max_grid);
    if (nbins + 2ull <= kLdsBins)
        hipLaunchKernelGGL(histogram_kernel<true>, dim3(grid), dim3(kThreads), (nbins + 2) * sizeof(uint32_t), s, x, n,
                           lo, scale, nbins, hist);
    else
        hipLaunchKernelGGL(histogram_kernel<false>, dim3(grid), dim3(kThreads), 0, s, x, n, lo, scale, nbins, hist);
    return hipGetLastError();
}

hipError_t launch_dark_sums(const uint16_t *d, uint64_t n_frames, uint64_t px, unsigned long long *s1,
                            unsigned long long *s2, uint32_t n_cu, hipStream_t s)
{
    if (px == 0) return hipSuccess;
    hipLaunchKernelGGL(fill_u64_kernel, dim3((uint32_t)((px + kThreads - 1) / kThreads)), dim3(kThreads), 0, s, s1, px);
    hipLaunchKernelGGL(fill_u64_kernel, dim3((uint32_t)((px + kThreads - 1) / kThreads)), dim3(kThreads), 0, s, s2, px);
    if (n_frames == 0) return hipGetLastError();
    const int vec = (px % 4 == 0) ? 4 : 1;
    const uint64_t bx = (px / vec + kThreads - 1) / kThreads;
    // enough workgroups to fill the chip: split the frames into chunks
    const uint64_t want = 8ull * n_cu;
    uint64_t chunks = (want + bx - 1) / bx;
    if (chunks > n_frames) chunks = n_frames;
    uint64_t chunk = (n_frames + chunks - 1) / chunks;
    if (chunk > kDarkChunkMax) chunk = kDarkChunkMax;
    chunks = (n_frames + chunk - 1) / chunk;
    if (bx > 0x7FFFFFFFull || chunks > 65535ull) return hipErrorInvalidValue;
    if (vec == 4)
        hipLaunchKernelGGL(dark_sums_kernel<4>, dim3((uint32_t)bx, (uint32_t)chunks), dim3(kThreads), 0, s, d, n_frames,
                           px, chunk, s1, s2);
    else
        hipLaunchKernelGGL(dark_sums_kernel<1>, dim3((uint32_t)bx, (uint32_t)chunks), dim3(kThreads), 0, s, d, n_frames,
                           px, chunk, s1, s2);
    return hipGetLastError();
}

}  // namespace pdc
