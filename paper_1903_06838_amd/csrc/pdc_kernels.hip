// HIP kernels for gfx950: detector correction, bank-median common mode, photon
// finding and hit-list compaction.
//
// Arithmetic contract (identical to the public header): binary32, one rounding
// per operation, no contraction (this file is built with -ffp-contract=off and
// the pragma below), no fast-math, subnormals preserved.
#include <hip/hip_runtime.h>
#include <math.h>

#include "pdc_device.h"
#include "pdc_internal.h"

#pragma clang fp contract(off)

namespace pdc {

__global__ void init_state_kernel(BatchState *st)
{
    if (threadIdx.x == 0) {
        st->cursor = 0;
        st->overflow = 0;
        st->fallback = 0;
        st->total = 0;
        st->n_fallback = 0;
    }
}

hipError_t launch_init_state(BatchState *state, hipStream_t s)
{
    hipLaunchKernelGGL(init_state_kernel, dim3(1), dim3(64), 0, s, state);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// v1 frame kernel: one workgroup per unit at a time (grid-stride over units).
//   load rows [r0-1, r1+1) of the tile (halo rows for the 3x3 window)
//   u = dark/gain corrected value -> LDS, row layout
//   per group of sort_rows rows: copy the banks into a sort buffer padded with
//   +inf, bitonic sort, subtract the lower median in place (LDS now holds v)
//   seeds, 3x3 local maximum, masked charge sum, photon count
//   ordered block compaction -> LDS hit list -> staging chunk
// ---------------------------------------------------------------------------
constexpr int kV1Threads = 256;

size_t frame_kernel_v1_lds_bytes(int strip_rows, int W, int nb, int sort_width, int sort_rows,
                                 uint32_t max_unit_hits)
{
    size_t rows = (size_t)strip_rows + 2;
    size_t floats = rows * W + (size_t)sort_rows * nb * sort_width;
    floats = (floats + 1) & ~(size_t)1;  // 8-byte align the hit list
    return floats * 4 + (size_t)max_unit_hits * 8;
}

template <bool KEEP>
__global__ void __launch_bounds__(kV1Threads) frame_kernel_v1(FrameKernelArgs A)
{
    extern __shared__ float lds[];
    __shared__ uint32_t s_wave[kV1Threads / 64];
    __shared__ unsigned long long s_photons;
    __shared__ uint64_t s_base;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int W = A.W, B = A.B, nb = A.nb, H = A.H, Pw = A.sort_width;
    const int rows_max = A.strip_rows + 2;
    float *s_v = lds;
    float *s_sort = s_v + (size_t)rows_max * W;
    size_t hit_off = (size_t)rows_max * W + (size_t)A.sort_rows * nb * Pw;
    hit_off = (hit_off + 1) & ~(size_t)1;
    uint2 *s_hits = reinterpret_cast<uint2 *>(lds + hit_off);
    const uint64_t npix = (uint64_t)A.T * H * W;
    const int kmed = (B - 1) / 2;

    uint64_t chunk_cur = 0, chunk_end = 0;  // staging chunk (used by thread 0)

    const uint64_t n_iter = A.unit_list ? A.n_list : A.n_units;
    for (uint64_t it = blockIdx.x; it < n_iter; it += gridDim.x) {
        const uint64_t unit = A.unit_list ? A.unit_list[it] : it;
        const uint64_t f = unit / (uint64_t)A.units_per_frame;
        const int su = (int)(unit - f * (uint64_t)A.units_per_frame);
        // rows r0..r1 (own) and lr0..lr1 (loaded) count from tile_base; rows
        // on either side of row gb belong to different tiles
        int t, r0, r1, lr0, lr1, gb = INT32_MAX;
        if (A.strips) {  // a persistent-kernel strip: global rows, may cross one tile edge
            const V2Strip S = A.strips[su];
            t = 0;
            r0 = S.g0;
            r1 = S.g1;
            lr0 = S.lg0;
            lr1 = S.lg1;
            gb = S.gb;
        } else {
            t = su / A.strips_per_tile;
            r0 = (su - t * A.strips_per_tile) * A.strip_rows;
            r1 = min(r0 + A.strip_rows, H);
            lr0 = max(r0 - 1, 0);
            lr1 = min(r1 + 1, H);
        }
        const int nrows = lr1 - lr0;
        const uint16_t *fr = A.frames + f * npix;
        const uint32_t tile_base = (uint32_t)t * (uint32_t)H * (uint32_t)W;

        // load + correct: u (auto-ranging: the reported range's planes, +inf
        // for an invalid code, counted on own rows)
        uint32_t ninv = 0;
        for (int i = tid; i < nrows * W; i += kV1Threads) {
            uint32_t p = tile_base + (uint32_t)lr0 * W + i;
            if (A.gain_mode) {
                bool bad;
                s_v[i] = dark_gain_ranged(fr[p], A.gain_mode, A.ped[p], A.k[p], A.ped, A.k, npix, p, bad);
                const int row = lr0 + i / W;
                if (bad && row >= r0 && row < r1) ++ninv;
            } else {
                s_v[i] = dark_gain(fr[p], A.ped[p], A.k[p]);
            }
        }
        if (ninv && !A.unit_list) atomicAdd(A.invalid + f, ninv);  // list mode: counted already
        __syncthreads();

        // thresholded-mean common mode, computed ahead: v = ((u - c1) - c2) - c3
        if (A.cm) {
            const float *cf = A.cm + f * (uint64_t)A.cm_regions * 3;
            for (int i = tid; i < nrows * W; i += kV1Threads) {
                const int row = i / W, c = i - row * W;
                const uint32_t grow = (uint32_t)t * H + lr0 + row;  // global row
                const uint32_t reg = A.cm_tile ? grow / (uint32_t)H : grow * (uint32_t)nb + c / B;
                const float *cv = cf + (uint64_t)reg * 3;
                const float u = s_v[i];
                s_v[i] = !(u < INFINITY) ? 0.0f : __fsub_rn(__fsub_rn(__fsub_rn(u, cv[0]), cv[1]), cv[2]);
            }
            __syncthreads();
        }
        // bank medians, a group of rows at a time; v = u - m in place
        for (int g0 = 0; g0 < (A.cm ? 0 : nrows); g0 += A.sort_rows) {
            const int gr = min(A.sort_rows, nrows - g0);
            const int total = gr * nb * Pw;
            for (int i = tid; i < total; i += kV1Threads) {
                int seg = i / Pw;
                int j = i - seg * Pw;
                int row = seg / nb;
                int b = seg - row * nb;
                s_sort[i] = j < B ? s_v[(g0 + row) * W + b * B + j] : INFINITY;
            }
            __syncthreads();
            for (int k = 2; k <= Pw; k <<= 1)
                for (int j = k >> 1; j > 0; j >>= 1) {
                    for (int q = tid; q < total / 2; q += kV1Threads) {
                        int i = (q / j) * 2 * j + (q % j);
                        int l = i + j;
                        bool asc = ((i & (Pw - 1)) & k) == 0;
                        float x = s_sort[i], y = s_sort[l];
                        if (asc ? (x > y) : (x < y)) {
                            s_sort[i] = y;
                            s_sort[l] = x;
                        }
                    }
                    __syncthreads();
                }
            for (int i = tid; i < gr * W; i += kV1Threads) {
                int row = i / W;
                int c = i - row * W;
                const float *seg = s_sort + (size_t)(row * nb + c / B) * Pw;
                float m;
                if (A.gain_mode) {
                    // the lower median of the valid values: invalid ones (+inf)
                    // sort last; an all-invalid bank has m = 0
                    int lo = 0, hi = B;
                    while (lo < hi) {
                        const int mid = (lo + hi) >> 1;
                        if (seg[mid] < INFINITY) lo = mid + 1;
                        else hi = mid;
                    }
                    m = lo > 0 ? seg[(lo - 1) / 2] : 0.0f;
                } else {
                    m = seg[kmed];
                }
                float u = s_v[(g0 + row) * W + c];
                if (!(u < INFINITY)) u = m;  // invalid: v = fl(m - m) = +0
                s_v[(g0 + row) * W + c] = __fsub_rn(u, m);
                // kept for patches: the own rows' medians, once per bank
                const int rl = lr0 + g0 + row;  // row in the tile
                if (A.meds && rl >= r0 && rl < r1 && c % B == 0)
                    A.meds[f * ((uint64_t)A.T * H * nb) + ((uint64_t)t * H + rl) * nb + c / B] = m;
            }
            __syncthreads();
        }
        if (tid == 0) s_photons = 0;

        if (KEEP) {
            const int off = (r0 - lr0) * W;
            float *dst = A.corrected + f * npix + tile_base + (uint64_t)r0 * W;
            for (int i = tid; i < (r1 - r0) * W; i += kV1Threads) dst[i] = s_v[off + i];
        }

        // photon finding with ordered (raster) compaction
        const int npx = (r1 - r0) * W;
        uint32_t count = 0;
        unsigned long long my_ph = 0;
        for (int base = 0; base < npx; base += kV1Threads) {
            int i = base + tid;
            bool hit = false;
            uint32_t pix = 0;
            float qsum = 0.0f;
            if (i < npx) {
                int r = r0 + i / W;
                int c = i - (i / W) * W;
                float vp = s_v[(r - lr0) * W + c];
                if (vp > A.t_seed) {
                    uint32_t p = tile_base + (uint32_t)r * W + c;
                    bool is_max = true;
                    for (int dr = -1; dr <= 1; ++dr)
                        for (int dc = -1; dc <= 1; ++dc) {
                            if (dr == 0 && dc == 0) continue;
                            int rr = r + dr, cc = c + dc;
                            if (rr < lr0 || rr >= lr1 || cc < 0 || cc >= W || ((rr >= gb) != (r >= gb))) continue;
                            float vq = s_v[(rr - lr0) * W + cc];
                            uint32_t q = tile_base + (uint32_t)rr * W + cc;
                            if (!(vp > vq || (vp == vq && p < q))) is_max = false;
                        }
                    if (is_max) {
                        for (int dr = -1; dr <= 1; ++dr)
                            for (int dc = -1; dc <= 1; ++dc) {
                                int rr = r + dr, cc = c + dc;
                                if (rr < lr0 || rr >= lr1 || cc < 0 || cc >= W || ((rr >= gb) != (r >= gb)))
                                    continue;
                                float vj = s_v[(rr - lr0) * W + cc];
                                qsum = __fadd_rn(qsum, vj > A.t_nb ? vj : 0.0f);
                            }
                        hit = true;
                        pix = p;
                        my_ph += photon_count(qsum, A.photon_adu);
                    }
                }
            }
            unsigned long long ballot = __ballot(hit);
            uint32_t pre = __popcll(ballot & ((1ull << lane) - 1ull));
            if (lane == 0) s_wave[wave] = __popcll(ballot);
            __syncthreads();
            uint32_t woff = 0, round_total = 0;
            for (int w = 0; w < kV1Threads / 64; ++w) {
                uint32_t cw = s_wave[w];
                if (w < wave) woff += cw;
                round_total += cw;
            }
            if (hit) s_hits[count + woff + pre] = make_uint2(pix, __float_as_uint(qsum));
            count += round_total;
            __syncthreads();
        }
        if (my_ph) atomicAdd(&s_photons, my_ph);
        __syncthreads();

        if (tid == 0) {
            uint64_t base = chunk_cur;
            if (count > 0) {
                if (chunk_cur + count > chunk_end) {
                    uint64_t sz = count > kChunkHits ? (uint64_t)count : kChunkHits;
                    chunk_cur = atomicAdd(&A.state->cursor, (unsigned long long)sz);
                    chunk_end = chunk_cur + sz;
                }
                if (chunk_cur + count <= A.pool_cap) {
                    base = chunk_cur;
                    chunk_cur += count;
                } else {
                    base = kNoBase;
                    atomicOr(&A.state->overflow, 1u);
                }
            }
            A.unit_base[unit] = base;
            A.unit_count[unit] = count;
            A.unit_photons[unit] = s_photons;
            s_base = base;
        }
        __syncthreads();
        const uint64_t base = s_base;
        if (base != kNoBase)
            for (uint32_t i = tid; i < count; i += kV1Threads) A.pool[base + i] = s_hits[i];
        __syncthreads();
    }
}

hipError_t launch_frame_kernel_v1(const FrameKernelArgs &a, uint32_t grid, size_t lds_bytes,
                                  bool keep_corrected, hipStream_t s)
{
    auto k = keep_corrected ? frame_kernel_v1<true> : frame_kernel_v1<false>;
    if (lds_bytes > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k, dim3(grid), dim3(kV1Threads), lds_bytes, s, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Block-wide exclusive scan helpers (256 threads = 4 waves of 64).
// ---------------------------------------------------------------------------
constexpr int kScanThreads = 256;

template <typename T>
__device__ __forceinline__ T wave_inclusive_scan(T x)
{
    const int lane = threadIdx.x & 63;
    for (int d = 1; d < 64; d <<= 1) {
        T y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    return x;
}

// Returns the exclusive prefix of x over the block; *block_total gets the sum.
template <typename T>
__device__ __forceinline__ T block_exclusive_scan(T x, T *s_tmp, T *block_total)
{
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    T inc = wave_inclusive_scan(x);
    if (lane == 63) s_tmp[wave] = inc;
    __syncthreads();
    T off = 0, tot = 0;
    for (int w = 0; w < kScanThreads / 64; ++w) {
        T v = s_tmp[w];
        if (w < wave) off += v;
        tot += v;
    }
    __syncthreads();
    *block_total = tot;
    return off + inc - x;
}

__global__ void __launch_bounds__(kScanThreads)
frame_sums_kernel(const uint32_t *unit_count, const unsigned long long *unit_photons,
                  uint64_t n_frames, int32_t upf, uint32_t *unit_local, uint32_t *frame_hits,
                  unsigned long long *frame_photons)
{
    __shared__ uint32_t s_tmp[kScanThreads / 64];
    __shared__ unsigned long long s_ph;
    const uint64_t f = blockIdx.x;
    if (f >= n_frames) return;
    if (threadIdx.x == 0) s_ph = 0;
    __syncthreads();
    const uint64_t u0 = f * (uint64_t)upf;
    uint32_t carry = 0;
    unsigned long long ph = 0;
    for (int base = 0; base < upf; base += kScanThreads) {
        int i = base + threadIdx.x;
        uint32_t c = i < upf ? unit_count[u0 + i] : 0u;
        if (i < upf) ph += unit_photons[u0 + i];
        uint32_t tot;
        uint32_t ex = block_exclusive_scan<uint32_t>(c, s_tmp, &tot);
        if (i < upf) unit_local[u0 + i] = carry + ex;
        carry += tot;
    }
    if (ph) atomicAdd(&s_ph, ph);
    __syncthreads();
    if (threadIdx.x == 0) {
        frame_hits[f] = carry;
        frame_photons[f] = s_ph;
    }
}

hipError_t launch_frame_sums(const uint32_t *unit_count, const unsigned long long *unit_photons,
                             uint64_t n_frames, int32_t units_per_frame, uint32_t *unit_local,
                             uint32_t *frame_hits, unsigned long long *frame_photons, hipStream_t s)
{
    if (n_frames == 0) return hipSuccess;
    hipLaunchKernelGGL(frame_sums_kernel, dim3((uint32_t)n_frames), dim3(kScanThreads), 0, s,
                       unit_count, unit_photons, n_frames, units_per_frame, unit_local,
                       frame_hits, frame_photons);
    return hipGetLastError();
}

__global__ void __launch_bounds__(kScanThreads)
frame_scan_kernel(const uint32_t *frame_hits, uint64_t n_frames, unsigned long long *frame_offset,
                  BatchState *st)
{
    __shared__ unsigned long long s_tmp[kScanThreads / 64];
    unsigned long long carry = 0;
    for (uint64_t base = 0; base < n_frames; base += kScanThreads) {
        uint64_t i = base + threadIdx.x;
        unsigned long long c = i < n_frames ? frame_hits[i] : 0ull;
        unsigned long long tot;
        unsigned long long ex = block_exclusive_scan<unsigned long long>(c, s_tmp, &tot);
        if (i < n_frames) frame_offset[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) {
        frame_offset[n_frames] = carry;
        st->total = carry;
    }
}

hipError_t launch_frame_scan(const uint32_t *frame_hits, uint64_t n_frames,
                             unsigned long long *frame_offset, BatchState *state, hipStream_t s)
{
    hipLaunchKernelGGL(frame_scan_kernel, dim3(1), dim3(kScanThreads), 0, s, frame_hits, n_frames,
                       frame_offset, state);
    return hipGetLastError();
}

// Each wave copies the staged runs of kScatterUnits consecutive units into
// the raster-order list.  A unit's run is short (about a hundred hits at
// occupancy 0.01), so one unit per wave left each wave two dependent memory
// round trips for little data; here lanes 0..kScatterUnits-1 read the units'
// counts, bases and destinations at once, and the first two 64-hit rows of
// every run are loaded before any is stored, so up to 2 kScatterUnits loads
// per lane are in flight.  Longer runs finish row by row.  Units whose run
// was not staged (kNoBase) or would end past hits_cap (only after a staging
// overflow; the batch is then recomputed) copy nothing.
constexpr int kScatterUnits = 4;

__global__ void __launch_bounds__(256)
scatter_kernel(const uint32_t *unit_count, const uint64_t *unit_base, const uint32_t *unit_local,
               const unsigned long long *frame_offset, const uint2 *pool, uint64_t n_units,
               int32_t upf, uint2 *hits, uint64_t hits_cap)
{
    constexpr int U = kScatterUnits;
    const uint64_t u0 = ((uint64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * U;
    const int lane = threadIdx.x & 63;
    if (u0 >= n_units) return;
    uint32_t c = 0;
    uint64_t b = 0, dst = 0;
    if (lane < U && u0 + lane < n_units) {
        const uint64_t unit = u0 + lane;
        c = unit_count[unit];
        b = unit_base[unit];
        dst = frame_offset[unit / (uint64_t)upf] + unit_local[unit];
        if (b == kNoBase || dst + c > hits_cap) c = 0;
    }
    uint32_t cu[U];
    uint64_t bu[U], du[U];
#pragma unroll
    for (int k = 0; k < U; ++k) {
        cu[k] = (uint32_t)__builtin_amdgcn_readlane((int)c, k);
        bu[k] = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(b >> 32), k) << 32) |
                (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, k);
        du[k] = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(dst >> 32), k) << 32) |
                (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)dst, k);
    }
    uint2 v[U][2];
#pragma unroll
    for (int k = 0; k < U; ++k)
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const uint32_t i = (uint32_t)lane + 64u * r;
            if (i < cu[k]) v[k][r] = pool[bu[k] + i];
        }
#pragma unroll
    for (int k = 0; k < U; ++k)
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const uint32_t i = (uint32_t)lane + 64u * r;
            if (i < cu[k]) hits[du[k] + i] = v[k][r];
        }
#pragma unroll
    for (int k = 0; k < U; ++k)
        for (uint32_t i = (uint32_t)lane + 128u; i < cu[k]; i += 64) hits[du[k] + i] = pool[bu[k] + i];
}

hipError_t launch_scatter(const uint32_t *unit_count, const uint64_t *unit_base,
                          const uint32_t *unit_local, const unsigned long long *frame_offset,
                          const uint2 *pool, uint64_t n_units, int32_t units_per_frame,
                          uint2 *hits, uint64_t hits_cap, hipStream_t s)
{
    if (n_units == 0) return hipSuccess;
    const uint64_t per_block = 4 * (uint64_t)kScatterUnits;  // 4 waves
    const uint64_t blocks = (n_units + per_block - 1) / per_block;
    hipLaunchKernelGGL(scatter_kernel, dim3((uint32_t)blocks), dim3(256), 0, s, unit_count,
                       unit_base, unit_local, frame_offset, pool, n_units, units_per_frame, hits,
                       hits_cap);
    return hipGetLastError();
}

// Like scatter_kernel, but each hit goes straight to its 16-byte record
// (frame, pixel, charge, photon count) at its raster position; records past
// out_cap are not written (the caller's destination keeps the first ones).
__global__ void __launch_bounds__(256)
scatter_records_kernel(const uint32_t *unit_count, const uint64_t *unit_base, const uint32_t *unit_local,
                       const unsigned long long *frame_offset, const uint2 *pool, uint64_t n_units, int32_t upf,
                       float photon_adu, HitRecord *out, uint64_t out_cap)
{
    const uint64_t unit = (uint64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (unit >= n_units) return;
    const uint32_t c = unit_count[unit];
    const uint64_t b = unit_base[unit];
    if (c == 0 || b == kNoBase) return;
    const uint64_t f = unit / (uint64_t)upf;
    const uint64_t dst = frame_offset[f] + unit_local[unit];
    for (uint32_t i = lane; i < c && dst + i < out_cap; i += 64) {
        const uint2 h = pool[b + i];
        const float q = __uint_as_float(h.y);
        HitRecord r;
        r.frame = (uint32_t)f;
        r.pixel = h.x;
        r.charge = q;
        r.nphot = photon_count(q, photon_adu);
        out[dst + i] = r;
    }
}

hipError_t launch_scatter_records(const uint32_t *unit_count, const uint64_t *unit_base,
                                  const uint32_t *unit_local, const unsigned long long *frame_offset,
                                  const uint2 *pool, uint64_t n_units, int32_t units_per_frame, float photon_adu,
                                  HitRecord *out, uint64_t out_cap, hipStream_t s)
{
    if (n_units == 0) return hipSuccess;
    uint64_t blocks = (n_units + 3) / 4;
    hipLaunchKernelGGL(scatter_records_kernel, dim3((uint32_t)blocks), dim3(256), 0, s, unit_count, unit_base,
                       unit_local, frame_offset, pool, n_units, units_per_frame, photon_adu, out, out_cap);
    return hipGetLastError();
}

__global__ void __launch_bounds__(256)
format_hits_kernel(const uint2 *hits, const unsigned long long *frame_offset, uint64_t n_frames,
                   uint64_t first, uint64_t n, float photon_adu, HitRecord *out)
{
    uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    uint64_t g = first + i;
    // largest f with frame_offset[f] <= g
    uint64_t lo = 0, hi = n_frames;  // frame_offset[hi] = total > g
    while (hi - lo > 1) {
        uint64_t mid = (lo + hi) / 2;
        if (frame_offset[mid] <= g) lo = mid;
        else hi = mid;
    }
    uint2 h = hits[g];
    float q = __uint_as_float(h.y);
    HitRecord r;
    r.frame = (uint32_t)lo;
    r.pixel = h.x;
    r.charge = q;
    r.nphot = photon_count(q, photon_adu);
    out[i] = r;
}

hipError_t launch_format_hits(const uint2 *hits, const unsigned long long *frame_offset,
                              uint64_t n_frames, uint64_t first, uint64_t n, float photon_adu,
                              HitRecord *out, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    uint64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(format_hits_kernel, dim3((uint32_t)blocks), dim3(256), 0, s, hits,
                       frame_offset, n_frames, first, n, photon_adu, out);
    return hipGetLastError();
}

}  // namespace pdc
