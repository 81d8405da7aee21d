// Persistent frame kernel for gfx950.
//
// One workgroup (8 waves) owns a strip of rows of one tile for a range of
// frames.  The strip's dark and 1/gain planes are loaded once into registers
// and stay there for every frame; only the 2-byte raw words stream from HBM.
// Per frame:
//   phase 1 (each wave, its own bank-rows): load raw words (prefetched one
//     frame ahead), correct them (Fig. b), write u to LDS, find each bank's
//     lower median exactly by ballot-counted pivot passes (common mode,
//     Fig. c), derive the seed threshold, and append seed pixels to a
//     workgroup list;
//   phase 2 (all waves, over the pooled seeds): 3x3 local maximum with the
//     raster tie-break, masked 3x3 charge sum, photon count (Fig. e and the
//     charge summing section); hits mark a per-bank-row column bitmap;
//   phase 3 (wave 0): prefix over bank-rows, staging chunk claim;
//   phase 4 (all waves): each hit's raster position = bank-row prefix +
//     number of hits left of it in its bank-row (bitmap popcount).
//
// Lane layout: a bank-row (B pixels of one row) is held by one wave as NQ
// pair-slots; lane l of pair-slot q holds columns 128q + 2l and 128q + 2l + 1
// of the bank (value-slots 2q and 2q+1).  Absent pixels hold +inf.
#include <hip/hip_runtime.h>
#include <math.h>

#include "pdc_device.h"
#include "pdc_internal.h"

#pragma clang fp contract(off)

namespace pdc {

constexpr int kV2Waves = 16;
constexpr int kV2Threads = kV2Waves * 64;

__device__ __forceinline__ uint32_t popc64(uint64_t m) { return (uint32_t)__popcll(m); }

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

__device__ __forceinline__ float uniform_f(float x)
{
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
}

// Sum over the 64 lanes of a wave, wave-uniform result (DPP reduction; the
// summation order is fixed but it only feeds a search heuristic).
__device__ __forceinline__ float wave_sum(float x)
{
    int v = __float_as_int(x);
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, false));  // quad_perm 1,0,3,2
    v = __float_as_int(x);
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, v, 0x4E, 0xF, 0xF, false));  // quad_perm 2,3,0,1
    v = __float_as_int(x);
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, v, 0x141, 0xF, 0xF, false)); // row_half_mirror
    v = __float_as_int(x);
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, v, 0x140, 0xF, 0xF, false)); // row_mirror
    v = __float_as_int(x);
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, v, 0x142, 0xA, 0xF, false)); // row_bcast15
    v = __float_as_int(x);
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, v, 0x143, 0xC, 0xF, false)); // row_bcast31
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 63));
}

// Smallest binary32 value th such that fl(th - m) > t (fl(x - m) is
// monotone in x, so fl(u - m) > t  <=>  u >= th).  Wave-uniform.
__device__ __forceinline__ float seed_threshold(float m, float t)
{
    float th = uniform_f(__fadd_rn(m, t));
    for (int i = 0; i < 64 && !(__fsub_rn(th, m) > t); ++i) th = uniform_f(key2f(f2key(th) + 1));
    for (int i = 0; i < 64; ++i) {
        float d = uniform_f(key2f(f2key(th) - 1));
        if (__fsub_rn(d, m) > t) th = d;
        else break;
    }
    return th;
}

template <int NV>
__device__ __forceinline__ int count_below(const float (&x)[NV], float p)
{
    int c = 0;
#pragma unroll
    for (int v = 0; v < NV; ++v) c += popc64(ballot(x[v] < p));
    return c;
}

// Wave-uniform minimum (max_mode false) or maximum of the lanes' values.
__device__ __forceinline__ float wave_minmax(float x, bool max_mode)
{
    int v = __float_as_int(x);
#define PDC_MM(ctrl, rm)                                                                          \
    {                                                                                             \
        float o = __int_as_float(__builtin_amdgcn_update_dpp(v, v, ctrl, rm, 0xF, false));        \
        x = max_mode ? fmaxf(x, o) : fminf(x, o);                                                 \
        v = __float_as_int(x);                                                                    \
    }
    PDC_MM(0xB1, 0xF)
    PDC_MM(0x4E, 0xF)
    PDC_MM(0x141, 0xF)
    PDC_MM(0x140, 0xF)
    PDC_MM(0x142, 0xA)
    PDC_MM(0x143, 0xC)
#undef PDC_MM
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 63));
}

// Exact element of rank k (0-based, ascending) among the n_valid finite lane
// values of x (absent values are +inf).  Bracketing search on counts:
// count(x < lo) <= k < count(x < hi) holds throughout.  The first pass tests
// est - w and est + w together (widening until they bracket); later passes
// interpolate the pivot from the bracket counts, bisecting in key space when
// the interpolated pivot coincides with a bound or the bracket stops halving.
// Once at most two values remain in [lo, hi), the answer is the smallest value
// >= lo (if it has rank k) or the largest value < hi.  All state is
// wave-uniform.
template <int NV>
__device__ float bank_median(const float (&x)[NV], int n_valid, int k, float est, float w)
{
    float lo = uniform_f(est - w), hi = uniform_f(est + w);
    int clo = count_below<NV>(x, lo), chi = count_below<NV>(x, hi);
    for (int i = 0; i < 40 && !(clo <= k && k < chi); ++i) {
        w = w + w;
        if (clo > k) {
            hi = lo;
            chi = clo;
            lo = uniform_f(i < 38 ? est - w : -INFINITY);
            clo = i < 38 ? count_below<NV>(x, lo) : 0;
        } else {
            lo = hi;
            clo = chi;
            hi = uniform_f(i < 38 ? est + w : INFINITY);
            chi = i < 38 ? count_below<NV>(x, hi) : n_valid;
        }
    }
    int n = chi - clo;
    int last_n = 4 * n_valid;
    for (int it = 0; it < 200 && n > 2; ++it) {
        // interpolated pivot: lo + (hi - lo) * (k - clo + 1/2) / n lies in [lo, hi]
        float q = lo + (hi - lo) * (((float)(k - clo) + 0.5f) * __builtin_amdgcn_rcpf((float)n));
        q = uniform_f(q);
        const int32_t qb = __float_as_int(q);
        if (2 * n > last_n || qb == __float_as_int(lo) || qb == __float_as_int(hi) ||
            !(lo > -INFINITY && hi < INFINITY)) {
            const int32_t klo = f2key(lo), khi = f2key(hi);
            if ((int64_t)khi - (int64_t)klo <= 1) return lo;  // [lo, hi) holds only the value lo
            q = key2f((int32_t)(((int64_t)klo + (int64_t)khi) >> 1));
            last_n = 4 * n_valid;  // the next step interpolates again
        } else {
            last_n = n;
        }
        const int c = count_below<NV>(x, q);
        if (c <= k) {
            lo = q;
            clo = c;
        } else {
            hi = q;
            chi = c;
        }
        n = chi - clo;
    }
    float r;
    if (k == clo) {
        r = INFINITY;
#pragma unroll
        for (int v = 0; v < NV; ++v) r = __builtin_fminf(r, x[v] >= lo ? x[v] : INFINITY);
        r = wave_minmax(r, false);
    } else {
        r = -INFINITY;
#pragma unroll
        for (int v = 0; v < NV; ++v) r = __builtin_fmaxf(r, x[v] < hi ? x[v] : -INFINITY);
        r = wave_minmax(r, true);
    }
    return r;
}

// Start point for the search: each lane takes the median of three of its
// values (lanes short of a third value borrow the neighbour lane's), then the
// median of three across lane pairs of its quad, and the wave averages those.
// Photon pixels rarely survive two median-of-three stages.
template <int NV>
__device__ __forceinline__ float median_estimate(const float (&x)[NV])
{
    float m3;
    if (NV >= 3) {
        const float nb1 = __shfl_xor(x[1], 1, 64);
        const float c = x[2] < INFINITY ? x[2] : (nb1 < INFINITY ? nb1 : x[0]);
        m3 = __builtin_amdgcn_fmed3f(x[0], x[1], c);
    } else {
        const float c = __shfl_xor(x[0], 1, 64);
        m3 = __builtin_amdgcn_fmed3f(x[0], x[1], c < INFINITY ? c : x[0]);
    }
    const bool lv = x[0] < INFINITY;
    m3 = lv ? m3 : INFINITY;
    const int v = __float_as_int(m3);
    const float a = __int_as_float(__builtin_amdgcn_update_dpp(v, v, 0xB1, 0xF, 0xF, false));  // quad_perm 1,0,3,2
    const float b = __int_as_float(__builtin_amdgcn_update_dpp(v, v, 0x4E, 0xF, 0xF, false));  // quad_perm 2,3,0,1
    float n9 = __builtin_amdgcn_fmed3f(m3, a, b);
    n9 = lv ? (n9 < INFINITY ? n9 : m3) : 0.0f;
    const float sum = wave_sum(n9);
    const int nl = popc64(ballot(lv));
    return uniform_f(sum * __builtin_amdgcn_rcpf((float)nl));
}

struct V2Layout {
    uint32_t u, med, bits, cnt, seed, q, nseed, pref, total;  // float offsets
};

__device__ __forceinline__ V2Layout v2_layout(int rmax, int W, int nb, int seed_cap)
{
    V2Layout L;
    uint32_t o = 0;
    L.u = o;
    o += (uint32_t)rmax * W;
    L.med = o;
    o += (uint32_t)rmax * nb;
    L.bits = o;
    o += 2u * rmax * nb * 8;
    L.cnt = o;
    o += 2u * rmax * nb;
    L.seed = o;
    o += 2u * seed_cap;
    L.q = o;
    o += 2u * seed_cap;
    L.nseed = o;
    o += 2;
    L.pref = o;
    o += (uint32_t)rmax * nb + 1;
    L.total = o;
    return L;
}

size_t frame_kernel_v2_lds_bytes(int rmax, int W, int nb, int seed_cap)
{
    size_t o = (size_t)rmax * W + (size_t)rmax * nb + 2ull * rmax * nb * 8 + 2ull * rmax * nb +
               4ull * seed_cap + 2 + (size_t)rmax * nb + 1;
    return o * 4;
}

template <int NQ, int GMAX, bool KEEP>
__global__ void __launch_bounds__(kV2Threads) frame_kernel_v2(V2Args A)
{
    extern __shared__ float lds[];
    __shared__ unsigned long long s_photons;
    __shared__ uint64_t s_base;

    constexpr int NV = 2 * NQ;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int W = A.W, B = A.B, nb = A.nb, H = A.H;
    const V2Layout L = v2_layout(A.rmax, W, nb, A.seed_cap);
    float *s_u = lds + L.u;
    float *s_med = lds + L.med;
    uint32_t *s_bits = reinterpret_cast<uint32_t *>(lds + L.bits);
    uint32_t *s_cnt = reinterpret_cast<uint32_t *>(lds + L.cnt);
    uint32_t *s_seed = reinterpret_cast<uint32_t *>(lds + L.seed);
    float *s_q = lds + L.q;
    uint32_t *s_nseed = reinterpret_cast<uint32_t *>(lds + L.nseed);
    uint32_t *s_pref = reinterpret_cast<uint32_t *>(lds + L.pref);

    const int item = A.wg_item[blockIdx.x];
    const int strip = item % A.n_strips;
    const int fg = item / A.n_strips;
    const V2Strip S = A.strips[strip];
    const int t = S.tile;
    const int lr0 = max(S.r0 - 1, 0);
    const int lr1 = min(S.r1 + 1, H);
    const int R = lr1 - lr0;
    const int own_lo = S.r0 - lr0, own_hi = S.r1 - lr0;
    const int BR = R * nb;
    const uint64_t npix = (uint64_t)A.T * H * W;
    const uint64_t f_begin = (A.n_frames * (uint64_t)fg) / A.n_fgroups;
    const uint64_t f_end = (A.n_frames * (uint64_t)(fg + 1)) / A.n_fgroups;
    const int kmed = (B - 1) / 2;
    const uint32_t row_base = ((uint32_t)t * H + lr0) * (uint32_t)W;  // pixel index of loaded row 0

    // lane l of pair-slot q holds bank columns 128q + 2l and 128q + 2l + 1
    bool lane_ok[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) lane_ok[q] = 128 * q + 2 * lane < B;
    const uint32_t lane_off = 2u * lane;
    // this wave's bank-rows g < ng: bank-row index i = wave + 8g, its local row
    // and its first pixel (offset from row_base), all wave-uniform
    const int ng = BR > wave ? min(GMAX, (BR - wave + kV2Waves - 1) / kV2Waves) : 0;
    int row_[GMAX];
    uint32_t gb_[GMAX];
#pragma unroll
    for (int g = 0; g < GMAX; ++g) {
        const int i = wave + kV2Waves * g;
        row_[g] = i / nb;
        gb_[g] = (uint32_t)row_[g] * W + (uint32_t)(i - row_[g] * nb) * B;
    }

    // resident calibration of this wave's bank-rows
    float pd[GMAX][NQ][2], kk[GMAX][NQ][2];
#pragma unroll
    for (int g = 0; g < GMAX; ++g) {
        const bool gv = g < ng;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            pd[g][q][0] = pd[g][q][1] = 0.0f;
            kk[g][q][0] = kk[g][q][1] = 0.0f;
            if (gv && lane_ok[q]) {
                const uint32_t o = row_base + gb_[g] + 128 * q + lane_off;
                const float2 pp = *reinterpret_cast<const float2 *>(A.ped + o);
                const float2 kp = *reinterpret_cast<const float2 *>(A.k + o);
                pd[g][q][0] = pp.x;
                pd[g][q][1] = pp.y;
                kk[g][q][0] = kp.x;
                kk[g][q][1] = kp.y;
            }
        }
    }
    // clear both parities of the per-frame LDS lists
    for (int x = tid; x < 2 * A.rmax * nb * 8; x += kV2Threads) s_bits[x] = 0;
    for (int x = tid; x < 2 * A.rmax * nb; x += kV2Threads) s_cnt[x] = 0;
    if (tid < 2) s_nseed[tid] = 0;
    if (tid == 0) s_photons = 0;

    uint64_t chunk_cur = 0, chunk_end = 0;  // staging chunk of thread 0
    uint32_t raw[GMAX][NQ];
    auto load_raw = [&](uint64_t f) {
        const uint32_t *fr = reinterpret_cast<const uint32_t *>(A.frames + f * npix + row_base);
#pragma unroll
        for (int g = 0; g < GMAX; ++g) {
            const bool gv = g < ng;
#pragma unroll
            for (int q = 0; q < NQ; ++q)
                raw[g][q] = (gv && lane_ok[q]) ? __builtin_nontemporal_load(fr + ((gb_[g] + 128 * q + lane_off) >> 1)) : 0u;
        }
    };
    if (f_begin < f_end) load_raw(f_begin);
    __syncthreads();

    for (uint64_t f = f_begin; f < f_end; ++f) {
        const int par = (int)(f & 1);
        uint32_t cur[GMAX][NQ];
#pragma unroll
        for (int g = 0; g < GMAX; ++g)
#pragma unroll
            for (int q = 0; q < NQ; ++q) cur[g][q] = raw[g][q];
        if (f + 1 < f_end) load_raw(f + 1);

        // ---------------- phase 1: correction, bank medians, seeds --------
        uint32_t seedbits = 0;  // bit (g*NV + v) set: seed at this lane's value-slot v of bank-row g
        float xs[GMAX][NV];
#pragma unroll
        for (int g = 0; g < GMAX; ++g) {
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                if (g < ng && lane_ok[q]) {
                    xs[g][2 * q] = dark_gain(cur[g][q] & 0xFFFFu, pd[g][q][0], kk[g][q][0]);
                    xs[g][2 * q + 1] = dark_gain(cur[g][q] >> 16, pd[g][q][1], kk[g][q][1]);
                    *reinterpret_cast<float2 *>(s_u + gb_[g] + 128 * q + lane_off) =
                        make_float2(xs[g][2 * q], xs[g][2 * q + 1]);
                } else {
                    xs[g][2 * q] = INFINITY;
                    xs[g][2 * q + 1] = INFINITY;
                }
            }
        }
#pragma unroll
        for (int g = 0; g < GMAX; ++g) {
            if (g >= ng) break;
            const float est = median_estimate<NV>(xs[g]);
            const float m = bank_median<NV>(xs[g], B, kmed, est, A.rank_width * 12.0f);
            const int i = wave + kV2Waves * g;
            const int row = row_[g];
            if (lane == 0) s_med[i] = m;
            if (row >= own_lo && row < own_hi) {
                if (KEEP) {
#pragma unroll
                    for (int q = 0; q < NQ; ++q)
                        if (lane_ok[q]) {
                            float2 v2 = make_float2(__fsub_rn(xs[g][2 * q], m), __fsub_rn(xs[g][2 * q + 1], m));
                            *reinterpret_cast<float2 *>(A.corrected + f * npix + row_base + gb_[g] + 128 * q +
                                                        lane_off) = v2;
                        }
                }
                const float th = seed_threshold(m, A.t_seed);
#pragma unroll
                for (int v = 0; v < NV; ++v)
                    if (xs[g][v] >= th && xs[g][v] < INFINITY) seedbits |= 1u << (g * NV + v);
            }
        }
        // append this wave's seeds to the pooled list
        {
            const uint32_t ns = (uint32_t)__popc(seedbits);
            uint32_t incl = ns;
            for (int d = 1; d < 64; d <<= 1) {
                uint32_t y = __shfl_up(incl, d, 64);
                if (lane >= d) incl += y;
            }
            const uint32_t wtot = __shfl(incl, 63, 64);
            uint32_t base = 0;
            if (lane == 0 && wtot) base = atomicAdd(&s_nseed[par], wtot);
            base = __shfl(base, 0, 64);
            uint32_t pos = base + incl - ns;
            uint32_t bits = seedbits;
            while (bits) {
                const int b = __ffs(bits) - 1;
                bits &= bits - 1;
                const int g = b / NV, v = b - (b / NV) * NV;
                const int i = wave + kV2Waves * g;
                const int col = (i - (i / nb) * nb) * B + 128 * (v >> 1) + 2 * lane + (v & 1);
                if (pos < (uint32_t)A.seed_cap) s_seed[par * A.seed_cap + pos] = ((uint32_t)i << 16) | (uint32_t)col;
                ++pos;
            }
        }
        __syncthreads();  // B1

        // ---------------- phase 2: local maximum, charge, count ----------
        const uint32_t nseed = s_nseed[par];
        const bool overflow = nseed > (uint32_t)A.seed_cap;
        if (!overflow) {
            unsigned long long my_ph = 0;
            for (uint32_t j = tid; j < nseed; j += kV2Threads) {
                const uint32_t key = s_seed[par * A.seed_cap + j];
                const int i = key >> 16, col = key & 0xFFFF;
                const int row = i / nb, bank = i - (i / nb) * nb;
                const float vp = __fsub_rn(s_u[row * W + col], s_med[i]);
                float nv[3][3];
                bool ex[3][3];
                bool is_max = true;
#pragma unroll
                for (int dr = 0; dr < 3; ++dr)
#pragma unroll
                    for (int dc = 0; dc < 3; ++dc) {
                        const int rr = row + dr - 1, cc = col + dc - 1;
                        ex[dr][dc] = rr >= 0 && rr < R && cc >= 0 && cc < W;
                        nv[dr][dc] = 0.0f;
                        if (ex[dr][dc]) {
                            const int bk = cc >= (bank + 1) * B ? bank + 1 : (cc < bank * B ? bank - 1 : bank);
                            nv[dr][dc] = __fsub_rn(s_u[rr * W + cc], s_med[rr * nb + bk]);
                            if (!(dr == 1 && dc == 1)) {
                                const bool later = dr > 1 || (dr == 1 && dc > 1);
                                const float vq = nv[dr][dc];
                                if (!(vp > vq || (vp == vq && later))) is_max = false;
                            }
                        }
                    }
                float qsum = -1.0f;
                if (is_max) {
                    qsum = 0.0f;
#pragma unroll
                    for (int dr = 0; dr < 3; ++dr)
#pragma unroll
                        for (int dc = 0; dc < 3; ++dc)
                            if (ex[dr][dc]) qsum = __fadd_rn(qsum, nv[dr][dc] > A.t_nb ? nv[dr][dc] : 0.0f);
                    const int cb = col - bank * B;
                    atomicOr(&s_bits[(par * A.rmax * nb + i) * 8 + (cb >> 5)], 1u << (cb & 31));
                    atomicAdd(&s_cnt[par * A.rmax * nb + i], 1u);
                    my_ph += photon_count(qsum, A.photon_adu);
                }
                s_q[par * A.seed_cap + j] = qsum;
            }
            if (my_ph) atomicAdd(&s_photons, my_ph);
        }
        __syncthreads();  // B2

        // ---------------- phase 3: bank-row prefix, staging claim ---------
        if (wave == 0) {
            uint32_t total = 0;
            if (!overflow) {
                for (int base = 0; base < BR; base += 64) {
                    const int i = base + lane;
                    const uint32_t c = i < BR ? s_cnt[par * A.rmax * nb + i] : 0u;
                    uint32_t incl = c;
                    for (int d = 1; d < 64; d <<= 1) {
                        uint32_t y = __shfl_up(incl, d, 64);
                        if (lane >= d) incl += y;
                    }
                    if (i < BR) s_pref[i] = total + incl - c;
                    total += __shfl(incl, 63, 64);
                }
            }
            if (lane == 0) {
                const uint64_t unit = f * (uint64_t)A.n_strips + strip;
                uint64_t base = chunk_cur;
                if (overflow) {
                    atomicOr(&A.state->fallback, 1u);
                    base = kNoBase;
                } else if (total > 0) {
                    if (chunk_cur + total > chunk_end) {
                        const uint64_t sz = total > kChunkHits ? (uint64_t)total : kChunkHits;
                        chunk_cur = atomicAdd(&A.state->cursor, (unsigned long long)sz);
                        chunk_end = chunk_cur + sz;
                    }
                    if (chunk_cur + total <= A.pool_cap) {
                        base = chunk_cur;
                        chunk_cur += total;
                    } else {
                        base = kNoBase;
                        atomicOr(&A.state->overflow, 1u);
                    }
                }
                A.unit_base[unit] = base;
                A.unit_count[unit] = total;
                A.unit_photons[unit] = s_photons;
                s_photons = 0;
                s_base = base;
                s_nseed[par ^ 1] = 0;
            }
        }
        __syncthreads();  // B3

        // ---------------- phase 4: raster-ordered write of the hits --------
        const uint64_t base = s_base;
        if (base != kNoBase && !overflow) {
            for (uint32_t j = tid; j < nseed; j += kV2Threads) {
                const float qv = s_q[par * A.seed_cap + j];
                if (qv < 0.0f) continue;
                const uint32_t key = s_seed[par * A.seed_cap + j];
                const int i = key >> 16, col = key & 0xFFFF;
                const int row = i / nb, bank = i - (i / nb) * nb;
                const int cb = col - bank * B;
                const uint32_t *bw = s_bits + (par * A.rmax * nb + i) * 8;
                uint32_t rank = 0;
                for (int w = 0; w < (cb >> 5); ++w) rank += __popc(bw[w]);
                rank += __popc(bw[cb >> 5] & ((1u << (cb & 31)) - 1u));
                const uint32_t pix = row_base + (uint32_t)row * W + col;
                A.pool[base + s_pref[i] + rank] = make_uint2(pix, __float_as_uint(qv));
            }
        }
        // clear the other parity's bitmaps and counters for the next frame
        for (int x = tid; x < A.rmax * nb * 8; x += kV2Threads) s_bits[(par ^ 1) * A.rmax * nb * 8 + x] = 0;
        for (int x = tid; x < A.rmax * nb; x += kV2Threads) s_cnt[(par ^ 1) * A.rmax * nb + x] = 0;
    }
}

template <int NQ, int GMAX>
static hipError_t launch_v2_t(const V2Args &a, uint32_t grid, size_t lds, bool keep, hipStream_t s)
{
    if (keep) {
        auto k = frame_kernel_v2<NQ, GMAX, true>;
        hipError_t e = hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k, dim3(grid), dim3(kV2Threads), lds, s, a);
    } else {
        auto k = frame_kernel_v2<NQ, GMAX, false>;
        hipError_t e = hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k, dim3(grid), dim3(kV2Threads), lds, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_frame_kernel_v2(const V2Args &a, int nq, int gmax, uint32_t grid, size_t lds, bool keep,
                                  hipStream_t s)
{
    if (nq == 2 && gmax == 4) return launch_v2_t<2, 4>(a, grid, lds, keep, s);
    if (nq == 1 && gmax == 8) return launch_v2_t<1, 8>(a, grid, lds, keep, s);
    return hipErrorInvalidValue;
}

}  // namespace pdc
