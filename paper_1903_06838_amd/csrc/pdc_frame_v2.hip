// Persistent frame kernel for gfx950.
//
// One workgroup (16 waves) owns a strip of rows (which may cross one tile
// edge) for a range of frames.  The strip's dark and 1/gain planes are loaded once into registers
// and stay there for every frame; only the 2-byte raw words stream from HBM.
// Per frame:
//   phase 1a (each wave, its own bank-rows): load raw words (prefetched one
//     frame ahead), correct them (Fig. b) and write u to LDS;
//   phase 1b (all waves): every bank-row's lower median, exactly, by a
//     bracketing count search with L lanes per bank-row (common mode, Fig. c);
//     the same lanes then test their values against the seed threshold the
//     median implies and append the seed pixels to a workgroup list;
//   phase 1c (each wave, its own bank-rows): Frames2 if kept, one frame later;
//   phase 2 (all waves, over the pooled seeds): 3x3 local maximum with the
//     raster tie-break, masked 3x3 charge sum, photon count (Fig. e and the
//     charge summing section); hits mark a per-bank-row column bitmap;
//   phase 3 (wave 0): prefix over bank-rows, staging chunk claim;
//   phase 4 (all waves): each hit's raster position = bank-row prefix +
//     number of hits left of it in its bank-row (bitmap popcount).
//
// Lane layouts.  Phases 1a and 1c: a bank-row (B pixels of one row) is held
// by one wave as NQ pair-slots; lane l of pair-slot q holds columns 128q + 2l
// and 128q + 2l + 1 of the bank (value-slots 2q and 2q+1); absent pixels hold
// +inf.  Phase 1b: bank-row i belongs to lane group i % (64 / L) of wave
// i / (64 / L) (single-gain kernels with a row step: a wave's four groups
// take every fourth row, see the median groups' lane constants); lane j of
// the group holds columns L v + j, v < V.
#include <hip/hip_runtime.h>
#include <math.h>

#include "pdc_device.h"
#include "pdc_exact.h"
#include "pdc_internal.h"

#pragma clang fp contract(off)

namespace pdc {

#ifdef PDC_PHASE_TIMERS
// Tracing build only (PDC_PHASE_TIMERS): shader-clock cycles each wave spends
// in each phase of the persistent kernel's frame loop, summed over the launch:
// [wave][0 A, 1 A->B barrier, 2 medians, 3 seeds, 4 local maxima, 5 hit
// writes, 6 B->A barrier, 7 unused].
__device__ unsigned long long g_phase_cycles[kV2Waves * 8];
#endif


__device__ __forceinline__ uint32_t popc64(uint64_t m) { return (uint32_t)__popcll(m); }

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

__device__ __forceinline__ float uniform_f(float x)
{
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
}

// Workgroup barrier for LDS only: it waits for the wave's own LDS accesses,
// while its global loads (the next frame's words) and stores stay in flight.
// Nothing a wave writes to global memory inside the frame loop is read by
// another wave of the workgroup.
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Inclusive prefix sum over the 64 lanes (DPP row shifts, then row
// broadcasts); all lanes must be active.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x)
{
    int v = (int)x;
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xF, 0xF, true);  // row_shr:1
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xF, 0xF, true);  // row_shr:2
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xF, 0xF, true);  // row_shr:4
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xF, 0xF, true);  // row_shr:8
    v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xA, 0xF, false); // row_bcast:15
    v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xC, 0xF, false); // row_bcast:31
    return (uint32_t)v;
}

// Group reductions over aligned groups of L lanes (L = 2, 4, 8 or 16; the
// groups lie inside 16-lane DPP rows).  Every lane of a group receives the
// group's result.  All lanes of the wave must be active.
template <int L>
__device__ __forceinline__ int gsum_i(int v)
{
    v += __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, false);                // quad_perm 1,0,3,2
    if (L >= 4) v += __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xF, 0xF, false);    // quad_perm 2,3,0,1
    if (L >= 8) v += __builtin_amdgcn_update_dpp(0, v, 0x141, 0xF, 0xF, false);   // row_half_mirror
    if (L >= 16) v += __builtin_amdgcn_update_dpp(0, v, 0x140, 0xF, 0xF, false);  // row_mirror
    return v;
}

template <int L>
__device__ __forceinline__ float gsum_f(float x)
{
#define PDC_GS(ctrl) x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), ctrl, 0xF, 0xF, false))
    PDC_GS(0xB1);
    if (L >= 4) PDC_GS(0x4E);
    if (L >= 8) PDC_GS(0x141);
    if (L >= 16) PDC_GS(0x140);
#undef PDC_GS
    return x;
}

// Mask of the lane's values below p: bit v is set when x[v] < p.  For finite
// p, x < p exactly when fl(x - p) has its sign bit set (a nonzero difference
// never rounds to +0, x == p gives +0, x = +inf gives +inf); p is clamped to
// the finite range, which changes no answer because the values are bounded far
// below FLT_MAX.  Each value costs a subtraction and an alignbit that shifts
// its sign bit in; the count is one popcount of the mask.
template <int V>
__device__ __forceinline__ uint32_t lane_mask(const float (&x)[V], float p)
{
    const float pc = __builtin_amdgcn_fmed3f(p, -3.40282347e38f, 3.40282347e38f);
    uint32_t m = 0;
#pragma unroll
    for (int v = V - 1; v >= 0; --v) m = __builtin_amdgcn_alignbit(m, __float_as_uint(__fsub_rn(x[v], pc)), 31);
    return m;
}

// [lo, hi) holds a single float (adjacent keys, both bounds finite or not).
__device__ __forceinline__ bool done_single(float lo, float hi)
{
    return (uint32_t)(f2key(hi) - f2key(lo)) <= 1u;
}

// Rough location of an L-lane group's median: medians of three of each lane's
// values (up to eight triples), averaged over the group.  Dense banks (no +inf
// inside the first B columns) take the triples that every lane holds; with
// invalid pixels (SPARSE) each lane takes the finite ones.  Only the work of
// the searches below depends on it, never their result.
template <int V, int L, bool SPARSE>
__device__ __forceinline__ float group_estimate(const float (&x)[V], int B)
{
    static_assert(V >= 3, "the start estimate takes triples of values per lane");
    constexpr int NT = V / 3 < 8 ? V / 3 : 8;
    if (!SPARSE && B >= 3 * L * NT) {  // uniform: every lane's NT triples lie inside the bank
        float s3 = __builtin_amdgcn_fmed3f(x[0], x[1], x[2]);
#pragma unroll
        for (int t = 1; t < NT; ++t) s3 += __builtin_amdgcn_fmed3f(x[3 * t], x[3 * t + 1], x[3 * t + 2]);
        return gsum_f<L>(s3) * (1.0f / (float)(NT * L));
    }
    float s3 = 0.0f;
    int n3 = 0;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const float a = x[3 * t];
        const float b = x[3 * t + 1] < INFINITY ? x[3 * t + 1] : a;
        const float c = x[3 * t + 2] < INFINITY ? x[3 * t + 2] : b;
        if (a < INFINITY) {
            s3 += __builtin_amdgcn_fmed3f(a, b, c);
            ++n3;
        }
    }
    const float ssum = gsum_f<L>(s3);
    const int nl = gsum_i<L>(n3);
    return nl > 0 ? ssum * __builtin_amdgcn_rcpf((float)nl) : 0.0f;
}

// The sides of the compare-exchanges below: e[j] is -inf for a lane whose
// bit j of its place in the group is clear (it keeps the smaller value of a
// pair) and +inf otherwise.  Made once per kernel and kept in registers (an
// opaque copy, so that the compiler does not recompute them per use).
struct SortSides {
    float e[4];
};

template <int L>
__device__ __forceinline__ SortSides sort_sides()
{
    const int gl = __lane_id() & (L - 1);
    SortSides sd;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        sd.e[j] = (gl >> j) & 1 ? INFINITY : -INFINITY;
        asm volatile("" : "+v"(sd.e[j]));
    }
    return sd;
}

// Ascending bitonic sort of one value per lane over an aligned L-lane group,
// then the value of lane r broadcast to the group.  Merges of size 2b start
// with the mirror partner inside the block, then halve with xor partners; a
// compare-exchange is one median of three: med3(y, partner, -inf) is the
// smaller of the two (kept by the lower lane of the pair), med3(y, partner,
// +inf) the larger (no NaN is present).  The pick is an OR over the group of
// the chosen lane's bits and zeros elsewhere.  All lanes must be active.
template <int L>
__device__ __forceinline__ float group_sort_pick(float y, int r, const SortSides &sd)
{
    const int gl = __lane_id() & (L - 1);
    const float e1 = sd.e[0], e2 = sd.e[1], e4 = sd.e[2], e8 = sd.e[3];
#define PDC_CX(partner, e) y = __builtin_amdgcn_fmed3f(y, (partner), (e));
#define PDC_DPP(ctrl) __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(y), ctrl, 0xF, 0xF, false))
    PDC_CX(PDC_DPP(0xB1), e1)                      // merge 2: mirror (xor 1)
    if (L >= 4) {
        PDC_CX(PDC_DPP(0x1B), e2)                  // merge 4: mirror in 4
        PDC_CX(PDC_DPP(0xB1), e1)
    }
    if (L >= 8) {
        PDC_CX(PDC_DPP(0x141), e4)                 // merge 8: row_half_mirror
        PDC_CX(PDC_DPP(0x4E), e2)                  // xor 2
        PDC_CX(PDC_DPP(0xB1), e1)
    }
    if (L >= 16) {
        PDC_CX(PDC_DPP(0x140), e8)                 // merge 16: row_mirror
        {
            // xor 4 = xor 3 (quad mirror) then xor 7 (half-row mirror)
            const int t = __builtin_amdgcn_mov_dpp(__float_as_int(y), 0x1B, 0xF, 0xF, false);
            PDC_CX(__int_as_float(__builtin_amdgcn_mov_dpp(t, 0x141, 0xF, 0xF, false)), e4)
        }
        PDC_CX(PDC_DPP(0x4E), e2)
        PDC_CX(PDC_DPP(0xB1), e1)
    }
#undef PDC_DPP
#undef PDC_CX
    int rb = gl == r ? __float_as_int(y) : 0;
#define PDC_GX(ctrl) rb |= __builtin_amdgcn_update_dpp(0, rb, ctrl, 0xF, 0xF, false);
    PDC_GX(0xB1)
    if (L >= 4) PDC_GX(0x4E)
    if (L >= 8) PDC_GX(0x141)
    if (L >= 16) PDC_GX(0x140)
#undef PDC_GX
    return __int_as_float(rb);
}

// Exact element of rank k (0-based, ascending) among the nval finite values
// held by an L-lane group (V values per lane, absent values +inf, lane value
// v also at src[L v] in LDS); every group of the wave searches its own bank
// at once.  Bracketing search on counts, count(x < lo) <= k < count(x < hi)
// throughout, with the lane masks of both bounds kept: the first bracket is
// the estimate and a bound placed from its count (widening until they
// bracket), later steps
// interpolate the pivot from the bracket counts and bisect in key space when
// the interpolated pivot is not strictly inside or the bracket stopped
// halving.  Once at most L values remain in [lo, hi) (the lane's are the bits
// of mhi & ~mlo) they are gathered from LDS into the group's lanes, sorted
// across them, and the answer is read off; a bracket that holds a single float
// (possibly many copies of it) gives that float.  Groups with act false return
// an unspecified value.
template <int V, int L, bool SPARSE>
__device__ float group_median(const float (&x)[V], const float *src, int nval, int k, float rw, bool act,
                              float *gsc, int B, const SortSides &sd)
{
    const float est = group_estimate<V, L, SPARSE>(x, B);

    // First bracket in two counts: the count below the estimate gives its
    // rank error e, and the second bound goes e + 4 rank widths beyond it on
    // the side of rank k (the estimate misses by about 5 ranks on these
    // banks; two bounds placed around it at once missed twice as often)
    float lo, hi;
    uint32_t mlo, mhi;
    int clo, chi;
    {
        const uint32_t m1 = lane_mask<V>(x, est);
        const int c1 = gsum_i<L>(__popc(m1));
        const bool up = c1 <= k;  // rank k lies at or above the estimate
        const float d = (float)((up ? k + 1 - c1 : c1 - k) + 4) * rw;
        const float p2 = up ? est + d : est - d;
        const uint32_t m2 = lane_mask<V>(x, p2);
        const int c2 = gsum_i<L>(__popc(m2));
        lo = up ? est : p2;
        hi = up ? p2 : est;
        mlo = up ? m1 : m2;
        mhi = up ? m2 : m1;
        clo = up ? c1 : c2;
        chi = up ? c2 : c1;
    }
    bool ok = !act || (clo <= k && k < chi);
    // widening: a start bracket that misses by m ranks moves its violated
    // bound (m + 3) rank widths beyond, doubling the step on repeated misses
    float sc = rw;
    for (int it = 0; it < 40; ++it) {
        if (__ballot(!ok) == 0) break;
        const bool down = clo > k;
        const float d = (float)((down ? clo - k : k + 1 - chi) + 3) * sc;
        sc = sc + sc;
        const float p = it < 38 ? (down ? lo - d : hi + d) : (down ? -INFINITY : INFINITY);
        const uint32_t mp = lane_mask<V>(x, p);
        const int cp = gsum_i<L>(__popc(mp));
        if (!ok) {
            if (down) {
                hi = lo;
                chi = clo;
                mhi = mlo;
                lo = p;
                clo = cp;
                mlo = mp;
            } else {
                lo = hi;
                clo = chi;
                mlo = mhi;
                hi = p;
                chi = cp;
                mhi = mp;
            }
            ok = clo <= k && k < chi;
        }
    }

    int last_n = 4 * nval;
    bool done = !act;
    for (int it = 0; it < 200; ++it) {
        const int n = chi - clo;
        float q = lo + (hi - lo) * (((float)(k - clo) + 0.5f) * __builtin_amdgcn_rcpf((float)n));
        // q is NaN or not strictly inside when a bound is infinite
        const bool interp = 2 * n <= last_n && q > lo && q < hi;
        bool single = false;  // [lo, hi) holds one float only (never when interp holds)
        if (!interp) {
            // bisect in key space: at most 32 such steps reach a bracket that
            // holds a single float, whatever the scale (a value-space midpoint
            // would halve a bracket [0, h) through the whole exponent range)
            const int32_t klo = f2key(lo), khi = f2key(hi);
            single = (uint32_t)(khi - klo) <= 1u;
            q = key2f((klo >> 1) + (khi >> 1) + (klo & khi & 1));
        }
        done = done || n <= L || single;
        if (__ballot(!done) == 0) break;
        last_n = interp ? n : 4 * nval;
        const uint32_t mq = lane_mask<V>(x, q);
        const int cq = gsum_i<L>(__popc(mq));
        if (!done) {
            if (cq <= k) {
                lo = q;
                clo = cq;
                mlo = mq;
            } else {
                hi = q;
                chi = cq;
                mhi = mq;
            }
        }
    }
    // Finish: the n <= L values in [lo, hi) are gathered from LDS into the
    // group's lanes (gsc: L floats per group, in lane order), sorted across the
    // lanes, and lane k - clo holds the answer.  A bracket that holds a single
    // float (n > L possible) has the answer lo.
    const int gl = __lane_id() & (L - 1);
    const bool gather = !done_single(lo, hi);
    uint32_t cm = gather ? mhi & ~mlo : 0u;
    const int c = __popc(cm);
    int incl = c;
    // (a shift from outside the 16-lane row reads 0, so with L = 16 the
    // group edge needs no test)
#define PDC_SCAN(ctrl, sh)                                                                       \
    {                                                                                            \
        const int o = __builtin_amdgcn_update_dpp(0, incl, ctrl, 0xF, 0xF, true);                 \
        incl += (L == 16 || gl >= sh) ? o : 0;                                                   \
    }
    PDC_SCAN(0x111, 1)
    if (L >= 4) PDC_SCAN(0x112, 2)
    if (L >= 8) PDC_SCAN(0x114, 4)
    if (L >= 16) PDC_SCAN(0x118, 8)
#undef PDC_SCAN
    float *gb = gsc - gl;  // the group's L slots
    int pos = incl - c;
    while (cm) {
        const int v = __builtin_ctz(cm);
        cm &= cm - 1u;
        if (pos < L) gb[pos] = src[L * v];
        ++pos;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    const int n = chi - clo;
    float y = (gather && gl < n) ? gb[gl] : INFINITY;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    // exactly one lane of the group (k - clo < n <= L) holds the answer
    const float pick = group_sort_pick<L>(y, k - clo, sd);
    return gather ? pick : lo;
}

// The L-lane group's values of a bank-row: lane gl takes src[L v] (src
// points at its first column) for L v < lim = B - gl, else pad.  Every slot
// is read into its own register first; when tail_only (wave-uniform:
// B > L (V - 1)) only the last slot can lie past the bank and the others
// are kept without a test.  (Reads under the two cases in separate branches
// put the values in different registers, and the join then copies them.)
template <int V, int L>
__device__ __forceinline__ void read_group(float (&x)[V], const float *src, int lim, bool tail_only, float pad)
{
#pragma unroll
    for (int v = 0; v < V; ++v) x[v] = src[L * v];
    if (!tail_only) {
#pragma unroll
        for (int v = 0; v < V - 1; ++v) x[v] = L * v < lim ? x[v] : pad;
    }
    x[V - 1] = L * (V - 1) < lim ? x[V - 1] : pad;
}

struct V2Layout {
    uint32_t u, med, bits, cnt, seed, hl, nseed, hcnt, pref, gs, total;  // float offsets
};

// LDS of one workgroup (floats): u, med, bits, cnt, the seed lists and the
// hit lists (key and charge of each local maximum, half a seed list long)
// are double-buffered by frame parity, the seed counts kept for three frames
// (frame f mod 3); pref and the median finish scratch gs are single.
__device__ __host__ __forceinline__ V2Layout v2_layout(int rmax, int W, int nb, int seed_cap)
{
    V2Layout L;
    // W + 1 floats before u: phase 2 reads a seed's neighbours at fixed
    // offsets from the row above, column left, without clamping (what lies
    // outside the rows or the tile is read and then masked)
    uint32_t o = ((uint32_t)W + 4u) & ~3u;
    L.u = o;
    o += 2u * rmax * W;
    L.med = o;
    o += 2u * rmax * nb;
    L.bits = o;
    o += 2u * rmax * nb * 8;
    L.cnt = o;
    o += 2u * rmax * nb;
    L.seed = o;
    o += 2u * seed_cap;
    o = (o + 1u) & ~1u;  // 8-byte hit entries
    L.hl = o;
    o += 2u * 2u * (uint32_t)(seed_cap / 2);
    L.nseed = o;
    o += 3;
    L.hcnt = o;
    o += 2;
    L.pref = o;
    o += (uint32_t)rmax * nb + 1;
    L.gs = o;
    o += 1024;
    L.total = o;
    return L;
}

size_t frame_kernel_v2_lds_bytes(int rmax, int W, int nb, int seed_cap)
{
    return (size_t)v2_layout(rmax, W, nb, seed_cap).total * 4;
}

// Item (frame group, strip) of block b among n: blocks are dealt to the 8 XCDs
// round-robin (block b to XCD b mod 8) and the items, in raster order, go to
// the blocks of one XCD after another, so neighbouring strips (which share halo
// rows) share an L2.
__device__ __forceinline__ int block_item(int b, int n)
{
    const int x = b & 7;
    int before = 0;
    for (int y = 0; y < x; ++y) before += (n - y + 7) >> 3;  // blocks of XCD y
    return before + (b >> 3);
}

// Seed key: loaded row (7 bits), bank (7 bits), column (11 bits).
__device__ __forceinline__ uint32_t seed_key(int row, int bank, int col)
{
    return ((uint32_t)row << 18) | ((uint32_t)bank << 11) | (uint32_t)col;
}

typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

// Pixels of a strip's loaded rows per thread in the flat correction pass:
// CH chunks of 4 (a strip holds at most 16 waves x 4 x 64 / L bank-rows of
// at most 256 / 128 pixels, i.e. 16384 pixels).
constexpr int kFlatChunks = 4;

// One workgroup's work: work item `item` of the launch over A's strips and
// frame groups (strip item % n_strips, frame group item / n_strips).
template <int NQ, int GMAX, int L, int V, bool KEEP, bool CMM, bool MG>
__device__ __forceinline__ void frame_body(const V2Args &A, const int item)
{
    // Single-gain kernels correct the strip as one flat block of pixels
    // (FLAT); auto-ranging kernels keep a wave per bank-row, whose lanes
    // look up their pixels' range planes.
    constexpr bool FLAT = !MG;
    extern __shared__ __align__(16) float lds[];
#ifdef PDC_PHASE_TIMERS
    __shared__ unsigned long long s_tm[kV2Waves * 8];
    if (threadIdx.x < kV2Waves * 8) s_tm[threadIdx.x] = 0;
#endif
    __shared__ unsigned long long s_photons;
    __shared__ uint64_t s_base;
    __shared__ uint64_t s_chunk[2];  // staging chunk in use: next free entry, end
    __shared__ uint32_t s_p2ctr, s_p4ctr;
    uint32_t *s_p2next = &s_p2ctr;  // next phase-2 seed chunk
    uint32_t *s_p4next = &s_p4ctr;  // next phase-4 hit chunk

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int W = A.W, B = A.B, nb = A.nb, H = A.H;
    const V2Layout Ly = v2_layout(A.rmax, W, nb, A.seed_cap);
    const int RW = A.rmax * W, RN = A.rmax * nb, cap = A.seed_cap, hcap = A.seed_cap / 2;
    float *s_u = lds + Ly.u;
    float *s_med = lds + Ly.med;
    uint32_t *s_bits = reinterpret_cast<uint32_t *>(lds + Ly.bits);
    uint32_t *s_cnt = reinterpret_cast<uint32_t *>(lds + Ly.cnt);
    uint32_t *s_seed = reinterpret_cast<uint32_t *>(lds + Ly.seed);
    uint2 *s_hl = reinterpret_cast<uint2 *>(lds + Ly.hl);
    uint32_t *s_hcnt = reinterpret_cast<uint32_t *>(lds + Ly.hcnt);
    uint32_t *s_nseed = reinterpret_cast<uint32_t *>(lds + Ly.nseed);
    uint32_t *s_pref = reinterpret_cast<uint32_t *>(lds + Ly.pref);
    float *s_gs = lds + Ly.gs;  // one slot per thread: median finish scratch

    const int strip = item % A.n_strips;
    const int fg = item / A.n_strips;
    const V2Strip S = A.strips[strip];
    const int lr0 = S.lg0;  // global rows
    const int R = S.lg1 - lr0;
    const int own_lo = S.g0 - lr0, own_hi = S.g1 - lr0;
    const int bnd = S.gb == INT32_MAX ? R : S.gb - lr0;  // loaded row where a second tile starts
    const int BR = R * nb;
    const uint64_t npix = (uint64_t)A.T * H * W;
    const uint64_t f_begin = (A.n_frames * (uint64_t)fg) / A.n_fgroups;
    const uint64_t f_end = (A.n_frames * (uint64_t)(fg + 1)) / A.n_fgroups;
    const int kmed = (B - 1) / 2;
    const uint32_t row_base = (uint32_t)lr0 * (uint32_t)W;  // pixel index of loaded row 0
    constexpr int kP3Wave = 0;  // wave that runs phase 3 (the first to issue on its SIMD)

    // lane l of pair-slot q holds bank columns 128q + 2l and 128q + 2l + 1
    bool lane_ok[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) lane_ok[q] = 128 * q + 2 * lane < B;
    const uint32_t lane_off = 2u * lane;
    const SortSides sides = sort_sides<L>();  // the bank-median finish's sort
    // Lane constants of the single-gain median groups: the bank-row mi of
    // the lane's group, the LDS offset of its first value, its row, its first
    // seed key and the mask of its value slots inside the bank.  Made once and
    // kept (opaque copies): recomputed per frame they cost three quarter-rate
    // multiplies and a 64-bit shift.  Group slot s = wave 64 / L + lane / L
    // takes bank-row s, except that with the row step d = 4 (16-lane groups)
    // the loaded rows go in blocks of 4 d, and the four groups of a wave take
    // one bank of rows j, j + d, j + 2 d, j + 3 d of a block, so that their
    // LDS reads fall in different banks; rows past the last whole block keep
    // bank-row s.  Either way slot s is active exactly when s < BR.
    int mi = 0, mrow = 0, moff = 0;
    uint32_t mkey0 = 0, mvmask = 0;
    if constexpr (!CMM && FLAT) {
        const int grp = lane / L, gl = lane - grp * L;
        mi = wave * (64 / L) + grp;
        if (L == 16 && A.med_row_step == 4) {
            constexpr int d = 4;
            const int per = 4 * d * nb;                  // bank-rows of a block
            if (mi < (R / (4 * d)) * per) {
                const int blk = mi / per, t = mi - blk * per;
                const int wi = t >> 2, g = t & 3;        // wave of the block, group
                mi = (blk * 4 * d + wi % d + d * g) * nb + wi / d;
            }
        }
        const bool act = mi < BR;
        mrow = act ? mi / nb : 0;
        const int bank = act ? mi - mrow * nb : 0;
        moff = mrow * W + bank * B + gl;
        mkey0 = seed_key(mrow, bank, bank * B + gl);
        const int lim = B - gl;
        mvmask = B > L * (V - 1) ? ((L * (V - 1) < lim) ? (1u << V) - 1u : (1u << (V - 1)) - 1u)
                                 : (uint32_t)((1ull << min(V, max(0, (lim + L - 1) / L))) - 1ull);
        asm volatile("" : "+v"(mi), "+v"(mrow), "+v"(moff), "+v"(mkey0), "+v"(mvmask));
    }
    // this wave's bank-rows g < ng: bank-row index i = wave + 16g, its local
    // row and its first pixel (offset from row_base), all wave-uniform
    const int ng = BR > wave ? min(GMAX, (BR - wave + kV2Waves - 1) / kV2Waves) : 0;
    int row_[GMAX], bank_[GMAX];
    uint32_t gb_[GMAX];
#pragma unroll
    for (int g = 0; g < GMAX; ++g) {
        const int i = wave + kV2Waves * g;
        row_[g] = i / nb;
        bank_[g] = i - row_[g] * nb;
        gb_[g] = (uint32_t)row_[g] * W + (uint32_t)bank_[g] * B;
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
    // FLAT: the loaded rows are one contiguous block of R W words of each
    // frame (W % 4 == 0), cut into 4-pixel chunks j = tid + 1024 c; each
    // chunk's dark and 1/gain values stay in registers
    const int nchunk = FLAT ? (R * W) >> 2 : 0;
    float4 pdq[kFlatChunks], kkq[kFlatChunks];
#pragma unroll
    for (int c = 0; c < kFlatChunks; ++c) {
        const int j = tid + kV2Threads * c;
        pdq[c] = kkq[c] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        if (FLAT && j < nchunk) {
            pdq[c] = *reinterpret_cast<const float4 *>(A.ped + row_base + 4u * j);
            kkq[c] = *reinterpret_cast<const float4 *>(A.k + row_base + 4u * j);
        }
    }
    // the calibration loads complete here (vmcnt 0): left pending, their first
    // use inside the frame loop would make the compiler wait there for every
    // load in flight, the next frame's prefetch included
    __builtin_amdgcn_s_waitcnt(0x0F70);
    for (int x = tid; x < 2 * RN * 8; x += kV2Threads) s_bits[x] = 0;
    for (int x = tid; x < 2 * RN; x += kV2Threads) s_cnt[x] = 0;
    if (tid < 3) s_nseed[tid] = 0;
    if (tid < 2) s_hcnt[tid] = 0;
    if (tid == 0) s_photons = 0;
    if (tid == 0) s_p2ctr = 0;
    if (tid == 0) s_p4ctr = 0;

    if (tid == 0) s_chunk[0] = s_chunk[1] = 0;
    uint32_t raw[GMAX][NQ];
    auto load_raw = [&](uint64_t f, const bool(&lok)[NQ]) {
        const uint32_t *fr = reinterpret_cast<const uint32_t *>(A.frames + f * npix + row_base);
#pragma unroll
        for (int g = 0; g < GMAX; ++g) {
            const bool gv = g < ng;
#pragma unroll
            for (int q = 0; q < NQ; ++q)
                // gb_[g] is even (W and B are), so the word address is a
                // wave-uniform base plus the lane
                raw[g][q] = (gv && lok[q]) ? __builtin_nontemporal_load(fr + ((gb_[g] >> 1) + 64 * q) + lane) : 0u;
        }
    };
    u32x2 rawq[kFlatChunks];
#pragma unroll
    for (int c = 0; c < kFlatChunks; ++c) rawq[c] = u32x2{0u, 0u};
    // (t: the thread index, an opaque copy made each frame, so that the
    // chunk tests are recomputed rather than kept in scalar registers)
    auto load_raw_flat = [&](uint64_t f, int t) {
        const u32x2 *fr = reinterpret_cast<const u32x2 *>(A.frames + f * npix + row_base);
#pragma unroll
        for (int c = 0; c < kFlatChunks; ++c) {
            const int j = t + kV2Threads * c;
            if (j < nchunk) rawq[c] = __builtin_nontemporal_load(fr + j);
        }
    };
    if (f_begin < f_end) {
        if constexpr (FLAT)
            load_raw_flat(f_begin, tid);
        else
            load_raw(f_begin, lane_ok);
    }
    __syncthreads();

    // Seeds of a bank-row held by an L-lane group in phase B (lane gl holds
    // columns L v + gl in xs, +inf where absent or invalid): fl(x - m) > t,
    // own rows only, appended to the pooled list sbuf (frame parity; order is
    // free, phase 4 restores raster order) counted in slot (frame mod 3), with
    // a DPP prefix of the lanes' counts and one LDS atomic per wave.  The test
    // is the sign of fl(t - fl(x - m)) (see append_seeds_dense), and +inf is
    // dropped by the sign of x - 2^100 (set for every finite value, which is
    // far below 2^100).  All lanes of the wave must call it.
    auto append_seeds = [&](const float(&xs)[V], float m, float t, bool own, int row, int bank, int gl, int sbuf,
                            int slot) {
        uint32_t sb = 0, fin = 0;
#pragma unroll
        for (int v = V - 1; v >= 0; --v) {
            sb = __builtin_amdgcn_alignbit(sb, __float_as_uint(__fsub_rn(t, __fsub_rn(xs[v], m))), 31);
            fin = __builtin_amdgcn_alignbit(fin, __float_as_uint(__fsub_rn(xs[v], 0x1p100f)), 31);
        }
        sb = own ? sb & fin : 0u;
        const uint32_t ns = (uint32_t)__popc(sb);
        const uint32_t incl = wave_incl_scan(ns);
        const uint32_t wtot = (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
        if (wtot) {
            uint32_t base = 0;
            if (lane == 0) base = atomicAdd(&s_nseed[slot], wtot);
            uint32_t pos = (uint32_t)__builtin_amdgcn_readfirstlane((int)base) + incl - ns;
            while (sb) {
                const int v = __ffs(sb) - 1;
                sb &= sb - 1;
                if (pos < (uint32_t)cap) s_seed[sbuf * cap + pos] = seed_key(row, bank, bank * B + L * v + gl);
                ++pos;
            }
        }
    };
    // The same for the single-gain median kernels: values of the slots in
    // vmask are finite (the others, past the bank, are dropped); a value is a
    // seed when fl(x - m) > t, that is when fl(t - fl(x - m)) < 0 (exact
    // difference of two finite values: its sign is the test, equality gives
    // +0), one sign bit per value shifted in from the last value down.
    auto append_seeds_dense = [&](const float(&xs)[V], float m, float t, bool own, uint32_t vmask, uint32_t key0,
                                  int sbuf, int slot) {
        uint32_t sb = 0;
#pragma unroll
        for (int v = V - 1; v >= 0; --v)
            sb = __builtin_amdgcn_alignbit(sb, __float_as_uint(__fsub_rn(t, __fsub_rn(xs[v], m))), 31);
        sb = own ? sb & vmask : 0u;
        const uint32_t ns = (uint32_t)__popc(sb);
        const uint32_t incl = wave_incl_scan(ns);
        const uint32_t wtot = (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
        if (wtot) {
            uint32_t base = 0;
            if (lane == 0) base = atomicAdd(&s_nseed[slot], wtot);
            uint32_t pos = (uint32_t)__builtin_amdgcn_readfirstlane((int)base) + incl - ns;
            while (sb) {
                const int v = __ffs(sb) - 1;
                sb &= sb - 1;
                if (pos < (uint32_t)cap) s_seed[sbuf * cap + pos] = key0 + (uint32_t)(L * v);
                ++pos;
            }
        }
    };

    // Software pipeline, two barriers per frame: iteration f runs
    //   A: frame f's phase 1a, frame f-1's Frames2, frame f-2's phase 3 (one
    //      wave, beside the others' 1a);
    //   B: frame f's phase 1b with the seed list, then, claimed in chunks by
    //      waves as they finish their median groups, frame f-1's phase 2
    //      (which lists its hits) and frame f-2's phase 4 (over that list).
    // Two more iterations drain it.  u, medians, seed lists, hit lists, hit
    // bitmaps and counts are double-buffered by frame parity (par for f and
    // f-2, pp for f-1); the seed counts are kept for three frames (f mod 3).
#ifdef PDC_PHASE_TIMERS
    unsigned long long tm_prev = __builtin_amdgcn_s_memtime();
#define PDC_PHASE(ph)                                                                     \
    {                                                                                     \
        const unsigned long long t_ = __builtin_amdgcn_s_memtime();                       \
        if ((threadIdx.x & 63) == 0) atomicAdd(&s_tm[(threadIdx.x >> 6) * 8 + (ph)], t_ - tm_prev); \
        tm_prev = t_;                                                                     \
    }
#else
#define PDC_PHASE(ph)
#endif
    // f mod 3, advanced with f (a 64-bit remainder per frame costs scalar
    // instructions and registers)
    int f3 = (int)(f_begin % 3);
    for (uint64_t f = f_begin; f < f_end + 2; ++f, f3 = f3 == 2 ? 0 : f3 + 1) {
        const bool cur_ok = f < f_end;
        const bool p1_ok = f >= f_begin + 1 && f - 1 < f_end;
        const bool p2_ok = f >= f_begin + 2;
        const int par = (int)(f & 1), pp = par ^ 1;
        const int sc0 = f3, sc1 = f3 == 0 ? 2 : f3 - 1, sc2 = f3 == 2 ? 0 : f3 + 1;  // seed counts of f, f-1, f-2
        const uint32_t nseed_1 = p1_ok ? s_nseed[sc1] : 0u;  // frame f-1
        const uint32_t nseed_2 = p2_ok ? s_nseed[sc2] : 0u;  // frame f-2
        const uint32_t nhit_2 = p2_ok ? s_hcnt[par] : 0u;    // frame f-2's listed hits
        // a seed list or a hit list that was full: the general kernel redoes the unit
        const bool ovf_1 = nseed_1 > (uint32_t)cap;
        const bool ovf_2 = nseed_2 > (uint32_t)cap || nhit_2 > (uint32_t)hcap;
        float *u_c = s_u + par * RW;
        const float *u_p = s_u + pp * RW;
        float *med_c = s_med + par * RN;
        const float *med_p = s_med + pp * RN;
        // the lane masks are recomputed each frame from an opaque copy of the
        // lane offset: hoisted out of the loop they would be kept in scalar
        // registers, which this kernel does not have to spare
        bool lok[NQ];
        {
            uint32_t lo = lane_off;
            asm volatile("" : "+v"(lo));
#pragma unroll
            for (int q = 0; q < NQ; ++q) lok[q] = 128u * q + lo < (uint32_t)B;
        }
        int tid_f = tid;  // the same for the flat chunk tests
        asm volatile("" : "+v"(tid_f));

        // ================= A: 1a(f) | Frames2(f-1) | 3(f-2) =======================
        if (FLAT && cur_ok) {
            // frame f's words were loaded at the end of the previous A
#pragma unroll
            for (int c = 0; c < kFlatChunks; ++c) {
                const int j = tid_f + kV2Threads * c;
                if (j < nchunk) {
                    const uint32_t w0 = rawq[c].x & 0x3FFF3FFFu, w1 = rawq[c].y & 0x3FFF3FFFu;
                    float4 o;
                    o.x = __fmul_rn(__fsub_rn((float)(w0 & 0xFFFFu), pdq[c].x), kkq[c].x);
                    o.y = __fmul_rn(__fsub_rn((float)(w0 >> 16), pdq[c].y), kkq[c].y);
                    o.z = __fmul_rn(__fsub_rn((float)(w1 & 0xFFFFu), pdq[c].z), kkq[c].z);
                    o.w = __fmul_rn(__fsub_rn((float)(w1 >> 16), pdq[c].w), kkq[c].w);
                    *reinterpret_cast<float4 *>(u_c + 4 * j) = o;
                }
            }
        }
        if (!FLAT && cur_ok) {
            uint32_t cur[GMAX][NQ];
#pragma unroll
            for (int g = 0; g < GMAX; ++g)
#pragma unroll
                for (int q = 0; q < NQ; ++q) cur[g][q] = raw[g][q];
            if (f + 1 < f_end) load_raw(f + 1, lok);
            if constexpr (!MG) {
#pragma unroll
                for (int g = 0; g < GMAX; ++g)
#pragma unroll
                    for (int q = 0; q < NQ; ++q)
                        if (g < ng && lok[q])
                            *reinterpret_cast<float2 *>(u_c + gb_[g] + 128 * q + lane_off) =
                                make_float2(dark_gain(cur[g][q] & 0xFFFFu, pd[g][q][0], kk[g][q][0]),
                                            dark_gain(cur[g][q] >> 16, pd[g][q][1], kk[g][q][1]));
            } else {
                // auto-ranging: range 0 from the resident planes and invalid
                // codes as +inf (counted on own rows) first; the rarer pixels in
                // ranges 1 and 2 then read their planes from memory
                uint32_t ninv = 0, slow = 0;  // slow: bit 2 (g NQ + q) + h for ranges 1, 2
#pragma unroll
                for (int g = 0; g < GMAX; ++g)
#pragma unroll
                    for (int q = 0; q < NQ; ++q)
                        if (g < ng && lok[q]) {
                            const uint32_t w = cur[g][q];
                            const int r0 = gain_range(w & 0xFFFFu, A.gain_mode), r1 = gain_range(w >> 16, A.gain_mode);
                            const float u0 = r0 == 0 ? dark_gain(w & 0xFFFFu, pd[g][q][0], kk[g][q][0]) : INFINITY;
                            const float u1 = r1 == 0 ? dark_gain(w >> 16, pd[g][q][1], kk[g][q][1]) : INFINITY;
                            *reinterpret_cast<float2 *>(u_c + gb_[g] + 128 * q + lane_off) = make_float2(u0, u1);
                            if (row_[g] >= own_lo && row_[g] < own_hi) ninv += (uint32_t)(r0 < 0) + (uint32_t)(r1 < 0);
                            slow |= ((uint32_t)(r0 > 0) | ((uint32_t)(r1 > 0) << 1)) << (2 * (g * NQ + q));
                        }
                while (slow) {
                    const int bit = __ffs(slow) - 1;
                    slow &= slow - 1;
                    const int gq = bit >> 1, h = bit & 1;
                    const int g = gq / NQ, q = gq - g * NQ;
                    const uint32_t off = gb_[g] + 128 * q + lane_off + h;
                    const uint32_t w = (cur[g][q] >> (16 * h)) & 0xFFFFu;
                    const uint64_t o = row_base + off + (uint64_t)gain_range(w, A.gain_mode) * npix;
                    u_c[off] = dark_gain(w, A.ped[o], A.k[o]);
                }
                const uint32_t tot = (uint32_t)__builtin_amdgcn_readlane((int)wave_incl_scan(ninv), 63);
                if (lane == 0 && tot) atomicAdd(A.invalid + f, tot);
            }
        }
        // frame f-1's hit bitmaps and counts (parity pp) are rebuilt by its
        // local maxima in B; their last reader, frame f-3, finished in B of f-1
        if (p1_ok) {
            for (int x = tid; x < RN * 8; x += kV2Threads) s_bits[pp * RN * 8 + x] = 0;
            for (int x = tid; x < RN; x += kV2Threads) s_cnt[pp * RN + x] = 0;
        }
        if (tid == 0) {
            s_nseed[sc0] = 0;  // frame f-3's count, last read before B of f-1
            s_hcnt[pp] = 0;    // frame f-3's hits were written in B of f-1
            *s_p2next = 0;
            *s_p4next = 0;
        }
        if (KEEP && !FLAT && p1_ok) {
            // Frames2 of frame f-1 (its u and medians, parity pp, are intact);
            // the flat kernels write Frames2 in phase B
#pragma unroll
            for (int g = 0; g < GMAX; ++g) {
                if (g >= ng) break;
                const int i = wave + kV2Waves * g;
                const int row = row_[g];
                if (row >= own_lo && row < own_hi) {
                    const float m = uniform_f(med_p[i]);
#pragma unroll
                    for (int q = 0; q < NQ; ++q)
                        if (lok[q]) {
                            const float2 u2 = *reinterpret_cast<const float2 *>(u_p + gb_[g] + 128 * q + lane_off);
                            *reinterpret_cast<float2 *>(A.corrected + (f - 1) * npix + row_base + gb_[g] + 128 * q +
                                                        lane_off) = make_float2(__fsub_rn(u2.x, m), __fsub_rn(u2.y, m));
                        }
                }
            }
        }
        if (p2_ok && wave == kP3Wave) {
            // bank-row prefix of frame f-2's hit counts (parity par), staging
            // chunk claim; the wave that runs it issues first, so it also
            // finishes its own phase 1a first
            uint32_t total = 0;
            if (!ovf_2) {
                for (int b0 = 0; b0 < BR; b0 += 64) {
                    const int i = b0 + lane;
                    const uint32_t c = i < BR ? s_cnt[par * RN + i] : 0u;
                    const uint32_t incl = wave_incl_scan(c);
                    if (i < BR) s_pref[i] = total + incl - c;
                    total += (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
                }
            }
            if (lane == 0) {
                // the chunk lives in LDS: in registers it would be spilled to
                // scratch, whose reload waits for the frame prefetch
                uint64_t chunk_cur = s_chunk[0], chunk_end = s_chunk[1];
                const uint64_t unit = (f - 2) * (uint64_t)A.n_strips + strip;
                uint64_t base = chunk_cur;
                if (ovf_2) {
                    // the seed list was full: the general kernel redoes this unit
                    atomicOr(&A.state->fallback, 1u);
                    if (A.fb_units) A.fb_units[atomicAdd(&A.state->n_fallback, 1ull)] = unit;
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
                A.unit_photons[unit] = s_photons;  // frame f-2's, summed in B of f-1
                s_photons = 0;
                s_base = base;
                s_chunk[0] = chunk_cur;
                s_chunk[1] = chunk_end;
            }
        }
        // the loads of frame f + 1 go out last in A, into the registers frame
        // f's words were in: they overlap phase B and the barriers, and no
        // wait in A (the staging claim's atomics) waits for them
        if (FLAT && f + 1 < f_end) load_raw_flat(f + 1, tid_f);
        PDC_PHASE(0);
        lds_barrier();  // A -> B
        PDC_PHASE(1);

        // ================= B: 1b(f) | 2(f-1) | 4(f-2) =============================
        if (CMM && cur_ok && A.cm_mode == 1) {
            // thresholded mean of each bank-row (Fig. c), stacked stages: the sum
            // of the noise values is exact, rounded once (the group's lanes add
            // two binary64 limbs); v replaces u in place and the median slot
            // holds 0.  A bank-row whose values span more than two limbs hold
            // marks the frame's seed list full, so that the general kernel
            // redoes the unit from the separately computed stage values.
            constexpr int G = 64 / L;
            const int grp = lane / L, gl = lane - grp * L;
            const int i = wave * G + grp;
            const bool act = i < BR;
            const int row = act ? i / nb : 0;
            const int bank = act ? i - row * nb : 0;
            float *dst = u_c + row * W + bank * B;
            float x[V];
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const int c = L * v + gl;
                x[v] = (act && c < B) ? dst[c] : INFINITY;  // +inf: absent or invalid, never noise
            }
            SumWindow win = {A.sum_lo, A.sum_hi};
            bool wide = false;
#pragma unroll
            for (int s = 0; s < 3; ++s) {
                if (s >= A.cm_stages) break;
                int n;
                bool fits;
                const float sum = region_sum<L, V, false>(x, A.t_cm, (uint32_t)B, win, n, fits);
                wide |= !fits;
                const int n0 = gsum_i<L>(n);
                const float cm = __fdiv_rn(sum, fmaxf((float)n0, A.cm_guard));
                win = next_window(win, cm);
#pragma unroll
                for (int v = 0; v < V; ++v) x[v] = __fsub_rn(x[v], cm);
            }
            if (act && wide && gl == 0) atomicAdd(&s_nseed[sc0], (uint32_t)cap + 1u);
            if (act) {
                float *f2 = (KEEP && FLAT && row >= own_lo && row < own_hi)
                                ? A.corrected + f * npix + row_base + row * W + bank * B
                                : nullptr;
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    const int c = L * v + gl;
                    if (c < B) {
                        const float y = x[v] < INFINITY ? x[v] : 0.0f;  // invalid: v = 0
                        dst[c] = y;
                        if (f2) f2[c] = y;
                    }
                }
                if (gl == 0) med_c[i] = 0.0f;
            }
            append_seeds(x, 0.0f, A.t_seed, act && row >= own_lo && row < own_hi, row, bank, gl, par, sc0);
        }
        if (CMM && cur_ok && A.cm_mode == 2) {
            // thresholded-mean common mode, computed ahead: v = ((u - c1) - c2) - c3
            // replaces u in place and the bank-row's median slot holds 0
            constexpr int G = 64 / L;
            const int grp = lane / L, gl = lane - grp * L;
            const int i = wave * G + grp;
            const bool act = i < BR;
            const int row = act ? i / nb : 0;
            const int bank = act ? i - row * nb : 0;
            float x[V];
#pragma unroll
            for (int v = 0; v < V; ++v) x[v] = INFINITY;
            if (act) {
                const uint32_t grow = (uint32_t)(lr0 + row);  // global row
                const uint32_t reg = A.cm_tile ? grow / (uint32_t)H : grow * (uint32_t)nb + bank;
                const float *cv = A.cm + (f * A.cm_regions + reg) * 3;
                const float c0 = cv[0], c1 = cv[1], c2 = cv[2];
                float *dst = u_c + row * W + bank * B;
                float *f2 = (KEEP && FLAT && row >= own_lo && row < own_hi)
                                ? A.corrected + f * npix + row_base + row * W + bank * B
                                : nullptr;
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    const int c = L * v + gl;
                    if (c < B) {
                        const float u = dst[c];
                        // an invalid pixel (+inf) becomes 0, so that v = 0
                        const float y = __fsub_rn(__fsub_rn(__fsub_rn(u, c0), c1), c2);
                        x[v] = y;
                        dst[c] = (MG && !(u < INFINITY)) ? 0.0f : y;
                        if (f2) f2[c] = y;
                    }
                }
                if (gl == 0) med_c[i] = 0.0f;
            }
            append_seeds(x, 0.0f, A.t_seed, act && row >= own_lo && row < own_hi, row, bank, gl, par, sc0);
        }
        if (!CMM && FLAT && cur_ok && wave * (64 / L) < BR) {  // waves without a bank-row skip the search
            const int gl = lane & (L - 1);
            const bool act = mi < BR;
            const float *src = u_c + moff;
            // every lane reads (inside the u buffers or the LDS that follows
            // them; an inactive group reads row 0) and columns past the bank
            // become +inf; lim is opaque so that the compares stay at the
            // reads rather than as loop-invariant masks
            int lim = B - gl;
            asm volatile("" : "+v"(lim));
            const bool tail_only = B > L * (V - 1);
            float x[V];
            read_group<V, L>(x, src, lim, tail_only, INFINITY);
            const float m = group_median<V, L, false>(x, src, B, kmed, A.rank_width, act, s_gs + tid, B, sides);
            if (act && gl == 0) {
                med_c[mi] = m;
                // kept for patches: the own rows' medians (each row has one owner)
                if (A.meds && mrow >= own_lo && mrow < own_hi)
                    A.meds[f * ((uint64_t)A.T * A.H * nb) + (uint64_t)lr0 * nb + (uint32_t)mi] = m;
            }
            const bool own = act && mrow >= own_lo && mrow < own_hi;
            if (KEEP && own) {
                float *f2 = A.corrected + f * npix + row_base + moff;
#pragma unroll
                for (int v = 0; v < V; ++v)
                    if (L * v < lim) f2[L * v] = __fsub_rn(x[v], m);
            }
            PDC_PHASE(2);
            // slots past the bank (+inf) are no seeds
            append_seeds_dense(x, m, A.t_seed, own, mvmask, mkey0, par, sc0);
        }
        if (!CMM && !FLAT && cur_ok && wave * (64 / L) < BR) {  // waves without a bank-row skip the search
            constexpr int G = 64 / L;
            const int grp = lane / L, gl = lane - grp * L;
            const int i = wave * G + grp;
            const bool act = i < BR;
            const int row = act ? i / nb : 0;
            const int bank = act ? i - row * nb : 0;
            const float *src = u_c + row * W + bank * B;
            // every lane reads (inside the u buffers or the LDS that follows
            // them; an inactive group reads row 0) and columns past the bank
            // become +inf; lim is opaque so that the compares stay here
            // rather than as loop-invariant masks
            int lim = B - gl;
            asm volatile("" : "+v"(lim));
            float x[V];
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const float t = src[L * v + gl];
                x[v] = L * v < lim ? t : INFINITY;
            }
            int nv = B, kq = kmed;
            bool actv = act;
            if constexpr (MG) {
                // the median of the valid values only (invalid ones are +inf)
                int nl = 0;
#pragma unroll
                for (int v = 0; v < V; ++v) nl += x[v] < INFINITY ? 1 : 0;
                nv = gsum_i<L>(nl);
                kq = nv > 0 ? (nv - 1) / 2 : 0;
                actv = act && nv > 0;
            }
            float m = group_median<V, L, MG>(x, src + gl, nv, kq, A.rank_width, actv, s_gs + tid, B, sides);
            if constexpr (MG) {
                if (!actv) m = 0.0f;
                // invalid pixels take the median: v = fl(m - m) = +0
                if (act) {
                    float *dst = u_c + row * W + bank * B;
#pragma unroll
                    for (int v = 0; v < V; ++v) {
                        const int c = L * v + gl;
                        if (c < B && !(x[v] < INFINITY)) dst[c] = m;
                    }
                }
            }
            if (act && gl == 0) {
                med_c[i] = m;
                // kept for patches: the own rows' medians (each row has one owner)
                if (A.meds && row >= own_lo && row < own_hi)
                    A.meds[f * ((uint64_t)A.T * A.H * nb) + (uint64_t)(lr0 + row) * nb + bank] = m;
            }
            append_seeds(x, m, A.t_seed, act && row >= own_lo && row < own_hi, row, bank, gl, par, sc0);
        }
        PDC_PHASE(3);
        if (p1_ok && !ovf_1) {
            // frame f-1's seeds in chunks of 64, claimed by whole waves as they
            // finish their median groups (waves without groups start at once)
            unsigned long long my_ph = 0;
            for (;;) {
                uint32_t c0 = 0;
                if (lane == 0) c0 = atomicAdd(s_p2next, 64u);
                c0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)c0);
                if (c0 >= nseed_1) break;
                const uint32_t j = c0 + lane;
                if (j < nseed_1) {
                    const uint32_t key = s_seed[pp * cap + j];
                    const int row = (int)(key >> 18), bank = (int)((key >> 11) & 127u), col = (int)(key & 2047u);
                    const int i = row * nb + bank;
                    const int cb = col - bank * B;
                    // the 3x3 neighbourhood from the row above and the column
                    // left; the left and right columns take the next bank's
                    // median at a bank edge.  Neighbours outside the loaded
                    // rows, across a tile edge or outside the row are -inf:
                    // never above the seed nor above t_nb.
                    const float *up = u_p + (row - 1) * W + (col - 1);
                    const float *mp = med_p + (row - 1) * nb + bank;
                    const int ml = cb == 0 ? -1 : 0, mr = cb == B - 1 ? 1 : 0;
                    const bool r0 = row >= 1 && row != bnd, r2 = row + 1 < R && row + 1 != bnd;
                    const bool c0 = col >= 1, c2 = col + 1 < W;
                    float nv[3][3];
#pragma unroll
                    for (int dr = 0; dr < 3; ++dr) {
                        const float m0 = mp[dr * nb + ml], m1 = mp[dr * nb], m2 = mp[dr * nb + mr];
                        const bool rin = dr == 1 || (dr == 0 ? r0 : r2);
                        const float a = __fsub_rn(up[dr * W], m0), b = __fsub_rn(up[dr * W + 1], m1),
                                    c = __fsub_rn(up[dr * W + 2], m2);
                        nv[dr][0] = rin && c0 ? a : -INFINITY;
                        nv[dr][1] = rin ? b : -INFINITY;
                        nv[dr][2] = rin && c2 ? c : -INFINITY;
                    }
                    const float vp = nv[1][1];
                    // strictly above the neighbours before it in raster order,
                    // at least the ones after it (ties go to the first)
                    const float me = fmaxf(fmaxf(nv[0][0], nv[0][1]), fmaxf(nv[0][2], nv[1][0]));
                    const float ml2 = fmaxf(fmaxf(nv[1][2], nv[2][0]), fmaxf(nv[2][1], nv[2][2]));
                    const bool is_max = vp > me && vp >= ml2;
                    if (is_max) {
                        float qsum = 0.0f;
#pragma unroll
                        for (int dr = 0; dr < 3; ++dr)
#pragma unroll
                            for (int dc = 0; dc < 3; ++dc)
                                qsum = __fadd_rn(qsum, nv[dr][dc] > A.t_nb ? nv[dr][dc] : 0.0f);
                        atomicOr(&s_bits[(pp * RN + i) * 8 + (cb >> 5)], 1u << (cb & 31));
                        atomicAdd(&s_cnt[pp * RN + i], 1u);
                        my_ph += photon_count(qsum, A.photon_adu);
                        // the hit list (any order; past its end the unit is redone)
                        const uint32_t h = atomicAdd(&s_hcnt[pp], 1u);
                        if (h < (uint32_t)hcap) s_hl[pp * hcap + h] = make_uint2(key, __float_as_uint(qsum));
                    }
                }
            }
            if (my_ph) atomicAdd(&s_photons, my_ph);
        }
        PDC_PHASE(4);
        if (p2_ok && !ovf_2) {
            // frame f-2's hits in raster position (bank-row prefix + hits left
            // of the hit in its bank-row), claimed in chunks of 64 like phase 2
            const uint64_t base = s_base;
            if (base != kNoBase) {
                for (;;) {
                    uint32_t c0 = 0;
                    if (lane == 0) c0 = atomicAdd(s_p4next, 64u);
                    c0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)c0);
                    if (c0 >= nhit_2) break;
                    const uint32_t j = c0 + lane;
                    if (j < nhit_2) {
                        const uint2 e = s_hl[par * hcap + j];
                        const uint32_t key = e.x;
                        const int row = (int)(key >> 18), bank = (int)((key >> 11) & 127u), col = (int)(key & 2047u);
                        const int i = row * nb + bank;
                        const int cb = col - bank * B;
                        const uint32_t *bw = s_bits + (par * RN + i) * 8;
                        uint32_t rank = 0;
                        for (int w = 0; w < (cb >> 5); ++w) rank += __popc(bw[w]);
                        rank += __popc(bw[cb >> 5] & ((1u << (cb & 31)) - 1u));
                        const uint32_t pix = row_base + (uint32_t)row * W + col;
                        A.pool[base + s_pref[i] + rank] = make_uint2(pix, e.y);
                    }
                }
            }
        }
        PDC_PHASE(5);
        lds_barrier();  // B -> next A
        PDC_PHASE(6);
    }
#ifdef PDC_PHASE_TIMERS
    __syncthreads();
    if (threadIdx.x < kV2Waves * 8) atomicAdd(&g_phase_cycles[threadIdx.x], s_tm[threadIdx.x]);
#endif
#undef PDC_PHASE
}

template <int NQ, int GMAX, int L, int V, bool KEEP, bool CMM, bool MG>
__global__ void __launch_bounds__(kV2Threads) __attribute__((amdgpu_waves_per_eu(4, 4))) frame_kernel_v2(V2Args A)
{
    frame_body<NQ, GMAX, L, V, KEEP, CMM, MG>(A, block_item((int)blockIdx.x, (int)gridDim.x));
}

// Several detectors' batches in one launch: the work items of detector d are
// [first[d], first[d + 1]) of the launch (finer frame groups than a launch
// of its own, so that items of unequal cost even out as they are handed
// out), and each workgroup runs the body
// compiled for its detector's lane layout and gain mode (median common mode,
// Frames2 not kept: the variants v2_mix_variant lists).
__global__ void __launch_bounds__(kV2Threads) __attribute__((amdgpu_waves_per_eu(4, 4))) frame_kernel_v2_mix(V2Mix M)
{
    // work items in launch order: consecutive workgroups go to different
    // chiplets, so each chiplet takes a share of every detector's items
    const int item = (int)blockIdx.x;
    int d = 0;
    while (d + 1 < M.n && item >= M.first[d + 1]) ++d;
    // fields are read from the argument memory where they are used (scalar
    // loads, cached): copied into registers up front they would be spilled
    const V2Args &A = M.a[d];
    const int it = item - M.first[d];
    switch (M.variant[d]) {
    case 0: frame_body<2, 4, 16, 13, false, false, false>(A, it); break;
    case 1: frame_body<2, 4, 16, 16, false, false, false>(A, it); break;
    case 2: frame_body<1, 8, 8, 8, false, false, false>(A, it); break;
    case 3: frame_body<1, 8, 8, 12, false, false, false>(A, it); break;
    case 4: frame_body<1, 8, 8, 16, false, false, false>(A, it); break;
    case 5: frame_body<2, 4, 16, 13, false, false, true>(A, it); break;
    case 6: frame_body<2, 4, 16, 16, false, false, true>(A, it); break;
    case 7: frame_body<1, 8, 8, 12, false, false, true>(A, it); break;
    case 8: frame_body<1, 8, 8, 16, false, false, true>(A, it); break;
    default: break;
    }
}

template <int NQ, int GMAX, int L, int V, bool KEEP, bool CMM, bool MG = false>
static hipError_t launch_v2_k(const V2Args &a, uint32_t grid, size_t lds, hipStream_t s)
{
    auto k = frame_kernel_v2<NQ, GMAX, L, V, KEEP, CMM, MG>;
    hipError_t e = hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k, dim3(grid), dim3(kV2Threads), lds, s, a);
    return hipGetLastError();
}

template <int NQ, int GMAX, int L, int V>
static hipError_t launch_v2_t(const V2Args &a, uint32_t grid, size_t lds, bool keep, hipStream_t s)
{
    return keep ? launch_v2_k<NQ, GMAX, L, V, true, false>(a, grid, lds, s)
                : launch_v2_k<NQ, GMAX, L, V, false, false>(a, grid, lds, s);
}

// Lanes per bank-row in the median phase and values per lane (L, V): 16 lanes
// for banks of more than 128 pixels, else 8 (strips hold at most 64 and 128
// bank-rows, so L * bank-rows <= 1024), V = ceil(B / L) rounded up to a
// compiled size.  Four to eight searches per wave and four waves per SIMD
// hide the latency of the reductions.
hipError_t launch_frame_kernel_v2(const V2Args &a, int nq, int gmax, uint32_t grid, size_t lds, bool keep,
                                  hipStream_t s)
{
    if (a.B < 1 || a.rmax * a.nb > 16 * gmax) return hipErrorInvalidValue;
    if (a.gain_mode) {  // auto-ranging variants: one lane layout per strip shape
        const bool cm = a.cm_mode != 0;
        if (nq == 2 && gmax == 4 && a.B <= 256) {
            if (cm) return keep ? launch_v2_k<2, 4, 16, 16, true, true, true>(a, grid, lds, s)
                                : launch_v2_k<2, 4, 16, 16, false, true, true>(a, grid, lds, s);
            if (a.B <= 16 * 13)
                return keep ? launch_v2_k<2, 4, 16, 13, true, false, true>(a, grid, lds, s)
                            : launch_v2_k<2, 4, 16, 13, false, false, true>(a, grid, lds, s);
            return keep ? launch_v2_k<2, 4, 16, 16, true, false, true>(a, grid, lds, s)
                        : launch_v2_k<2, 4, 16, 16, false, false, true>(a, grid, lds, s);
        }
        if (nq == 1 && gmax == 8 && a.B <= 128) {
            if (cm) return keep ? launch_v2_k<1, 8, 8, 16, true, true, true>(a, grid, lds, s)
                                : launch_v2_k<1, 8, 8, 16, false, true, true>(a, grid, lds, s);
            if (a.B <= 8 * 12)
                return keep ? launch_v2_k<1, 8, 8, 12, true, false, true>(a, grid, lds, s)
                            : launch_v2_k<1, 8, 8, 12, false, false, true>(a, grid, lds, s);
            return keep ? launch_v2_k<1, 8, 8, 16, true, false, true>(a, grid, lds, s)
                        : launch_v2_k<1, 8, 8, 16, false, false, true>(a, grid, lds, s);
        }
        return hipErrorInvalidValue;
    }
    if (a.cm_mode) {  // the thresholded-mean variant: no median search
        if (nq == 2 && gmax == 4 && a.B <= 256)
            return keep ? launch_v2_k<2, 4, 16, 16, true, true>(a, grid, lds, s)
                        : launch_v2_k<2, 4, 16, 16, false, true>(a, grid, lds, s);
        if (nq == 1 && gmax == 8 && a.B <= 128)
            return keep ? launch_v2_k<1, 8, 8, 16, true, true>(a, grid, lds, s)
                        : launch_v2_k<1, 8, 8, 16, false, true>(a, grid, lds, s);
        return hipErrorInvalidValue;
    }
    if (nq == 2 && gmax == 4 && a.B <= 256) {
        if (a.B <= 16 * 13) return launch_v2_t<2, 4, 16, 13>(a, grid, lds, keep, s);
        return launch_v2_t<2, 4, 16, 16>(a, grid, lds, keep, s);
    }
    if (nq == 1 && gmax == 8 && a.B <= 128) {
        if (a.B <= 8 * 8) return launch_v2_t<1, 8, 8, 8>(a, grid, lds, keep, s);
        if (a.B <= 8 * 12) return launch_v2_t<1, 8, 8, 12>(a, grid, lds, keep, s);
        return launch_v2_t<1, 8, 8, 16>(a, grid, lds, keep, s);
    }
    return hipErrorInvalidValue;
}

int v2_mix_variant(const V2Args &a, int nq, int gmax, bool keep)
{
    if (keep || a.cm_mode || a.meds || a.B < 1 || a.rmax * a.nb > 16 * gmax) return -1;
    const int mg = a.gain_mode ? 5 : 0;
    if (nq == 2 && gmax == 4 && a.B <= 256) return a.B <= 16 * 13 ? mg : mg + 1;
    if (nq == 1 && gmax == 8 && a.B <= 128) {
        if (a.B <= 8 * 8 && !a.gain_mode) return 2;
        return a.B <= 8 * 12 ? (a.gain_mode ? 7 : 3) : (a.gain_mode ? 8 : 4);
    }
    return -1;
}

size_t frame_kernel_v2_mix_static_lds()
{
    hipFuncAttributes fa{};
    if (hipFuncGetAttributes(&fa, (const void *)frame_kernel_v2_mix) != hipSuccess) return SIZE_MAX;
    return fa.sharedSizeBytes;
}

hipError_t launch_frame_kernel_v2_mix(const V2Mix &m, size_t lds, hipStream_t s)
{
    if (m.n < 1 || m.n > kMixMax) return hipErrorInvalidValue;
    for (int d = 0; d < m.n; ++d)
        if (m.variant[d] < 0 || m.first[d + 1] < m.first[d]) return hipErrorInvalidValue;
    const uint32_t grid = (uint32_t)m.first[m.n];
    if (grid == 0) return hipSuccess;
    hipError_t e = hipFuncSetAttribute((const void *)frame_kernel_v2_mix, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(frame_kernel_v2_mix, dim3(grid), dim3(kV2Threads), lds, s, m);
    return hipGetLastError();
}

}  // namespace pdc

#ifdef PDC_PHASE_TIMERS
// Tracing build only: copy the phase cycles of every launch since the last
// call to out[kV2Waves * 8] and clear them (synchronous).
extern "C" int pdc_debug_phase_cycles(unsigned long long *out)
{
    if (!out) return -1;
    if (hipDeviceSynchronize() != hipSuccess) return -3;
    if (hipMemcpyFromSymbol(out, HIP_SYMBOL(pdc::g_phase_cycles), sizeof(unsigned long long) * pdc::kV2Waves * 8) !=
        hipSuccess)
        return -3;
    static unsigned long long z[pdc::kV2Waves * 8];
    if (hipMemcpyToSymbol(HIP_SYMBOL(pdc::g_phase_cycles), z, sizeof z) != hipSuccess) return -3;
    return 0;
}
#endif
