// Internal interfaces between the host runtime (pdc_runtime.cpp) and the HIP
// kernels (pdc_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pdc {

// Sentinel for "this unit's hits could not be staged" (staging pool full).
constexpr uint64_t kNoBase = ~0ull;

// Waves per workgroup of the persistent kernel; 16 / kV2Waves workgroups
// share a compute unit (its LDS split between them, four waves per SIMD).
#ifndef PDC_V2_WAVES
#define PDC_V2_WAVES 16
#endif
constexpr int kV2Waves = PDC_V2_WAVES;
constexpr int kV2Threads = kV2Waves * 64;
constexpr int kV2GroupsPerCu = 16 / kV2Waves;
// Staging chunk claimed by one workgroup from the batch-wide pool cursor.
constexpr uint64_t kChunkHits = 8192;

// Device-side batch state, cleared by init_state before each run.
struct BatchState {
    unsigned long long cursor;    // next free staging slot
    unsigned int overflow;        // 1 if some unit could not be staged
    unsigned int fallback;        // 1 if the fast kernel left some unit to the general kernel
    unsigned long long total;     // total hits of the batch (set by the frame scan)
    unsigned long long n_fallback;  // units listed in the batch's fallback list
};

// Persistent kernel (v2): a strip owns frame rows [g0, g1), counted over all
// tiles (global row t * H + r), and loads rows [lg0, lg1): one halo row on
// each side that lies in the same tile.  A strip may cross one tile edge, at
// global row gb (a multiple of H; INT32_MAX if none): rows on either side of
// it are not neighbours.
struct V2Strip {
    int32_t lg0, lg1, g0, g1, gb, pad0, pad1, pad2;
};

// A work unit is (frame, strip): rows [r0, r0 + strip_rows) of one tile.
// Units are numbered frame-major, then tile, then strip, which is raster order
// of their pixels.
struct FrameKernelArgs {
    const uint16_t *frames;       // [n_frames][T][H][W]
    const float *ped;             // [T][H][W]
    const float *k;               // [T][H][W], k = 1/gain
    uint64_t n_frames;
    uint64_t n_units;
    int32_t T, H, W, B, nb;       // geometry; nb = W / B
    int32_t strip_rows;           // rows per strip
    int32_t strips_per_tile;
    int32_t units_per_frame;      // T * strips_per_tile
    int32_t sort_width;           // power of two >= B
    int32_t sort_rows;            // rows sorted together (v1)
    uint32_t max_unit_hits;       // upper bound on hits of one unit
    float t_seed, t_nb, photon_adu;
    uint2 *pool;                  // staging: {pixel, charge bits}
    uint64_t pool_cap;
    uint32_t *unit_count;         // [n_units]
    unsigned long long *unit_photons;  // [n_units]
    uint64_t *unit_base;          // [n_units] staging start or kNoBase
    BatchState *state;
    float *corrected;             // Frames2 or nullptr
    // unit-list mode: recompute only units unit_list[0..n_list) whose rows come
    // from the persistent kernel's strip table (units_per_frame = its strips)
    const uint64_t *unit_list;
    uint64_t n_list;
    const V2Strip *strips;
    const float *cm;              // thresholded-mean mode: [n_frames][cm_regions][3], else nullptr
    uint32_t cm_regions;          // regions per frame: banks (T*H*nb) or tiles (T)
    int32_t cm_tile;              // 1: a region is a tile, 0: a bank
    int32_t gain_mode;            // 0 single range; 1, 2 auto-ranging (ped, k hold 3 planes)
    uint32_t *invalid;            // [n_frames] invalid-code pixels, cleared before the launch
    float *meds;                  // [n_frames][T*H*nb] bank medians of the own rows, or nullptr
};

struct V2Args {
    const uint16_t *frames;
    const float *ped;
    const float *k;
    uint64_t n_frames;
    int32_t T, H, W, B, nb;
    int32_t n_strips;             // strips per frame
    int32_t n_fgroups;            // frame groups (frames split into contiguous ranges)
    int32_t rmax;                 // max loaded rows of a strip (own rows + halos)
    int32_t seed_cap;             // seeds per strip-frame held in LDS
    const V2Strip *strips;        // [n_strips], raster order
    float t_seed, t_nb, photon_adu;
    float rank_width;             // expected value spacing near a bank median (ADU per rank)
    uint2 *pool;
    uint64_t pool_cap;
    uint32_t *unit_count;
    unsigned long long *unit_photons;
    uint64_t *unit_base;
    BatchState *state;
    float *corrected;
    uint64_t *fb_units;           // units left to the general kernel (seed lists full), or nullptr
    const float *cm;              // as in FrameKernelArgs (cm_mode 2)
    uint32_t cm_regions;
    int32_t cm_tile;
    int32_t cm_mode;              // 0 median; 1 bank thresholded mean computed in the kernel;
                                  // 2 thresholded-mean stage values read from cm
    int32_t cm_stages;            // cm_mode 1: stages, noise threshold and guard
    float t_cm, cm_guard;
    int32_t sum_lo, sum_hi;       // cm_mode 1: Frames1 values are multiples of 2^sum_lo below 2^sum_hi
    int32_t gain_mode;
    uint32_t *invalid;
    float *meds;                  // as in FrameKernelArgs (median mode)
    int32_t med_row_step;         // single-gain median kernels with 16-lane groups: 4 when one
                                  // wave's four groups take every fourth row, else 0
};

size_t frame_kernel_v2_lds_bytes(int rmax, int W, int nb, int seed_cap);
// Several detectors' batches in one launch of the persistent kernel: the
// work items (strip, frame group) of detector d are [first[d], first[d + 1]).
constexpr int kMixMax = 8;
struct V2Mix {
    V2Args a[kMixMax];
    int32_t variant[kMixMax];     // from v2_mix_variant
    int32_t first[kMixMax + 1];
    int32_t n;
};
static_assert(sizeof(V2Mix) <= 4096, "V2Mix is passed as a kernel argument");
// The compiled body of the one launch for a batch, or -1 when it has none
// (Frames2 or common-mode values kept, thresholded mean): such batches take
// launches of their own.
int v2_mix_variant(const V2Args &a, int nq, int gmax, bool keep);
// Dynamic LDS lds: at least the largest v2 LDS of the detectors.
hipError_t launch_frame_kernel_v2_mix(const V2Mix &m, size_t lds, hipStream_t s);
// Static LDS of that kernel (every body's own variables), SIZE_MAX if unknown.
size_t frame_kernel_v2_mix_static_lds();
// a.cm_mode != 0 selects the thresholded-mean variant (no median search)
hipError_t launch_frame_kernel_v2(const V2Args &a, int nq, int gmax, uint32_t grid, size_t lds, bool keep,
                                  hipStream_t s);

// Thresholded-mean common mode (Fig. c), computed ahead of the frame kernels:
// cm[f][region][s] for stages s < stages, zeros after.  A region's sum is the
// exact sum of its noise pixels rounded once to binary32.
struct CmArgs {
    const uint16_t *frames;       // [n_frames][T][H][W]
    const float *ped, *k;         // [T][H][W]
    uint64_t n_frames;
    int32_t T, H, W, B, nb;
    int32_t stages;               // 1..3
    float t_cm;                   // pixels below it are noise
    float guard;                  // fl(sqrt(fl(region size)))
    int32_t sum_lo, sum_hi;       // Frames1 values are multiples of 2^sum_lo below 2^sum_hi
    int32_t gain_mode;            // as in FrameKernelArgs
    float *cm;
};
hipError_t launch_cm_bank(const CmArgs &a, uint32_t n_cu, hipStream_t s);
hipError_t launch_cm_tile(const CmArgs &a, uint32_t n_cu, hipStream_t s);

size_t frame_kernel_v1_lds_bytes(int strip_rows, int W, int nb, int sort_width, int sort_rows,
                                 uint32_t max_unit_hits);

hipError_t launch_init_state(BatchState *state, hipStream_t s);
hipError_t launch_frame_kernel_v1(const FrameKernelArgs &a, uint32_t grid, size_t lds_bytes,
                                  bool keep_corrected, hipStream_t s);
// Per frame: in-frame exclusive offsets of units, hit counts and photon totals.
hipError_t launch_frame_sums(const uint32_t *unit_count, const unsigned long long *unit_photons,
                             uint64_t n_frames, int32_t units_per_frame, uint32_t *unit_local,
                             uint32_t *frame_hits, unsigned long long *frame_photons,
                             hipStream_t s);
// Exclusive scan of frame hit counts: frame_offset[0..n_frames], total into state.
hipError_t launch_frame_scan(const uint32_t *frame_hits, uint64_t n_frames,
                             unsigned long long *frame_offset, BatchState *state, hipStream_t s);
// Copy each unit's staged hits to its place in the raster-order list.
hipError_t launch_scatter(const uint32_t *unit_count, const uint64_t *unit_base,
                          const uint32_t *unit_local, const unsigned long long *frame_offset,
                          const uint2 *pool, uint64_t n_units, int32_t units_per_frame,
                          uint2 *hits, uint64_t hits_cap, hipStream_t s);

// The 16-byte hit record of the public ABI.
struct HitRecord {
    uint32_t frame, pixel;
    float charge;
    uint32_t nphot;
};
// The staged runs straight into records at their raster positions (first
// out_cap of them).
hipError_t launch_scatter_records(const uint32_t *unit_count, const uint64_t *unit_base,
                                  const uint32_t *unit_local, const unsigned long long *frame_offset,
                                  const uint2 *pool, uint64_t n_units, int32_t units_per_frame, float photon_adu,
                                  HitRecord *out, uint64_t out_cap, hipStream_t s);
// Expand hits [first, first + n) of the raster-order list into records.
hipError_t launch_format_hits(const uint2 *hits, const unsigned long long *frame_offset,
                              uint64_t n_frames, uint64_t first, uint64_t n, float photon_adu,
                              HitRecord *out, hipStream_t s);

}  // namespace pdc
