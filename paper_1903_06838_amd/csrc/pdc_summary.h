// Internal launchers of the summaries (pdc_summary.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pdc {

// Histograms of up to this many bins are gathered in LDS per workgroup (48 KiB
// at most: three such workgroups share a CU).
constexpr uint64_t kLdsBins = 12288;
// Frames one thread sums for the dark statistics (keeps its 32-bit sum exact).
constexpr uint64_t kDarkChunkMax = 1ull << 18;

struct AccumulateArgs {
    const uint2 *hits;                     // raster-order list {pixel, charge bits}
    uint64_t n;                            // hits
    float photon_adu;
    uint32_t *count_map;                   // [pixels per frame] or nullptr
    uint32_t *spectrum;                    // [nbins + 2] or nullptr
    uint32_t *size_spectra;                // [9][nbins + 2] or nullptr (needs corrected)
    float lo, scale;                       // scale = nbins / (hi - lo) in binary32
    uint32_t nbins;
    const float *corrected;                // Frames2 [n_frames][T][H][W]
    const unsigned long long *frame_offset;  // [n_frames + 1]
    uint64_t n_frames;
    int32_t T, H, W;
    float t_nb;
};

hipError_t launch_fill_u32(uint32_t *p, uint64_t n, hipStream_t s);
// Read bytes (a multiple of 16, 16-byte aligned) from src once; *out receives
// an XOR of everything read.
hipError_t launch_stream_read(const void *src, uint64_t bytes, uint32_t *out, uint32_t n_cu, hipStream_t s);
bool accumulate_uses_lds(const AccumulateArgs &a);
hipError_t launch_accumulate_hits(const AccumulateArgs &a, uint32_t max_grid, hipStream_t s);
hipError_t launch_histogram(const float *x, uint64_t n, float lo, float scale, uint32_t nbins, uint32_t *hist,
                            uint32_t max_grid, hipStream_t s);
// s1, s2: [px] sums over the frames, cleared by this call.
hipError_t launch_dark_sums(const uint16_t *d, uint64_t n_frames, uint64_t px, unsigned long long *s1,
                            unsigned long long *s2, uint32_t n_cu, hipStream_t s);

}  // namespace pdc
