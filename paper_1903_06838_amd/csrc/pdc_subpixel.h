// Internal launchers of the subpixel stage (pdc_subpixel.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pdc {

// Parameter vector of the 25-64-64-2 network, float32, in this order:
// W1[25][64], b1[64], W2[64][64], b2[64], W3[64][2], b3[2].
constexpr int kMlpIn = 25, kMlpHidden = 64, kMlpOut = 2;
constexpr int kMlpParams = 25 * 64 + 64 + 64 * 64 + 64 + 64 * 2 + 2;  // 5954
constexpr int kOffW1 = 0, kOffB1 = 1600, kOffW2 = 1664, kOffB2 = 5760, kOffW3 = 5824, kOffB3 = 5952;
// A hit's network input: 25 bf16 words, then 7 zeros (64 bytes).
constexpr int kMlpInWords = 32;

// bfloat16 copies of the weights in the layouts the MFMA operand loads want
// (each row holds the contraction index contiguously):
//   w1t[64][32]  = W1^T, columns 25..31 zero        (forward, layer 1)
//   w2t[64][64]  = W2^T                               (forward, layer 2)
//   w2 [64][64]  = W2                                 (backward, dH1 = dH2 W2^T)
//   w3t[16][64]  = W3^T, rows 2..15 zero             (forward, layer 3)
//   w3p[64][32]  = W3, columns 2..31 zero             (backward, dH2 = dY W3^T)
constexpr int kPackW1t = 0, kPackW2t = 2048, kPackW2 = 6144, kPackW3t = 10240, kPackW3p = 11264;
constexpr int kPackElems = 13312;  // bf16 elements (26 KiB)

hipError_t launch_fill_zero(float *p, uint64_t n, hipStream_t s);
hipError_t launch_centroid_eta(const float *patches, uint64_t n, float t_nb, const float *eta, int nbins,
                               float *out, hipStream_t s);
hipError_t launch_eta_table(const float *patches, uint64_t n, float t_nb, int nbins, uint32_t *hist,
                            float *table, hipStream_t s);
hipError_t launch_mlp_pack(const float *theta, uint16_t *packed, hipStream_t s);
hipError_t launch_mlp_infer(const float *patches, uint64_t n, float inv_adu, const float *theta,
                            const uint16_t *packed, float *out, uint32_t max_grid, hipStream_t s);
// The same on the network's inputs (uint16 [n][kMlpInWords]).
hipError_t launch_mlp_infer_inputs(const uint16_t *inputs, uint64_t n, const float *theta, const uint16_t *packed,
                                   float *out, uint32_t max_grid, hipStream_t s);
// Gradient of sum((y - t)^2) / (2 n) over n hits: out[0..kMlpParams) gets the
// gradient, out[kMlpParams] gets sum((y - t)^2).  Each wave writes its partial
// sums to a slot of kMlpSlotStride floats; slots must hold
// mlp_grad_grid(n, max_grid) * 4 slots.  The result is deterministic.
constexpr int kMlpSlotStride = 5960;
uint32_t mlp_grad_grid(uint64_t n, uint32_t max_grid);
hipError_t launch_mlp_grad(const float *patches, const float *target, uint64_t n, float inv_adu,
                           const float *theta, const uint16_t *packed, float *out, float *slots, uint32_t max_grid,
                           hipStream_t s);
// One training step: the gradient of n >= 1 hits into the slots, then one
// kernel that sums them (grad[0..kMlpParams]), takes the Adam step (step >= 1)
// and refreshes the packed bf16 weights.
hipError_t launch_mlp_train(const float *patches, const float *target, uint64_t n, float inv_adu, float *theta,
                            float *m, float *v, uint16_t *packed, float *grad, float *slots, uint32_t max_grid,
                            float lr, int64_t step, hipStream_t s);
// patches float32 [n][25], or, when inputs is not NULL, the network's inputs
// uint16 [n][kMlpInWords] (bf16 of each value times inv_adu, zero padding)
hipError_t launch_capture_patches(const float *corrected, const uint2 *hits,
                                  const unsigned long long *frame_offset, uint64_t n_frames, uint64_t n, int T,
                                  int H, int W, float *patches, uint16_t *inputs, float inv_adu, hipStream_t s);
// Patches rebuilt from the frames: Frames2 of each window pixel from its raw
// word, the calibration and the frame's kept common-mode values (meds: bank
// medians [n_frames][T*H*nb]; or, with meds null, the thresholded mean's
// stage values cm [n_frames][cm_regions][3]).
struct PatchSrc {
    const uint16_t *frames;
    const float *ped, *k;
    int32_t T, H, W, B, nb, gain_mode;
    const float *meds;
    const float *cm;
    uint32_t cm_regions;
    int32_t cm_tile;
};
hipError_t launch_patches_from_frames(const PatchSrc &a, const uint2 *hits, const unsigned long long *frame_offset,
                                      uint64_t n_frames, uint64_t n, float *patches, uint16_t *inputs, float inv_adu,
                                      hipStream_t s);
// Centroid (+ eta) positions of the first n hits of a batch, from Frames2
// (corrected != NULL) or formed again from the frames (a); only_bad: replace
// only the positions in pos that are not finite or outside [-1, 1].
hipError_t launch_centroids(const PatchSrc &a, const float *corrected, const uint2 *hits,
                            const unsigned long long *frame_offset, uint64_t n_frames, uint64_t n, float t_nb,
                            const float *eta, int nbins, int only_bad, float *pos, hipStream_t s);
// The network's inputs of n float32 patches.
hipError_t launch_make_inputs(const float *patches, uint64_t n, float inv_adu, uint16_t *inputs, hipStream_t s);
hipError_t launch_mfma_probe(const uint16_t *A, const uint16_t *B, float *D, hipStream_t s);

}  // namespace pdc
