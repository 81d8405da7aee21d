/*
 * pdc_oracle.c -- plain CPU oracle for pixel-detector correction and photon
 * finding.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links or calls this
 * file; only the tests, the smoke check and the benchmark's CPU-baseline leg
 * do.  It shares no code, header or constant with the GPU library.
 *
 * It is deliberately slow and obvious: single-precision IEEE-754 arithmetic
 * (binary32, round to nearest even, every operation rounded on its own; build
 * with -ffp-contract=off and without -ffast-math), one frame at a time, loops
 * in a fixed order, the bank median by a full sort.
 *
 * Processing of one frame, following the paper's pipeline (Fig. a: dark, gain,
 * common mode, charge summing, photon counting, summary):
 *
 *   1. adc = raw & 0x3FFF                      14-bit ADC value
 *   2. t   = (float)adc - dark[p]              dark subtraction (Fig. b, "-")
 *   3. u   = t * k[p],  k[p] = 1.0f / gain[p]  gain correction (Fig. b, "/");
 *                                              the reciprocal is formed once per
 *                                              pixel, then multiplied
 *   4. m   = element of rank (B-1)/2 of the B values u of a bank (one row of B
 *            contiguous columns of a tile): the lower median.  The paper's
 *            common-mode section allows row/column/block common modes; the
 *            estimator here is the bank median.
 *   5. v   = u - m                             common-mode subtraction (Fig. c,
 *                                              "Frames2 = Frames1 - CM")
 *   6. p is a photon hit iff v[p] > T_seed and p beats each neighbour q of
 *      its 3x3 window inside the same tile: v[p] > v[q], or v[p] == v[q] and
 *      p < q (raster order).  The cloud's charge goes to its highest pixel
 *      (charge summing section).
 *   7. q_p = sum over the in-tile 3x3 window, rows top to bottom, columns left
 *      to right, starting from +0.0f, of (v[j] > T_nb ? v[j] : 0): pixels
 *      within noise are zeroed before summing (Fig. e "Signal" mask; subpixel
 *      section, zeroing of in-noise pixels).
 *   8. n_p = rint(q_p / E) (ties to even), E = single-photon signal: photon
 *      counting by division with the single-photon gain and rounding to the
 *      nearest integer (charge summing section).  Saturates at 2^32-1.
 *   9. hits are listed in (frame, pixel) order; per-frame hit counts and
 *      photon totals (summarization section: sparse photon lists).
 *
 * T_seed = n_seed * sigma and T_nb = n_nb * sigma are formed in binary32.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    uint32_t frame;   /* batch-relative frame index */
    uint32_t pixel;   /* (tile * rows + row) * cols + col */
    float charge;     /* q_p */
    uint32_t nphot;   /* n_p */
} oracle_hit;

/* Steps 1-3 on npix pixels: Frames1 = (adc - dark) * (1 / gain). */
void oracle_dark_gain(const uint16_t *raw, const float *dark, const float *gain,
                      int64_t npix, float *frames1)
{
    for (int64_t p = 0; p < npix; ++p) {
        float k = 1.0f / gain[p];
        float a = (float)(raw[p] & 0x3FFF);
        float t = a - dark[p];
        frames1[p] = t * k;
    }
}

static int cmp_float(const void *pa, const void *pb)
{
    float a = *(const float *)pa, b = *(const float *)pb;
    if (a < b) return -1;
    if (a > b) return 1;
    return 0;
}

/* Step 4: lower median of every bank.  medians[(t*H + r)*(W/B) + b]. */
void oracle_bank_medians(const float *frames1, int32_t T, int32_t H, int32_t W,
                         int32_t B, float *medians)
{
    float *tmp = (float *)malloc(sizeof(float) * (size_t)B);
    int32_t nb = W / B;
    for (int32_t t = 0; t < T; ++t)
        for (int32_t r = 0; r < H; ++r)
            for (int32_t b = 0; b < nb; ++b) {
                const float *row = frames1 + ((int64_t)t * H + r) * W + (int64_t)b * B;
                memcpy(tmp, row, sizeof(float) * (size_t)B);
                qsort(tmp, (size_t)B, sizeof(float), cmp_float);
                medians[((int64_t)t * H + r) * nb + b] = tmp[(B - 1) / 2];
            }
    free(tmp);
}

/* Steps 4-5: Frames2 = Frames1 - (bank median). */
void oracle_common_mode(const float *frames1, int32_t T, int32_t H, int32_t W,
                        int32_t B, float *frames2)
{
    int32_t nb = W / B;
    float *med = (float *)malloc(sizeof(float) * (size_t)T * H * nb);
    oracle_bank_medians(frames1, T, H, W, B, med);
    for (int32_t t = 0; t < T; ++t)
        for (int32_t r = 0; r < H; ++r)
            for (int32_t c = 0; c < W; ++c) {
                int64_t p = ((int64_t)t * H + r) * W + c;
                frames2[p] = frames1[p] - med[((int64_t)t * H + r) * nb + c / B];
            }
    free(med);
}

/* Step 8. */
static uint32_t photon_count(float q, float photon_adu)
{
    float x = q / photon_adu;
    if (x >= 4294967296.0f) return 0xFFFFFFFFu;
    return (uint32_t)rintf(x);
}

/* Steps 6-8 on one corrected frame; hits appended in raster order.
 * Returns the number of hits found (all of them are counted; at most
 * cap - *n_out are stored). */
int64_t oracle_find_hits(const float *v, int32_t T, int32_t H, int32_t W,
                         float t_seed, float t_nb, float photon_adu, uint32_t frame,
                         oracle_hit *out, int64_t cap, int64_t *n_out,
                         uint64_t *photons_out)
{
    int64_t found = 0;
    uint64_t photons = 0;
    for (int32_t t = 0; t < T; ++t)
        for (int32_t r = 0; r < H; ++r)
            for (int32_t c = 0; c < W; ++c) {
                int64_t p = ((int64_t)t * H + r) * W + c;
                float vp = v[p];
                if (!(vp > t_seed)) continue;
                int is_max = 1;
                for (int dr = -1; dr <= 1 && is_max; ++dr)
                    for (int dc = -1; dc <= 1; ++dc) {
                        if (dr == 0 && dc == 0) continue;
                        int32_t rr = r + dr, cc = c + dc;
                        if (rr < 0 || rr >= H || cc < 0 || cc >= W) continue;
                        int64_t q = ((int64_t)t * H + rr) * W + cc;
                        float vq = v[q];
                        int beats = (vp > vq) || (vp == vq && p < q);
                        if (!beats) { is_max = 0; break; }
                    }
                if (!is_max) continue;
                float qsum = 0.0f;
                for (int dr = -1; dr <= 1; ++dr)
                    for (int dc = -1; dc <= 1; ++dc) {
                        int32_t rr = r + dr, cc = c + dc;
                        if (rr < 0 || rr >= H || cc < 0 || cc >= W) continue;
                        float vj = v[((int64_t)t * H + rr) * W + cc];
                        qsum = qsum + (vj > t_nb ? vj : 0.0f);
                    }
                uint32_t n = photon_count(qsum, photon_adu);
                photons += n;
                if (*n_out < cap) {
                    out[*n_out].frame = frame;
                    out[*n_out].pixel = (uint32_t)p;
                    out[*n_out].charge = qsum;
                    out[*n_out].nphot = n;
                    *n_out += 1;
                }
                ++found;
            }
    if (photons_out) *photons_out = photons;
    return found;
}

/* Whole batch.  raw: uint16 [n_frames][T][H][W]; dark, gain: float [T][H][W].
 * hits: room for hit_cap records, *n_hits = records stored.
 * frame_hits[n_frames], frame_photons[n_frames]: per-frame totals (all hits).
 * corrected (may be NULL): Frames2, float [n_frames][T][H][W].
 * Returns the total number of hits (stored or not). */
int64_t oracle_process(const uint16_t *raw, int64_t n_frames, int32_t T, int32_t H,
                       int32_t W, int32_t B, const float *dark, const float *gain,
                       float sigma, float n_seed, float n_nb, float photon_adu,
                       oracle_hit *hits, int64_t hit_cap, int64_t *n_hits,
                       uint32_t *frame_hits, uint64_t *frame_photons, float *corrected)
{
    int64_t npix = (int64_t)T * H * W;
    float t_seed = n_seed * sigma;
    float t_nb = n_nb * sigma;
    float *f1 = (float *)malloc(sizeof(float) * (size_t)npix);
    float *f2 = (float *)malloc(sizeof(float) * (size_t)npix);
    int64_t total = 0;
    *n_hits = 0;
    for (int64_t f = 0; f < n_frames; ++f) {
        oracle_dark_gain(raw + f * npix, dark, gain, npix, f1);
        oracle_common_mode(f1, T, H, W, B, f2);
        if (corrected) memcpy(corrected + f * npix, f2, sizeof(float) * (size_t)npix);
        uint64_t ph = 0;
        int64_t nf = oracle_find_hits(f2, T, H, W, t_seed, t_nb, photon_adu, (uint32_t)f,
                                      hits, hit_cap, n_hits, &ph);
        if (frame_hits) frame_hits[f] = (uint32_t)nf;
        if (frame_photons) frame_photons[f] = ph;
        total += nf;
    }
    free(f1);
    free(f2);
    return total;
}
