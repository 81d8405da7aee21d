// Host runtime of libpdc: contexts, resident calibration, batches, buffers and
// the C ABI declared in include/pdc.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <set>
#include <string>
#include <vector>

#include "pdc.h"
#include "pdc_internal.h"
#include "pdc_subpixel.h"
#include "pdc_summary.h"

using namespace pdc;

namespace {

thread_local char g_thread_error[512] = "";

// Device scratch of pdc_process_frames_static, for callers that cannot
// allocate: a file-scope device array, one copy per GPU for as long as the
// process lives.  Host code never uses the array's name as an address; its
// address on each device comes from hipGetSymbolAddress, taken once per
// device by pdc_create with that device current.
constexpr uint64_t kStaticScratchBytes = PDC_STATIC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];
std::mutex g_scratch_mu;
unsigned char *g_scratch_ptr[kMaxDevices] = {};

// LDS budget of the v1 frame kernel (bytes per workgroup).
constexpr size_t kV1LdsBudget = 64 * 1024;
constexpr int kMaxOutstandingBatches = 256;

struct Detector {
    bool live = false;
    pdc_geometry g{};
    pdc_params p{};
    float t_seed = 0, t_nb = 0;
    float t_cm = 0, cm_guard = 0;         // thresholded-mean common mode (cm_mode 1 or 2)
    uint32_t cm_regions = 0;              // regions per frame
    int32_t sum_lo = 0, sum_hi = 0;       // window of Frames1: multiples of 2^sum_lo below 2^sum_hi
    float *d_ped = nullptr;
    float *d_k = nullptr;
    // derived launch shape of the general kernel (v1)
    int strip_rows = 0, strips_per_tile = 0, units_per_frame = 0, sort_width = 0, sort_rows = 0;
    uint32_t max_unit_hits = 0;
    size_t lds_bytes = 0;
    // persistent kernel (v2): resident calibration per strip
    bool v2_ok = false;
    int nq = 0, gmax = 0, n_strips = 0, rmax = 0, seed_cap = 0;
    int n_cu = 0;                         // compute units of the device (frame-group choice)
    int fg_mult = 1;                      // frame groups x this (pdc_autotune)
    int strip_cap = 0;                    // own rows per strip at most this (0: as many as fit; pdc_autotune_strips)
    uint32_t v2_max_unit_hits = 0;
    size_t v2_lds = 0;
    float rank_width = 0;
    // general kernel over persistent-kernel strips, for units whose seed lists overflowed
    bool fb_ok = false;
    int fb_strip_rows = 0, fb_sort_rows = 0;
    size_t fb_lds = 0;
    V2Strip *d_strips = nullptr;
    int pending = 0;
    bool release_requested = false;
};

// Device buffers of one batch; kept by the context and reused.
struct Buffers {
    uint64_t cap_units = 0, cap_frames = 0, cap_pool = 0, cap_corr = 0;
    uint32_t *unit_count = nullptr;
    unsigned long long *unit_photons = nullptr;
    uint64_t *unit_base = nullptr;
    uint32_t *unit_local = nullptr;
    uint32_t *frame_hits = nullptr;
    unsigned long long *frame_photons = nullptr;
    unsigned long long *frame_offset = nullptr;
    uint2 *pool = nullptr;
    uint2 *hits = nullptr;
    float *corrected = nullptr;
    float *cm = nullptr;               // [n_frames][regions][3] common-mode values
    uint64_t cap_cm = 0;
    float *meds = nullptr;             // [n_frames][bank-rows] medians (PDC_KEEP_MEDIANS)
    uint64_t cap_meds = 0;
    uint32_t *invalid = nullptr;       // [n_frames] pixels with an invalid gain code
    uint64_t cap_inv = 0;
    uint64_t *fb_units = nullptr;      // [n_units] units left to the general kernel
    uint64_t cap_fb = 0;
    BatchState *state = nullptr;
    BatchState *host_state = nullptr;  // pinned mirror
    hipEvent_t ev_start = nullptr, ev_main = nullptr, ev_end = nullptr;
    hipEvent_t ev_cm = nullptr;     // after the common-mode pass (thresholded-mean mode)
    hipEvent_t ev_state = nullptr;  // after the state copy: the batch's last work on its stream
    hipEvent_t ev_use = nullptr;    // after summary work on a caller's stream
    bool used = false;              // ev_use recorded since the batch was launched
};

struct Batch {
    uint64_t id = 0;
    int32_t det = -1;
    int path = 1;            // 1: general kernel, 2: persistent kernel
    int n_fg = 1;            // frame groups (path 2)
    double share = 1.0;      // fraction of the chip's compute units the batch is sized for
    int32_t upf = 0;         // units per frame
    const uint16_t *frames = nullptr;
    uint64_t n_frames = 0;
    uint64_t n_units = 0;
    uint64_t pool_cap = 0;
    hipStream_t stream = nullptr;
    bool keep = false;
    bool meds = false;       // PDC_KEEP_MEDIANS: common-mode values kept for patches
    bool checked = false;  // overflow handled, totals final
    int fb = 0;            // 1: overflowing units recomputed by the general kernel, 2: whole batch
    bool capture = false;  // being captured into a graph: kernels only, no events or copies
    bool mix_one = false;  // its frame kernel ran in one launch with the other batches of a mixed call
    int fg_more = 1;       // frame groups x this beyond the detector's choice (one-launch mixed calls)
    pdc_graph *graph = nullptr;  // launched from this graph, whose buffers it holds
    int gitem = 0;               // its item in that graph
    Buffers *buf = nullptr;
    HitRecord *records = nullptr;  // pdc_process_frames_static: hits go straight to these records
    uint64_t records_cap = 0;
};

void free_buffers(Buffers *b)
{
    if (!b) return;
    hipFree(b->unit_count);
    hipFree(b->unit_photons);
    hipFree(b->unit_base);
    hipFree(b->unit_local);
    hipFree(b->frame_hits);
    hipFree(b->frame_photons);
    hipFree(b->frame_offset);
    hipFree(b->pool);
    hipFree(b->hits);
    hipFree(b->corrected);
    hipFree(b->cm);
    hipFree(b->meds);
    hipFree(b->invalid);
    hipFree(b->fb_units);
    hipFree(b->state);
    if (b->host_state) hipHostFree(b->host_state);
    if (b->ev_start) hipEventDestroy(b->ev_start);
    if (b->ev_main) hipEventDestroy(b->ev_main);
    if (b->ev_cm) hipEventDestroy(b->ev_cm);
    if (b->ev_end) hipEventDestroy(b->ev_end);
    if (b->ev_state) hipEventDestroy(b->ev_state);
    if (b->ev_use) hipEventDestroy(b->ev_use);
    delete b;
}

}  // namespace

struct pdc_ctx {
    int device = -1;
    int n_cu = 0;
    int max_lds = 0;
    hipStream_t stream = nullptr;
    hipStream_t copy_stream = nullptr;  // result copies: they wait for their batch only
    std::vector<hipStream_t> mix_streams;  // concurrent batches of pdc_process_mixed
    bool mix_share = false;                // PDC_MIX_SHARE=1: size each mixed launch to its share of the chip
    bool mix_one = true;                   // mixed batches in one launch (PDC_MIX_FORKED=1: a launch each)
    std::vector<hipEvent_t> mix_events;
    std::vector<Detector> dets;
    std::map<uint64_t, Batch> batches;
    std::vector<Buffers *> spare;
    uint64_t next_batch = 1;
    std::string err;
    HitRecord *fmt_buf = nullptr;  // staging for host-destination get_hits
    uint64_t fmt_cap = 0;
    bool force_v1 = false;         // PDC_FORCE_GENERAL=1 in the environment
    int strip_rows = 0;            // PDC_STRIP_ROWS=n: own rows per strip at most n for new detectors
    bool tight_pool = false;       // PDC_DEBUG_TIGHT_POOL=1: first staging holds hit_capacity only
    hipStream_t capture_stream = nullptr;  // private stream for graph capture
    std::set<pdc_graph *> graphs;
};

// Captured batches: the kernels of one or more batches (items) of fixed size
// over fixed frame buffers, replayed by pdc_graph_launch into buffers the
// graph owns.
struct pdc_graph {
    pdc_ctx *ctx = nullptr;
    std::vector<Batch> proto;      // shape of each captured batch (path, groups, capacity, ...)
    std::vector<Buffers *> buf;    // the buffers each item's kernels read and write
    std::vector<uint64_t> batch;   // outstanding batch of each item, 0 if none
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool busy() const
    {
        for (uint64_t b : batch)
            if (b) return true;
        return false;
    }
};

namespace {

pdc_status fail(pdc_ctx *ctx, pdc_status st, const char *fmt, ...)
{
    char msg[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(msg, sizeof msg, fmt, ap);
    va_end(ap);
    if (ctx) ctx->err = msg;
    snprintf(g_thread_error, sizeof g_thread_error, "%s", msg);
    return st;
}

#define HIP_TRY(ctx, expr)                                                                   \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail((ctx), e_ == hipErrorOutOfMemory ? PDC_ENOMEM : PDC_EDEVICE,         \
                        "%s: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, __LINE__); \
    } while (0)

bool finite_in(float x, float lo, float hi) { return std::isfinite(x) && x >= lo && x <= hi; }

pdc_status check_geometry(const pdc_geometry *g)
{
    if (!g) return fail(nullptr, PDC_EINVAL, "geometry is NULL");
    if (g->n_tiles < 1 || g->rows < 1 || g->cols < 1 || g->bank_cols < 1)
        return fail(nullptr, PDC_EINVAL, "geometry sizes must be >= 1");
    if (g->cols > 2048 || g->bank_cols > 1024 || g->bank_cols > g->cols)
        return fail(nullptr, PDC_EINVAL, "cols <= 2048 and bank_cols <= min(cols, 1024) required");
    if (g->cols % g->bank_cols != 0)
        return fail(nullptr, PDC_EINVAL, "cols (%d) must be a multiple of bank_cols (%d)", g->cols,
                    g->bank_cols);
    if ((int64_t)g->n_tiles * g->rows * g->cols >= (int64_t)1 << 31)
        return fail(nullptr, PDC_EINVAL, "n_tiles*rows*cols must be < 2^31");
    if (g->gain_mode < 0 || g->gain_mode > 2) return fail(nullptr, PDC_EINVAL, "gain_mode must be 0, 1 or 2");
    return PDC_OK;
}

pdc_status check_params(const pdc_params *p, float *t_seed, float *t_nb)
{
    if (!p) return fail(nullptr, PDC_EINVAL, "params is NULL");
    if (!(std::isfinite(p->sigma) && p->sigma > 0.0f)) return fail(nullptr, PDC_EINVAL, "sigma must be finite and > 0");
    if (!(std::isfinite(p->n_seed) && p->n_seed >= 0.0f && std::isfinite(p->n_nb) && p->n_nb >= 0.0f))
        return fail(nullptr, PDC_EINVAL, "n_seed and n_nb must be finite and >= 0");
    volatile float ts = p->n_seed * p->sigma;  // binary32 products
    volatile float tn = p->n_nb * p->sigma;
    if (!std::isfinite(ts) || !std::isfinite(tn)) return fail(nullptr, PDC_EINVAL, "thresholds overflow");
    if (!(tn <= ts)) return fail(nullptr, PDC_EINVAL, "n_nb*sigma must be <= n_seed*sigma");
    if (!finite_in(p->photon_adu, 0x1p-24f, 0x1p24f))
        return fail(nullptr, PDC_EINVAL, "photon_adu must be in [2^-24, 2^24]");
    if (p->flags & ~(PDC_KEEP_CORRECTED | PDC_KEEP_MEDIANS))
        return fail(nullptr, PDC_EINVAL, "unknown flag bits 0x%x", p->flags);
    if (p->cm_mode != PDC_CM_MEDIAN && p->cm_mode != PDC_CM_BANK_MEAN && p->cm_mode != PDC_CM_TILE_MEAN)
        return fail(nullptr, PDC_EINVAL, "unknown cm_mode %d", p->cm_mode);
    if (p->cm_mode != PDC_CM_MEDIAN) {
        if (p->cm_stages < 1 || p->cm_stages > 3) return fail(nullptr, PDC_EINVAL, "cm_stages must be 1, 2 or 3");
        volatile float tc = p->n_cm * p->sigma;
        if (!(std::isfinite(p->n_cm) && p->n_cm >= 0.0f && std::isfinite(tc)))
            return fail(nullptr, PDC_EINVAL, "n_cm must be finite and >= 0 with n_cm*sigma finite");
    }
    if (t_seed) *t_seed = ts;
    if (t_nb) *t_nb = tn;
    return PDC_OK;
}

int n_ranges(const pdc_geometry &g) { return g.gain_mode ? 3 : 1; }

// Lowest set bit of a nonzero finite binary32 (c is an odd multiple of 2^lsb)
// and the smallest h with |c| < 2^h (zero: -149).
int f32_lsb_host(float c)
{
    uint32_t b;
    std::memcpy(&b, &c, 4);
    const int E = (int)((b >> 23) & 0xFFu);
    const uint32_t M = E ? ((b & 0x7FFFFFu) | 0x800000u) : (b & 0x7FFFFFu);
    return (E ? E : 1) - 150 + __builtin_ctz(M);
}
int f32_hi_host(float c)
{
    uint32_t b;
    std::memcpy(&b, &c, 4);
    b &= 0x7FFFFFFFu;
    if (!b) return -149;
    const int E = (int)(b >> 23);
    return E ? E - 126 : -149 + (32 - __builtin_clz(b));
}

// Window of every Frames1 value fl(fl(adc - dark) * k), adc in [0, 16383]: a
// multiple of 2^(min(0, lsb(dark)) + lsb(k)) (adc is an integer; a rounding to
// binary32 keeps such a multiple), at most the larger of |x(0)| and |x(16383)|
// in magnitude (x is monotone in adc).  The exact thresholded sums size their
// accumulators from it.
void frames1_window(const float *ped, const float *k, size_t n, int32_t *lo, int32_t *hi)
{
    int l = 0, h = -149;
    for (size_t i = 0; i < n; ++i) {
        const int lp = ped[i] == 0.0f ? 0 : std::min(0, f32_lsb_host(ped[i]));
        l = std::min(l, lp + f32_lsb_host(k[i]));
        volatile float a0 = 0.0f - ped[i], a1 = 16383.0f - ped[i];  // binary32
        volatile float x0 = a0 * k[i], x1 = a1 * k[i];
        h = std::max(h, std::max(f32_hi_host(x0), f32_hi_host(x1)));
    }
    *lo = l;
    *hi = h;
}

pdc_status check_planes(const pdc_geometry *g, const float *ped, const float *gain)
{
    if (!ped || !gain) return fail(nullptr, PDC_EINVAL, "pedestal and gain must be non-NULL");
    const int64_t n = (int64_t)n_ranges(*g) * g->n_tiles * g->rows * g->cols;
    for (int64_t i = 0; i < n; ++i) {
        float d = ped[i];
        if (!(std::isfinite(d) && std::fabs(d) <= 0x1p24f && (d == 0.0f || std::fabs(d) >= 0x1p-64f)))
            return fail(nullptr, PDC_EINVAL, "pedestal[%lld] = %g outside the valid range", (long long)i, (double)d);
        float k = gain[i];
        if (!finite_in(k, 0x1p-24f, 0x1p24f))
            return fail(nullptr, PDC_EINVAL, "gain[%lld] = %g outside [2^-24, 2^24]", (long long)i, (double)k);
    }
    return PDC_OK;
}

int next_pow2(int x)
{
    int p = 1;
    while (p < x) p <<= 1;
    return p;
}

// Launch shape of the v1 kernel for a geometry; false if it does not fit.
bool plan_v1(Detector &d)
{
    const pdc_geometry &g = d.g;
    int nb = g.cols / g.bank_cols;
    d.sort_width = next_pow2(g.bank_cols);
    for (int s = 16; s >= 1; --s) {
        int sr = std::min(s, g.rows);
        uint32_t mh = (uint32_t)((sr + 1) / 2) * (uint32_t)((g.cols + 1) / 2);
        for (int srt = sr + 2; srt >= 1; --srt) {
            size_t lds = frame_kernel_v1_lds_bytes(sr, g.cols, nb, d.sort_width, srt, mh);
            if (lds <= kV1LdsBudget) {
                d.strip_rows = sr;
                d.sort_rows = srt;
                d.max_unit_hits = mh;
                d.lds_bytes = lds;
                d.strips_per_tile = (g.rows + sr - 1) / sr;
                d.units_per_frame = g.n_tiles * d.strips_per_tile;
                // prefer more rows per strip only while the sort still holds a few rows
                if (srt >= std::min(sr + 2, 4)) return true;
                break;
            }
        }
    }
    return d.strip_rows > 0;
}

// Plan of the persistent kernel: strips of at most rmax loaded rows, as many
// strips x frame groups as there are compute units; false if the geometry is
// outside its fast path (odd widths, banks wider than 256, or too little LDS).
bool plan_v2(pdc_ctx *ctx, Detector &d)
{
    const pdc_geometry &g = d.g;
    d.v2_ok = false;
    if ((g.cols & 1) || (g.bank_cols & 1) || g.bank_cols > 256 || g.bank_cols < 2)
        return false;
    // single-gain kernels read each strip as a block of 4-pixel chunks
    if (!g.gain_mode && (g.cols % 4))
        return false;
    const int nb = g.cols / g.bank_cols;
    d.nq = g.bank_cols > 128 ? 2 : 1;
    d.gmax = d.nq == 2 ? 4 : 8;
    const int max_bank_rows = kV2Waves * d.gmax;  // a bank-row group per wave and slot
    const int rmax_lim = max_bank_rows / nb;
    if (rmax_lim < 3) return false;
    const int own_max = d.strip_cap > 0 ? std::min(rmax_lim - 2, d.strip_cap) : rmax_lim - 2;
    // Strips of at most own_max own rows over the frame's rows counted across
    // tiles (global row t * H + r): a strip may cross a tile edge, which
    // evens out strips when H is not a multiple of own_max (CSPAD: 198 strips
    // of 29-30 rows rather than 224 of 26-27); the halo row on each side is
    // loaded only when it lies in the same tile.  With tiles shorter than a
    // strip each tile is cut on its own, so a strip holds at most one edge.
    const int64_t TH = (int64_t)g.n_tiles * g.rows;
    std::vector<std::pair<int, int>> own;  // [g0, g1)
    if (g.rows >= own_max) {
        const int64_t n_st = (TH + own_max - 1) / own_max;
        for (int64_t j = 0; j < n_st; ++j) own.emplace_back((int)(TH * j / n_st), (int)(TH * (j + 1) / n_st));
    } else {
        for (int t = 0; t < g.n_tiles; ++t) own.emplace_back(t * g.rows, (t + 1) * g.rows);
    }
    std::vector<V2Strip> strips;
    int rmax = 0, own_rows_max = 0;
    for (const auto &o : own) {
        const int g0 = o.first, g1 = o.second;
        if (g1 <= g0) continue;
        const int t0 = g0 / g.rows, t1 = (g1 - 1) / g.rows;
        if (t1 > t0 + 1) return false;
        V2Strip S{};
        S.g0 = g0;
        S.g1 = g1;
        S.lg0 = g0 % g.rows ? g0 - 1 : g0;
        S.lg1 = g1 % g.rows ? g1 + 1 : g1;
        S.gb = t1 > t0 ? t1 * g.rows : INT32_MAX;
        strips.push_back(S);
        rmax = std::max(rmax, S.lg1 - S.lg0);
        own_rows_max = std::max(own_rows_max, g1 - g0);
    }
    if (rmax * nb > max_bank_rows) return false;
    d.n_strips = (int)strips.size();
    d.rmax = rmax;
    // local maxima of a strip's own rows: at most every other row and column
    // of each tile part (two parts when the strip crosses a tile edge)
    d.v2_max_unit_hits = (uint32_t)((own_rows_max + 3) / 2) * (uint32_t)((g.cols + 1) / 2);
    // seed lists: as large as the workgroup's LDS allows (the kernel's
    // registers admit one workgroup per compute unit anyway), at least 1024
    // entries; 512 bytes stay free for the kernel's static LDS (the one-launch
    // mixed kernel holds every body's own variables)
    const size_t lds_wg = (size_t)ctx->max_lds / kV2GroupsPerCu;
#ifdef PDC_PHASE_TIMERS
    const size_t static_lds = 2048;  // the tracing build's per-wave counters
#else
    const size_t static_lds = 512;
#endif
    const size_t lds_cap = lds_wg > static_lds ? lds_wg - static_lds : 0;
    size_t base = frame_kernel_v2_lds_bytes(rmax, g.cols, nb, 0);
    if (base + 4 * 4 * 1024 > lds_cap) return false;
    d.seed_cap = (int)std::min<size_t>((lds_cap - base) / 16, 16384);
    d.v2_lds = frame_kernel_v2_lds_bytes(rmax, g.cols, nb, d.seed_cap);
    // the general kernel sized for one of these strips (own rows + halo), to
    // redo the units whose seed lists overflow
    d.fb_ok = false;
    {
        const int sw = (int)next_pow2(g.bank_cols);
        for (int srt = own_rows_max + 2; srt >= 1 && !d.fb_ok; --srt) {
            const size_t lds = frame_kernel_v1_lds_bytes(own_rows_max, g.cols, nb, sw, srt, d.v2_max_unit_hits);
            if (lds <= lds_cap) {
                d.fb_ok = true;
                d.fb_strip_rows = own_rows_max;
                d.fb_sort_rows = srt;
                d.fb_lds = lds;
            }
        }
    }
    d.rank_width = d.p.sigma / (0.4f * (float)g.bank_cols);
    d.n_cu = ctx->n_cu;
    if (d.d_strips) {  // a new plan of the same detector (no batch holds the old one)
        hipFree(d.d_strips);
        d.d_strips = nullptr;
    }
    if (hipMalloc((void **)&d.d_strips, strips.size() * sizeof(V2Strip)) != hipSuccess) return false;
    if (hipMemcpy(d.d_strips, strips.data(), strips.size() * sizeof(V2Strip), hipMemcpyHostToDevice) != hipSuccess)
        return false;
    d.v2_ok = true;
    return true;
}

template <typename T>
hipError_t grow(T **ptr, uint64_t &cap, uint64_t need)
{
    if (need <= cap && *ptr) return hipSuccess;
    hipFree(*ptr);
    *ptr = nullptr;
    cap = 0;
    uint64_t n = std::max<uint64_t>(need, 1);
    hipError_t e = hipMalloc((void **)ptr, n * sizeof(T));
    if (e == hipSuccess) cap = n;
    return e;
}

pdc_status ensure_buffers(pdc_ctx *ctx, Buffers *b, uint64_t n_units, uint64_t n_frames,
                          uint64_t pool_cap, uint64_t corr_floats, uint64_t cm_floats = 0, uint64_t meds_floats = 0)
{
    if (!b->state) {
        HIP_TRY(ctx, hipMalloc((void **)&b->state, sizeof(BatchState)));
        HIP_TRY(ctx, hipHostMalloc((void **)&b->host_state, sizeof(BatchState), hipHostMallocDefault));
        HIP_TRY(ctx, hipEventCreate(&b->ev_start));
        HIP_TRY(ctx, hipEventCreate(&b->ev_main));
        HIP_TRY(ctx, hipEventCreate(&b->ev_cm));
        HIP_TRY(ctx, hipEventCreate(&b->ev_end));
        HIP_TRY(ctx, hipEventCreateWithFlags(&b->ev_state, hipEventDisableTiming));
        HIP_TRY(ctx, hipEventCreateWithFlags(&b->ev_use, hipEventDisableTiming));
    }
    if (n_units > b->cap_units || !b->unit_count) {
        uint64_t c0 = 0, c1 = 0, c2 = 0, c3 = 0;
        HIP_TRY(ctx, grow(&b->unit_count, c0, n_units));
        HIP_TRY(ctx, grow(&b->unit_photons, c1, n_units));
        HIP_TRY(ctx, grow(&b->unit_base, c2, n_units));
        HIP_TRY(ctx, grow(&b->unit_local, c3, n_units));
        b->cap_units = std::max<uint64_t>(n_units, 1);
    }
    if (n_frames > b->cap_frames || !b->frame_hits) {
        uint64_t c0 = 0, c1 = 0, c2 = 0;
        HIP_TRY(ctx, grow(&b->frame_hits, c0, n_frames));
        HIP_TRY(ctx, grow(&b->frame_photons, c1, n_frames));
        HIP_TRY(ctx, grow(&b->frame_offset, c2, n_frames + 1));
        b->cap_frames = std::max<uint64_t>(n_frames, 1);
    }
    if (pool_cap > b->cap_pool || !b->pool) {
        uint64_t c0 = 0, c1 = 0;
        HIP_TRY(ctx, grow(&b->pool, c0, pool_cap));
        HIP_TRY(ctx, grow(&b->hits, c1, pool_cap));
        b->cap_pool = std::max<uint64_t>(pool_cap, 1);
    }
    if (corr_floats > b->cap_corr) {
        HIP_TRY(ctx, grow(&b->corrected, b->cap_corr, corr_floats));
    }
    if (cm_floats > b->cap_cm) {
        HIP_TRY(ctx, grow(&b->cm, b->cap_cm, cm_floats));
    }
    if (meds_floats > b->cap_meds) {
        HIP_TRY(ctx, grow(&b->meds, b->cap_meds, meds_floats));
    }
    if (n_frames > b->cap_inv || !b->invalid) {
        HIP_TRY(ctx, grow(&b->invalid, b->cap_inv, n_frames));
    }
    if (n_units > b->cap_fb || !b->fb_units) {
        HIP_TRY(ctx, grow(&b->fb_units, b->cap_fb, n_units));
    }
    return PDC_OK;
}

uint32_t v1_grid(uint64_t n_units)
{
    return (uint32_t)std::min<uint64_t>(n_units, 256 * 8);
}

uint64_t pool_capacity(const Detector &d, int path, uint64_t hit_capacity, uint32_t grid)
{
    // Each workgroup may hold a partly used chunk, and each chunk may leave a
    // tail smaller than one unit's hits.
    uint64_t per_chunk_waste = path == 2 ? d.v2_max_unit_hits : d.max_unit_hits;
    uint64_t slack = (uint64_t)grid * (kChunkHits + per_chunk_waste) +
                     (hit_capacity / kChunkHits + 1) * per_chunk_waste;
    return hit_capacity + slack;
}

uint32_t batch_grid(const Detector &d, const Batch &bt)
{
    return bt.path == 2 ? (uint32_t)(bt.n_fg * d.n_strips) : v1_grid(bt.n_units);
}

// Thresholded-mean stage values of every frame of the batch into b->cm.
hipError_t launch_cm_pass(pdc_ctx *ctx, const Detector &d, const Batch &bt)
{
    if (bt.n_frames == 0) return hipSuccess;
    CmArgs c{};
    c.frames = bt.frames;
    c.ped = d.d_ped;
    c.k = d.d_k;
    c.n_frames = bt.n_frames;
    c.T = d.g.n_tiles;
    c.H = d.g.rows;
    c.W = d.g.cols;
    c.B = d.g.bank_cols;
    c.nb = d.g.cols / d.g.bank_cols;
    c.stages = d.p.cm_stages;
    c.t_cm = d.t_cm;
    c.guard = d.cm_guard;
    c.sum_lo = d.sum_lo;
    c.sum_hi = d.sum_hi;
    c.gain_mode = d.g.gain_mode;
    c.cm = bt.buf->cm;
    if (d.p.cm_mode == PDC_CM_BANK_MEAN) return launch_cm_bank(c, (uint32_t)ctx->n_cu, bt.stream);
    return launch_cm_tile(c, (uint32_t)ctx->n_cu, bt.stream);
}

// Arguments of the general kernel common to whole-batch and unit-list runs.
void fill_v1_args(const Detector &d, const Batch &bt, FrameKernelArgs &a)
{
    Buffers *b = bt.buf;
    a.frames = bt.frames;
    a.ped = d.d_ped;
    a.k = d.d_k;
    a.n_frames = bt.n_frames;
    a.n_units = bt.n_units;
    a.T = d.g.n_tiles;
    a.H = d.g.rows;
    a.W = d.g.cols;
    a.B = d.g.bank_cols;
    a.nb = d.g.cols / d.g.bank_cols;
    a.strip_rows = d.strip_rows;
    a.strips_per_tile = d.strips_per_tile;
    a.units_per_frame = d.units_per_frame;
    a.sort_width = d.sort_width;
    a.sort_rows = d.sort_rows;
    a.max_unit_hits = d.max_unit_hits;
    a.t_seed = d.t_seed;
    a.t_nb = d.t_nb;
    a.photon_adu = d.p.photon_adu;
    a.pool = b->pool;
    a.pool_cap = bt.pool_cap;
    a.unit_count = b->unit_count;
    a.unit_photons = b->unit_photons;
    a.unit_base = b->unit_base;
    a.state = b->state;
    a.corrected = bt.keep ? b->corrected : nullptr;
    a.cm = d.p.cm_mode ? b->cm : nullptr;
    a.cm_regions = d.cm_regions;
    a.cm_tile = d.p.cm_mode == PDC_CM_TILE_MEAN;
    a.gain_mode = d.g.gain_mode;
    a.invalid = b->invalid;
    a.meds = bt.meds && !d.p.cm_mode ? b->meds : nullptr;
}

// End of a batch's work on its stream: the timing event, then the state copy
// that finish_batch reads.
pdc_status record_end(pdc_ctx *ctx, Buffers *b, hipStream_t s)
{
    HIP_TRY(ctx, hipEventRecord(b->ev_end, s));
    HIP_TRY(ctx, hipMemcpyAsync(b->host_state, b->state, sizeof(BatchState), hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipEventRecord(b->ev_state, s));
    return PDC_OK;
}

// Per-frame sums, offsets and the raster-ordered list, then the state copy.
pdc_status enqueue_tail(pdc_ctx *ctx, Batch &bt)
{
    Buffers *b = bt.buf;
    hipStream_t s = bt.stream;
    HIP_TRY(ctx, launch_frame_sums(b->unit_count, b->unit_photons, bt.n_frames, bt.upf,
                                   b->unit_local, b->frame_hits, b->frame_photons, s));
    HIP_TRY(ctx, launch_frame_scan(b->frame_hits, bt.n_frames, b->frame_offset, b->state, s));
    if (bt.records)
        HIP_TRY(ctx, launch_scatter_records(b->unit_count, b->unit_base, b->unit_local, b->frame_offset, b->pool,
                                            bt.n_units, bt.upf, ctx->dets[bt.det].p.photon_adu, bt.records,
                                            bt.records_cap, s));
    else
        HIP_TRY(ctx, launch_scatter(b->unit_count, b->unit_base, b->unit_local, b->frame_offset, b->pool,
                                    bt.n_units, bt.upf, b->hits, b->cap_pool, s));
    if (bt.capture) return PDC_OK;
    return record_end(ctx, b, s);
}

// The persistent kernel computes a bank's thresholded mean itself unless the
// stage values are kept for patches.
bool cm_inline_of(const Detector &d, const Batch &bt)
{
    return d.p.cm_mode == PDC_CM_BANK_MEAN && bt.path == 2 && !bt.meds;
}

// A batch's work before its frame kernel: state, timing events, invalid
// counts and the common-mode pass.
pdc_status enqueue_pre(pdc_ctx *ctx, Batch &bt)
{
    Detector &d = ctx->dets[bt.det];
    Buffers *b = bt.buf;
    hipStream_t s = bt.stream;
    HIP_TRY(ctx, launch_init_state(b->state, s));
    if (!bt.capture) HIP_TRY(ctx, hipEventRecord(b->ev_start, s));
    if (d.g.gain_mode) HIP_TRY(ctx, launch_fill_u32(b->invalid, bt.n_frames, s));
    if (d.p.cm_mode && !cm_inline_of(d, bt)) HIP_TRY(ctx, launch_cm_pass(ctx, d, bt));
    if (!bt.capture) HIP_TRY(ctx, hipEventRecord(b->ev_cm, s));
    return PDC_OK;
}

// Rows between the bank-rows that one wave's four 16-lane median groups read:
// 4 or 0 (consecutive bank-rows).  Each group reads 16 consecutive LDS words
// per value slot from its bank-row's start; every fourth row is taken when it
// spreads the four windows more evenly over the 64 LDS banks (W = 388: starts
// 16 banks apart, no conflict, against four-way conflicts for consecutive
// bank-rows).
static int median_row_step(int W, int B, int nb)
{
    auto worst = [](const int(&off)[4]) {
        int cnt[64] = {}, mx = 0;
        for (int g = 0; g < 4; ++g)
            for (int k = 0; k < 16; ++k) mx = std::max(mx, ++cnt[(off[g] + k) & 63]);
        return mx;
    };
    int off[4];
    for (int g = 0; g < 4; ++g) off[g] = (g / nb) * W + (g % nb) * B;
    int best = 0, best_w = worst(off);
    for (int step : {4}) {
        for (int g = 0; g < 4; ++g) off[g] = g * step * W;
        const int w = worst(off);
        if (w < best_w) {
            best = step;
            best_w = w;
        }
    }
    return best;
}

// Arguments of the persistent kernel for a batch.
void fill_v2_args(const Detector &d, const Batch &bt, V2Args &a)
{
    const Buffers *b = bt.buf;
    const bool cm_inline = cm_inline_of(d, bt);
    a = V2Args{};
    a.frames = bt.frames;
    a.ped = d.d_ped;
    a.k = d.d_k;
    a.n_frames = bt.n_frames;
    a.T = d.g.n_tiles;
    a.H = d.g.rows;
    a.W = d.g.cols;
    a.B = d.g.bank_cols;
    a.nb = d.g.cols / d.g.bank_cols;
    a.n_strips = d.n_strips;
    a.n_fgroups = bt.n_fg;
    a.rmax = d.rmax;
    a.seed_cap = d.seed_cap;
    a.strips = d.d_strips;
    a.t_seed = d.t_seed;
    a.t_nb = d.t_nb;
    a.photon_adu = d.p.photon_adu;
    a.rank_width = d.rank_width;
    a.pool = b->pool;
    a.pool_cap = bt.pool_cap;
    a.unit_count = b->unit_count;
    a.unit_photons = b->unit_photons;
    a.unit_base = b->unit_base;
    a.state = b->state;
    a.corrected = bt.keep ? b->corrected : nullptr;
    a.fb_units = d.fb_ok ? b->fb_units : nullptr;
    a.cm = cm_inline ? nullptr : b->cm;
    a.cm_regions = d.cm_regions;
    a.cm_tile = d.p.cm_mode == PDC_CM_TILE_MEAN;
    a.cm_mode = d.p.cm_mode == PDC_CM_MEDIAN ? 0 : (cm_inline ? 1 : 2);
    a.cm_stages = d.p.cm_stages;
    a.t_cm = d.t_cm;
    a.cm_guard = d.cm_guard;
    a.sum_lo = d.sum_lo;
    a.sum_hi = d.sum_hi;
    a.med_row_step = d.nq == 2 ? median_row_step(a.W, a.B, a.nb) : 0;
    a.gain_mode = d.g.gain_mode;
    a.invalid = b->invalid;
    a.meds = bt.meds && !d.p.cm_mode ? b->meds : nullptr;
}

// After the frame kernel: its timing event, then the scans and scatter.
pdc_status enqueue_post(pdc_ctx *ctx, Batch &bt)
{
    if (!bt.capture) HIP_TRY(ctx, hipEventRecord(bt.buf->ev_main, bt.stream));
    return enqueue_tail(ctx, bt);
}

pdc_status enqueue(pdc_ctx *ctx, Batch &bt)
{
    pdc_status rc = enqueue_pre(ctx, bt);
    if (rc != PDC_OK) return rc;
    Detector &d = ctx->dets[bt.det];
    hipStream_t s = bt.stream;
    if (bt.n_units > 0 && bt.path == 2) {
        V2Args a;
        fill_v2_args(d, bt, a);
        HIP_TRY(ctx, launch_frame_kernel_v2(a, d.nq, d.gmax, batch_grid(d, bt), d.v2_lds, bt.keep, s));
    } else if (bt.n_units > 0) {
        FrameKernelArgs a{};
        fill_v1_args(d, bt, a);
        HIP_TRY(ctx, launch_frame_kernel_v1(a, batch_grid(d, bt), d.lds_bytes, bt.keep, s));
    }
    return enqueue_post(ctx, bt);
}

// The one-launch form of a mixed call: 2 to kMixMax batches whose detectors
// all take the persistent kernel through a compiled body of the mixed kernel
// (v2_mix_variant: median common mode, nothing kept), with the largest LDS
// beside the kernel's own static variables.  Otherwise the batches launch on
// their own.
bool mix_one_launch(pdc_ctx *ctx, const std::vector<int32_t> &dets)
{
    if (!ctx->mix_one || dets.size() < 2 || dets.size() > (size_t)kMixMax) return false;
    static const size_t static_lds = frame_kernel_v2_mix_static_lds();
    size_t lds = 0;
    for (int32_t det : dets) {
        const Detector &d = ctx->dets[det];
        if (!d.v2_ok) return false;
        V2Args a{};
        a.B = d.g.bank_cols;
        a.nb = d.g.cols / d.g.bank_cols;
        a.rmax = d.rmax;
        a.gain_mode = d.g.gain_mode;
        a.cm_mode = d.p.cm_mode == PDC_CM_MEDIAN ? 0 : 1;
        if ((d.p.flags & PDC_KEEP_MEDIANS) || v2_mix_variant(a, d.nq, d.gmax, (d.p.flags & PDC_KEEP_CORRECTED) != 0) < 0)
            return false;
        lds = std::max(lds, d.v2_lds);
    }
    return static_lds != SIZE_MAX && lds + static_lds <= (size_t)ctx->max_lds / kV2GroupsPerCu;
}

// Frame groups of a batch in the one launch, beyond its detector's choice:
// finer work items, so that workgroups of detectors of unequal cost per pixel
// even out across the chip as they are handed out.
constexpr int kMixFgMore = 2;

// Enqueue the batches of a mixed call, each on its own stream (streams[i]),
// forked from and joined back into the stream s (events: at least
// streams.size() + 1).  With one launch, the batches' work before and after
// the frame kernel stays on their streams and the kernel runs on s.
pdc_status enqueue_mixed(pdc_ctx *ctx, std::vector<Batch *> &bts, hipStream_t s, const std::vector<hipStream_t> &streams,
                         const std::vector<hipEvent_t> &events)
{
    const int n_str = (int)streams.size();
    // the streams forked so far are joined back also after a failure, so that
    // none is left waiting on (or, under capture, capturing from) s
    int forked = 0;
    auto fork = [&]() -> pdc_status {
        HIP_TRY(ctx, hipEventRecord(events[0], s));
        for (; forked < n_str; ++forked) HIP_TRY(ctx, hipStreamWaitEvent(streams[forked], events[0], 0));
        return PDC_OK;
    };
    auto join = [&]() -> pdc_status {
        pdc_status r = PDC_OK;
        for (int j = 0; j < forked; ++j) {
            hipError_t e = hipEventRecord(events[1 + j], streams[j]);
            if (e == hipSuccess) e = hipStreamWaitEvent(s, events[1 + j], 0);
            if (e != hipSuccess && r == PDC_OK) r = fail(ctx, PDC_EDEVICE, "join: %s", hipGetErrorString(e));
        }
        forked = 0;
        return r;
    };
    pdc_status rc = fork();
    if (rc != PDC_OK) {
        join();
        return rc;
    }
    std::vector<int32_t> dets;
    for (const Batch *bt : bts) dets.push_back(bt->det);
    bool one = mix_one_launch(ctx, dets);
    for (const Batch *bt : bts) one = one && bt->path == 2 && bt->n_units > 0;
    if (!one) {
        for (Batch *bt : bts)
            if ((rc = enqueue(ctx, *bt)) != PDC_OK) break;
        pdc_status rj = join();
        return rc != PDC_OK ? rc : rj;
    }
    for (Batch *bt : bts)
        if ((rc = enqueue_pre(ctx, *bt)) != PDC_OK) break;
    pdc_status rj = join();
    if (rc != PDC_OK || rj != PDC_OK) return rc != PDC_OK ? rc : rj;
    V2Mix m{};
    size_t lds = 0;
    int first = 0;
    for (size_t i = 0; i < bts.size(); ++i) {
        bts[i]->mix_one = true;
        const Batch &bt = *bts[i];
        const Detector &d = ctx->dets[bt.det];
        fill_v2_args(d, bt, m.a[i]);
        m.variant[i] = v2_mix_variant(m.a[i], d.nq, d.gmax, bt.keep);
        m.first[i] = first;
        first += (int)batch_grid(d, bt);
        lds = std::max(lds, d.v2_lds);
    }
    m.first[bts.size()] = first;
    m.n = (int32_t)bts.size();
    HIP_TRY(ctx, launch_frame_kernel_v2_mix(m, lds, s));
    rc = fork();
    for (Batch *bt : bts)
        if (rc == PDC_OK) rc = enqueue_post(ctx, *bt);
    rj = join();
    return rc != PDC_OK ? rc : rj;
}

// Redo the units the persistent kernel listed as overflowing with the general
// kernel over the same strips, then the scans and scatter again.
pdc_status enqueue_partial(pdc_ctx *ctx, Batch &bt, uint64_t n_list)
{
    Detector &d = ctx->dets[bt.det];
    Buffers *b = bt.buf;
    hipStream_t s = bt.stream;
    if (d.p.cm_mode == PDC_CM_BANK_MEAN && !bt.meds)
        HIP_TRY(ctx, launch_cm_pass(ctx, d, bt));  // the kernel computed it inline
    FrameKernelArgs a{};
    fill_v1_args(d, bt, a);
    a.n_units = bt.n_units;
    a.units_per_frame = d.n_strips;
    a.strip_rows = d.fb_strip_rows;
    a.sort_rows = d.fb_sort_rows;
    a.max_unit_hits = d.v2_max_unit_hits;
    a.unit_list = b->fb_units;
    a.n_list = n_list;
    a.strips = d.d_strips;
    HIP_TRY(ctx, launch_frame_kernel_v1(a, v1_grid(n_list), d.fb_lds, bt.keep, s));
    return enqueue_tail(ctx, bt);
}

// Frame groups of a persistent launch: each workgroup takes one strip for a
// contiguous range of frames, one workgroup per compute unit at a time, and
// spends two extra pipeline iterations draining.  The count minimises
// rounds x (frames per group + 2), the iterations a compute unit runs: large
// batches get enough groups to fill whole rounds of the chip (CSPAD's 198
// strips alone would leave 58 of 256 units idle), small ones stay in one round.
int frame_groups(int n_cu, int n_strips, uint64_t n_frames, int mult)
{
    const int max_fg = (int)std::max<uint64_t>(1, std::min<uint64_t>(64, n_frames));
    int best = 1;
    uint64_t best_cost = ~0ull;
    for (int g = 1; g <= max_fg; ++g) {
        const uint64_t wgs = (uint64_t)g * n_strips;
        const uint64_t rounds = (wgs + n_cu - 1) / n_cu;
        const uint64_t cost = rounds * ((n_frames + g - 1) / g + 2);
        if (cost < best_cost) {
            best_cost = cost;
            best = g;
        }
    }
    // more rounds of the same fill, if tuned so (finer dynamic balancing)
    return (int)std::max<uint64_t>(1, std::min<uint64_t>((uint64_t)best * (uint64_t)std::max(1, mult), n_frames));
}

// Choose the kernel for a batch and size its unit arrays.
void set_path(const Detector &d, Batch &bt, int path)
{
    bt.path = path;
    if (path == 2) {
        const int fgb = frame_groups(d.n_cu * kV2GroupsPerCu, d.n_strips, bt.n_frames, d.fg_mult * bt.fg_more);
        const uint64_t fg = (uint64_t)std::max(1.0, std::floor((double)fgb * bt.share));
        bt.n_fg = (int)std::max<uint64_t>(1, std::min<uint64_t>(fg, bt.n_frames));
        bt.upf = d.n_strips;
    } else {
        bt.n_fg = 1;
        bt.upf = d.units_per_frame;
    }
    bt.n_units = bt.n_frames * (uint64_t)bt.upf;
}

Batch *find_batch(pdc_ctx *ctx, uint64_t id)
{
    auto it = ctx->batches.find(id);
    return it == ctx->batches.end() ? nullptr : &it->second;
}

// Frames2 and common-mode floats a batch's buffers hold.
uint64_t corr_floats(const Detector &d, const Batch &bt)
{
    return bt.keep ? bt.n_frames * (uint64_t)d.g.n_tiles * d.g.rows * d.g.cols : 0;
}
uint64_t cm_floats(const Detector &d, const Batch &bt)
{
    return d.p.cm_mode ? bt.n_frames * (uint64_t)d.cm_regions * 3 : 0;
}

// Bank medians kept for patches (the thresholded mean keeps its stage values
// in cm anyway).
uint64_t meds_floats(const Detector &d, const Batch &bt)
{
    return bt.meds && !d.p.cm_mode ? bt.n_frames * (uint64_t)d.g.n_tiles * d.g.rows * (d.g.cols / d.g.bank_cols) : 0;
}

Buffers *take_buffers(pdc_ctx *ctx)
{
    if (ctx->spare.empty()) return new (std::nothrow) Buffers;
    Buffers *b = ctx->spare.back();
    ctx->spare.pop_back();
    return b;
}

// Move a batch launched from a graph onto buffers of its own before it is
// recomputed from the start, which may grow them: the graph's kernels keep
// the addresses they were captured with.  The graph is free again.
pdc_status detach_from_graph(pdc_ctx *ctx, Batch &bt)
{
    if (!bt.graph) return PDC_OK;
    Buffers *b = take_buffers(ctx);
    if (!b) return fail(ctx, PDC_ENOMEM, "host allocation failed");
    const Detector &d = ctx->dets[bt.det];
    pdc_status rc = ensure_buffers(ctx, b, bt.n_units, bt.n_frames, bt.pool_cap, corr_floats(d, bt), cm_floats(d, bt));
    if (rc != PDC_OK) {
        ctx->spare.push_back(b);
        return rc;
    }
    bt.graph->batch[bt.gitem] = 0;
    bt.graph = nullptr;
    bt.buf = b;
    return PDC_OK;
}

// Wait for a batch; if its staging pool overflowed, run it again with exact
// capacity so that its hit list is complete.
pdc_status finish_batch(pdc_ctx *ctx, Batch &bt)
{
    HIP_TRY(ctx, hipEventSynchronize(bt.buf->ev_state));
    if (bt.checked) return PDC_OK;
    Detector &d = ctx->dets[bt.det];
    BatchState st = *bt.buf->host_state;
    for (int attempt = 0; attempt < 3; ++attempt) {
        if (st.fallback && bt.path == 2 && d.fb_ok) {
            // some strip-frames had more seed pixels than the persistent kernel
            // holds on chip: the general kernel redoes just those units
            pdc_status rc = enqueue_partial(ctx, bt, st.n_fallback);
            if (rc != PDC_OK) return rc;
            bt.fb = 1;
            HIP_TRY(ctx, hipEventSynchronize(bt.buf->ev_state));
            st = *bt.buf->host_state;
        } else if (st.fallback) {
            // no general-kernel plan for these strips: redo the whole batch
            pdc_status rc = detach_from_graph(ctx, bt);
            if (rc != PDC_OK) return rc;
            set_path(d, bt, 1);
            bt.fb = 2;
            const uint64_t cap = pool_capacity(d, 1, st.total, batch_grid(d, bt));
            rc = ensure_buffers(ctx, bt.buf, bt.n_units, bt.n_frames, cap, 0);
            if (rc != PDC_OK) return rc;
            bt.pool_cap = cap;
            rc = enqueue(ctx, bt);
            if (rc != PDC_OK) return rc;
            HIP_TRY(ctx, hipEventSynchronize(bt.buf->ev_state));
            st = *bt.buf->host_state;
        }
        if (!st.overflow) {
            bt.checked = true;
            return PDC_OK;
        }
        // staging overflow: run again with room for the exact total (and for
        // the chunks of a unit-list recomputation)
        uint64_t cap = pool_capacity(d, bt.path, st.total, batch_grid(d, bt));
        if (bt.fb == 1) cap += (uint64_t)v1_grid(st.n_fallback) * (kChunkHits + d.v2_max_unit_hits);
        pdc_status rc = detach_from_graph(ctx, bt);
        if (rc != PDC_OK) return rc;
        rc = ensure_buffers(ctx, bt.buf, bt.n_units, bt.n_frames, cap, 0);
        if (rc != PDC_OK) return rc;
        bt.pool_cap = cap;
        rc = enqueue(ctx, bt);
        if (rc != PDC_OK) return rc;
        HIP_TRY(ctx, hipEventSynchronize(bt.buf->ev_state));
        st = *bt.buf->host_state;
    }
    return fail(ctx, PDC_EDEVICE, "staging overflow persisted after resizing");
}

void maybe_free_detector(pdc_ctx *ctx, int32_t det)
{
    Detector &d = ctx->dets[det];
    if (d.live && d.release_requested && d.pending == 0) {
        hipFree(d.d_ped);
        hipFree(d.d_k);
        hipFree(d.d_strips);
        d = Detector{};
    }
}

// A batch's plan and buffers, not yet enqueued (on failure nothing is held).
pdc_status setup_batch(pdc_ctx *ctx, int32_t det, const uint16_t *frames_dev, uint64_t n_frames,
                       uint64_t hit_capacity, hipStream_t stream, double share, Batch &bt, int fg_more = 1)
{
    if (det < 0 || det >= (int32_t)ctx->dets.size() || !ctx->dets[det].live || ctx->dets[det].release_requested)
        return fail(ctx, PDC_ESTATE, "unknown detector %d", det);
    if (n_frames > 0 && !frames_dev) return fail(ctx, PDC_EINVAL, "frames_dev is NULL");
    if (n_frames > ((uint64_t)1 << 31)) return fail(ctx, PDC_EINVAL, "n_frames must be <= 2^31");
    Detector &d = ctx->dets[det];
    bt = Batch{};
    bt.det = det;
    bt.frames = frames_dev;
    bt.n_frames = n_frames;
    bt.share = share;
    bt.fg_more = fg_more;
    set_path(d, bt, d.v2_ok ? 2 : 1);
    bt.stream = stream;
    bt.keep = (d.p.flags & PDC_KEEP_CORRECTED) != 0;
    bt.meds = (d.p.flags & PDC_KEEP_MEDIANS) != 0;
    bt.pool_cap = ctx->tight_pool ? hit_capacity : pool_capacity(d, bt.path, hit_capacity, batch_grid(d, bt));
    Buffers *b = take_buffers(ctx);
    if (!b) return fail(ctx, PDC_ENOMEM, "host allocation failed");
    pdc_status rc = ensure_buffers(ctx, b, bt.n_units, n_frames, bt.pool_cap, corr_floats(d, bt), cm_floats(d, bt),
                                   meds_floats(d, bt));
    if (rc != PDC_OK) {
        ctx->spare.push_back(b);
        return rc;
    }
    bt.buf = b;
    return PDC_OK;
}

// An enqueued batch becomes outstanding under the next id.
uint64_t register_batch(pdc_ctx *ctx, Batch &bt)
{
    bt.id = ctx->next_batch++;
    ctx->dets[bt.det].pending += 1;
    ctx->batches[bt.id] = bt;
    return bt.id;
}

}  // namespace

extern "C" {

const char *pdc_strerror(pdc_status s)
{
    switch (s) {
    case PDC_OK: return "ok";
    case PDC_WARN_TRUNCATED: return "hit list truncated to the destination capacity";
    case PDC_EINVAL: return "invalid argument";
    case PDC_ENOMEM: return "out of memory";
    case PDC_EDEVICE: return "device or HIP runtime error";
    case PDC_ESTATE: return "invalid state (unknown or released object)";
    default: return "unknown status";
    }
}

const char *pdc_last_error(const pdc_ctx *ctx)
{
    if (!ctx) return g_thread_error;
    return ctx->err.c_str();
}

pdc_status pdc_create(int32_t device, pdc_ctx **out)
{
    if (!out) return fail(nullptr, PDC_EINVAL, "out is NULL");
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) return fail(nullptr, PDC_EDEVICE, "no HIP device");
    if (device < 0 || device >= n) return fail(nullptr, PDC_EDEVICE, "device %d out of range (%d devices)", device, n);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess)
        return fail(nullptr, PDC_EDEVICE, "hipGetDeviceProperties failed");
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(nullptr, PDC_EDEVICE, "device %d is %s, this library is built for gfx950", device, prop.gcnArchName);
    pdc_ctx *ctx = new (std::nothrow) pdc_ctx;
    if (!ctx) return fail(nullptr, PDC_ENOMEM, "host allocation failed");
    ctx->device = device;
    ctx->n_cu = prop.multiProcessorCount;
    {
        const char *fv = std::getenv("PDC_FORCE_GENERAL");
        ctx->force_v1 = fv && fv[0] == '1';
        const char *sr = std::getenv("PDC_STRIP_ROWS");
        ctx->strip_rows = sr ? std::max(0, std::atoi(sr)) : 0;
        const char *ms = std::getenv("PDC_MIX_SHARE");
        ctx->mix_share = ms && ms[0] == '1';
        const char *mf = std::getenv("PDC_MIX_FORKED");
        ctx->mix_one = !(mf && mf[0] == '1');
        const char *tp = std::getenv("PDC_DEBUG_TIGHT_POOL");
        ctx->tight_pool = tp && tp[0] == '1';
    }
    {
        int lds = 0;
        if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device) != hipSuccess) lds = 65536;
        ctx->max_lds = lds;
    }
    if (hipSetDevice(device) != hipSuccess || hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&ctx->copy_stream, hipStreamNonBlocking) != hipSuccess) {
        if (ctx->stream) hipStreamDestroy(ctx->stream);
        delete ctx;
        return fail(nullptr, PDC_EDEVICE, "stream creation failed");
    }
    if (device < kMaxDevices) {
        // the static scratch's address on this device (device current)
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        if (!g_scratch_ptr[device]) {
            void *p = nullptr;
            if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) == hipSuccess && p)
                g_scratch_ptr[device] = static_cast<unsigned char *>(p);
        }
    }
    *out = ctx;
    return PDC_OK;
}

pdc_status pdc_destroy(pdc_ctx *ctx)
{
    if (!ctx) return PDC_OK;
    hipSetDevice(ctx->device);
    hipDeviceSynchronize();
    for (auto &kv : ctx->batches)
        if (!kv.second.graph) free_buffers(kv.second.buf);
    for (Buffers *b : ctx->spare) free_buffers(b);
    for (pdc_graph *g : ctx->graphs) {
        hipGraphExecDestroy(g->exec);
        hipGraphDestroy(g->graph);
        for (Buffers *b : g->buf) free_buffers(b);
        delete g;
    }
    if (ctx->capture_stream) hipStreamDestroy(ctx->capture_stream);
    for (Detector &d : ctx->dets)
        if (d.live) {
            hipFree(d.d_ped);
            hipFree(d.d_k);
            hipFree(d.d_strips);
        }
    hipFree(ctx->fmt_buf);
    hipStreamDestroy(ctx->stream);
    hipStreamDestroy(ctx->copy_stream);
    for (hipStream_t st : ctx->mix_streams) hipStreamDestroy(st);
    for (hipEvent_t ev : ctx->mix_events) hipEventDestroy(ev);
    delete ctx;
    return PDC_OK;
}

pdc_status pdc_check_calibration(const pdc_geometry *geom, const float *pedestal, const float *gain,
                                 const pdc_params *params)
{
    pdc_status rc = check_geometry(geom);
    if (rc != PDC_OK) return rc;
    rc = check_params(params, nullptr, nullptr);
    if (rc != PDC_OK) return rc;
    rc = check_planes(geom, pedestal, gain);
    if (rc != PDC_OK) return rc;
    g_thread_error[0] = 0;
    return PDC_OK;
}

pdc_status pdc_calibrate(pdc_ctx *ctx, const pdc_geometry *geom, const float *pedestal,
                         const float *gain, const pdc_params *params, int32_t *det_out)
{
    if (!ctx || !det_out) return fail(ctx, PDC_EINVAL, "ctx and det_out must be non-NULL");
    pdc_status rc = pdc_check_calibration(geom, pedestal, gain, params);
    if (rc != PDC_OK) return fail(ctx, rc, "%s", g_thread_error);
    Detector d;
    d.g = *geom;
    d.p = *params;
    check_params(params, &d.t_seed, &d.t_nb);
    if (params->cm_mode != PDC_CM_MEDIAN) {
        volatile float tc = params->n_cm * params->sigma;  // binary32
        d.t_cm = tc;
        const bool tile = params->cm_mode == PDC_CM_TILE_MEAN;
        const uint64_t rsize = tile ? (uint64_t)geom->rows * geom->cols : (uint64_t)geom->bank_cols;
        volatile float rs = (float)rsize;
        d.cm_guard = std::sqrt((float)rs);
        d.cm_regions = tile ? (uint32_t)geom->n_tiles
                            : (uint32_t)((uint64_t)geom->n_tiles * geom->rows * (geom->cols / geom->bank_cols));
    }
    if (!plan_v1(d)) return fail(ctx, PDC_EINVAL, "geometry does not fit the kernel's on-chip budget");
    const size_t n = (size_t)n_ranges(*geom) * geom->n_tiles * geom->rows * geom->cols;
    std::vector<float> k(n);
    for (size_t i = 0; i < n; ++i) {
        volatile float r = 1.0f / gain[i];  // binary32 division
        k[i] = r;
    }
    if (params->cm_mode != PDC_CM_MEDIAN) frames1_window(pedestal, k.data(), n, &d.sum_lo, &d.sum_hi);
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, hipMalloc((void **)&d.d_ped, n * sizeof(float)));
    HIP_TRY(ctx, hipMalloc((void **)&d.d_k, n * sizeof(float)));
    HIP_TRY(ctx, hipMemcpy(d.d_ped, pedestal, n * sizeof(float), hipMemcpyHostToDevice));
    HIP_TRY(ctx, hipMemcpy(d.d_k, k.data(), n * sizeof(float), hipMemcpyHostToDevice));
    d.strip_cap = ctx->strip_rows;
    if (!ctx->force_v1) plan_v2(ctx, d);
    d.live = true;
    for (size_t i = 0; i < ctx->dets.size(); ++i)
        if (!ctx->dets[i].live) {
            ctx->dets[i] = d;
            *det_out = (int32_t)i;
            return PDC_OK;
        }
    ctx->dets.push_back(d);
    *det_out = (int32_t)ctx->dets.size() - 1;
    return PDC_OK;
}

pdc_status pdc_release_detector(pdc_ctx *ctx, int32_t det)
{
    if (!ctx) return fail(nullptr, PDC_EINVAL, "ctx is NULL");
    if (det < 0 || det >= (int32_t)ctx->dets.size() || !ctx->dets[det].live || ctx->dets[det].release_requested)
        return fail(ctx, PDC_ESTATE, "unknown detector %d", det);
    ctx->dets[det].release_requested = true;
    maybe_free_detector(ctx, det);
    return PDC_OK;
}

pdc_status process_batch(pdc_ctx *ctx, int32_t det, const uint16_t *frames_dev, uint64_t n_frames,
                         uint64_t hit_capacity, void *hip_stream, double share, uint64_t *batch_out);

pdc_status pdc_batch_bytes(pdc_ctx *ctx, int32_t det, uint64_t n_frames, uint64_t hit_capacity, uint64_t *bytes)
{
    if (!ctx || !bytes) return fail(ctx, PDC_EINVAL, "ctx and bytes must be non-NULL");
    if (det < 0 || det >= (int32_t)ctx->dets.size() || !ctx->dets[det].live || ctx->dets[det].release_requested)
        return fail(ctx, PDC_ESTATE, "unknown detector %d", det);
    if (n_frames > ((uint64_t)1 << 31)) return fail(ctx, PDC_EINVAL, "n_frames must be <= 2^31");
    const Detector &d = ctx->dets[det];
    Batch bt;
    bt.det = det;
    bt.n_frames = n_frames;
    set_path(d, bt, d.v2_ok ? 2 : 1);
    bt.keep = (d.p.flags & PDC_KEEP_CORRECTED) != 0;
    bt.meds = (d.p.flags & PDC_KEEP_MEDIANS) != 0;
    const uint64_t pool = pool_capacity(d, bt.path, hit_capacity, batch_grid(d, bt));
    uint64_t b = bt.n_units * (sizeof(uint32_t) + sizeof(unsigned long long) + sizeof(uint64_t) + sizeof(uint32_t));
    b += n_frames * (sizeof(uint32_t) + sizeof(unsigned long long)) + (n_frames + 1) * sizeof(unsigned long long);
    b += pool * 2 * sizeof(uint2);
    b += 4 * (corr_floats(d, bt) + cm_floats(d, bt) + meds_floats(d, bt));
    b += n_frames * sizeof(uint32_t) + bt.n_units * sizeof(uint64_t) + sizeof(BatchState);
    *bytes = b;
    return PDC_OK;
}

pdc_status pdc_process_frames(pdc_ctx *ctx, int32_t det, const uint16_t *frames_dev, uint64_t n_frames,
                              uint64_t hit_capacity, void *hip_stream, uint64_t *batch_out)
{
    return process_batch(ctx, det, frames_dev, n_frames, hit_capacity, hip_stream, 1.0, batch_out);
}

pdc_status pdc_process_frames_static(pdc_ctx *ctx, int32_t det, const uint16_t *frames_dev, uint64_t n_frames,
                                     pdc_hit *hits_dev, uint64_t hits_capacity, uint32_t *frame_hits_dev,
                                     uint64_t *frame_photons_dev, void *hip_stream, uint64_t *n_hits_total)
{
    if (!ctx) return fail(nullptr, PDC_EINVAL, "ctx is NULL");
    if (det < 0 || det >= (int32_t)ctx->dets.size() || !ctx->dets[det].live || ctx->dets[det].release_requested)
        return fail(ctx, PDC_ESTATE, "unknown detector %d", det);
    Detector &d = ctx->dets[det];
    if (d.p.flags & (PDC_KEEP_CORRECTED | PDC_KEEP_MEDIANS))
        return fail(ctx, PDC_EINVAL,
                    "static: a PDC_KEEP_CORRECTED or PDC_KEEP_MEDIANS detector needs pdc_process_frames (kept buffers)");
    if (n_frames == 0) {
        if (n_hits_total) *n_hits_total = 0;
        return PDC_OK;
    }
    if (!frames_dev || !frame_hits_dev || !frame_photons_dev || (hits_capacity > 0 && !hits_dev))
        return fail(ctx, PDC_EINVAL, "static: frames_dev, frame_hits_dev, frame_photons_dev (and hits_dev) must be non-NULL");
    if (n_frames > ((uint64_t)1 << 31)) return fail(ctx, PDC_EINVAL, "n_frames must be <= 2^31");
    unsigned char *base = ctx->device < kMaxDevices ? g_scratch_ptr[ctx->device] : nullptr;
    if (!base) return fail(ctx, PDC_EDEVICE, "static: no address of the static scratch on device %d", ctx->device);
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    Batch bt;
    bt.det = det;
    bt.frames = frames_dev;
    bt.n_frames = n_frames;
    set_path(d, bt, d.v2_ok ? 2 : 1);
    bt.stream = hip_stream ? (hipStream_t)hip_stream : ctx->stream;
    bt.capture = true;  // kernels only: no events, no copies to pinned memory
    bt.records = reinterpret_cast<HitRecord *>(hits_dev);
    bt.records_cap = hits_capacity;
    // carve the scratch: batch state, per-unit and per-frame arrays, the
    // common-mode values of the mean modes, then the staging pool
    Buffers b;
    uint64_t off = 0;
    bool fits = true;
    auto carve = [&](uint64_t bytes) -> unsigned char * {
        off = (off + 255) & ~(uint64_t)255;
        unsigned char *p = base + off;
        if (bytes > kStaticScratchBytes - std::min(off, kStaticScratchBytes)) fits = false;
        off += bytes;
        return p;
    };
    const uint64_t U = n_frames * (uint64_t)std::max(d.units_per_frame, d.n_strips);  // either path
    b.state = reinterpret_cast<BatchState *>(carve(sizeof(BatchState)));
    b.unit_count = reinterpret_cast<uint32_t *>(carve(4 * U));
    b.unit_photons = reinterpret_cast<unsigned long long *>(carve(8 * U));
    b.unit_base = reinterpret_cast<uint64_t *>(carve(8 * U));
    b.unit_local = reinterpret_cast<uint32_t *>(carve(4 * U));
    b.fb_units = reinterpret_cast<uint64_t *>(carve(8 * U));
    b.frame_offset = reinterpret_cast<unsigned long long *>(carve(8 * (n_frames + 1)));
    b.invalid = reinterpret_cast<uint32_t *>(carve(4 * n_frames));
    b.cm = reinterpret_cast<float *>(carve(4 * cm_floats(d, bt)));
    b.frame_hits = frame_hits_dev;
    b.frame_photons = reinterpret_cast<unsigned long long *>(frame_photons_dev);
    off = (off + 255) & ~(uint64_t)255;
    const uint64_t pool_bytes = fits && off < kStaticScratchBytes ? kStaticScratchBytes - off : 0;
    b.pool = reinterpret_cast<uint2 *>(base + std::min(off, kStaticScratchBytes));
    b.cap_pool = pool_bytes / sizeof(uint2);
    bt.buf = &b;
    // room for the staging chunks every workgroup may hold open
    const uint64_t slack = pool_capacity(d, bt.path, 0, batch_grid(d, bt));
    if (!fits || b.cap_pool <= slack)
        return fail(ctx, PDC_EINVAL,
                    "static: %llu frames need more than the %llu-byte static scratch (per-unit arrays and staging "
                    "slack); process fewer frames per call",
                    (unsigned long long)n_frames, (unsigned long long)kStaticScratchBytes);
    bt.pool_cap = b.cap_pool;
    BatchState st{};
    auto wait_state = [&]() -> pdc_status {
        HIP_TRY(ctx, hipMemcpyAsync(&st, b.state, sizeof st, hipMemcpyDeviceToHost, bt.stream));
        HIP_TRY(ctx, hipStreamSynchronize(bt.stream));
        return PDC_OK;
    };
    pdc_status rc = enqueue(ctx, bt);
    if (rc == PDC_OK) rc = wait_state();
    if (rc == PDC_OK && st.fallback && !st.overflow) {
        if (bt.path == 2 && d.fb_ok) {
            // strip-frames whose seeds overflowed the on-chip lists: the
            // general kernel redoes them into the same staging pool
            rc = enqueue_partial(ctx, bt, st.n_fallback);
        } else {
            set_path(d, bt, 1);
            rc = enqueue(ctx, bt);
        }
        if (rc == PDC_OK) rc = wait_state();
    }
    if (rc != PDC_OK) return rc;
    if (st.overflow)
        return fail(ctx, PDC_ENOMEM,
                    "static: the batch's hits overflow the staging pool of the static scratch (%llu entries); "
                    "process fewer frames per call",
                    (unsigned long long)bt.pool_cap);
    if (n_hits_total) *n_hits_total = st.total;
    return st.total > hits_capacity ? PDC_WARN_TRUNCATED : PDC_OK;
}

pdc_status pdc_process_mixed(pdc_ctx *ctx, const pdc_mixed_item *items, int32_t n_items, void *hip_stream,
                             uint64_t *batch_out)
{
    if (!ctx || !items || !batch_out || n_items < 1 || n_items > 64)
        return fail(ctx, PDC_EINVAL, "ctx, items and batch_out must be non-NULL, 1 <= n_items <= 64");
    for (int i = 0; i < n_items; ++i) {
        const int32_t det = items[i].det;
        if (det < 0 || det >= (int32_t)ctx->dets.size() || !ctx->dets[det].live || ctx->dets[det].release_requested)
            return fail(ctx, PDC_ESTATE, "item %d: unknown detector %d", i, det);
        if (items[i].n_frames > 0 && !items[i].frames_dev) return fail(ctx, PDC_EINVAL, "item %d: frames_dev is NULL", i);
    }
    if ((int)ctx->batches.size() + n_items > kMaxOutstandingBatches)
        return fail(ctx, PDC_ESTATE, "too many outstanding batches (release some)");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    const int n_str = std::min(n_items, 8);
    while ((int)ctx->mix_streams.size() < n_str) {
        hipStream_t st = nullptr;
        HIP_TRY(ctx, hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
        ctx->mix_streams.push_back(st);
    }
    while ((int)ctx->mix_events.size() < n_str + 1) {
        hipEvent_t ev = nullptr;
        HIP_TRY(ctx, hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        ctx->mix_events.push_back(ev);
    }
    // each batch is sized for the share of the chip its pixels are of the whole
    double work = 0.0;
    for (int i = 0; i < n_items; ++i) {
        const pdc_geometry &g = ctx->dets[items[i].det].g;
        work += (double)items[i].n_frames * g.n_tiles * g.rows * g.cols;
    }
    hipStream_t hs = hip_stream ? (hipStream_t)hip_stream : ctx->stream;
    std::vector<Batch> bts(n_items);
    std::vector<Batch *> ptrs(n_items);
    std::vector<int32_t> mix_dets;
    for (int i = 0; i < n_items; ++i) mix_dets.push_back(items[i].det);
    const int fg_more = mix_one_launch(ctx, mix_dets) ? kMixFgMore : 1;
    auto drop = [&](int upto) {
        for (int j = 0; j < upto; ++j) ctx->spare.push_back(bts[j].buf);
    };
    for (int i = 0; i < n_items; ++i) {
        const pdc_geometry &g = ctx->dets[items[i].det].g;
        const double px = (double)items[i].n_frames * g.n_tiles * g.rows * g.cols;
        const double share = ctx->mix_share && work > 0.0 ? std::min(1.0, px / work) : 1.0;
        pdc_status rc = setup_batch(ctx, items[i].det, items[i].frames_dev, items[i].n_frames, items[i].hit_capacity,
                                    ctx->mix_streams[i % n_str], share, bts[i], fg_more);
        if (rc != PDC_OK) {
            drop(i);
            return rc;
        }
        ptrs[i] = &bts[i];
    }
    const std::vector<hipStream_t> streams(ctx->mix_streams.begin(), ctx->mix_streams.begin() + n_str);
    pdc_status rc = enqueue_mixed(ctx, ptrs, hs, streams, ctx->mix_events);
    if (rc != PDC_OK) {
        drop(n_items);
        return rc;
    }
    for (int i = 0; i < n_items; ++i) batch_out[i] = register_batch(ctx, bts[i]);
    return PDC_OK;
}

pdc_status process_batch(pdc_ctx *ctx, int32_t det, const uint16_t *frames_dev, uint64_t n_frames,
                         uint64_t hit_capacity, void *hip_stream, double share, uint64_t *batch_out)
{
    if (!ctx || !batch_out) return fail(ctx, PDC_EINVAL, "ctx and batch_out must be non-NULL");
    if ((int)ctx->batches.size() >= kMaxOutstandingBatches)
        return fail(ctx, PDC_ESTATE, "too many outstanding batches (release some)");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    Batch bt;
    pdc_status rc = setup_batch(ctx, det, frames_dev, n_frames, hit_capacity,
                                hip_stream ? (hipStream_t)hip_stream : ctx->stream, share, bt);
    if (rc != PDC_OK) return rc;
    rc = enqueue(ctx, bt);
    if (rc != PDC_OK) {
        ctx->spare.push_back(bt.buf);
        return rc;
    }
    *batch_out = register_batch(ctx, bt);
    return PDC_OK;
}

pdc_status pdc_get_hits(pdc_ctx *ctx, uint64_t batch, pdc_hit *dst, uint64_t dst_capacity, int32_t dst_is_device,
                        uint64_t *n_hits_total, uint32_t *per_frame_hits, uint64_t *per_frame_photons)
{
    if (!ctx) return fail(nullptr, PDC_EINVAL, "ctx is NULL");
    Batch *bt = find_batch(ctx, batch);
    if (!bt) return fail(ctx, PDC_ESTATE, "unknown batch %llu", (unsigned long long)batch);
    if (dst_capacity > 0 && !dst) return fail(ctx, PDC_EINVAL, "dst is NULL with dst_capacity > 0");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    pdc_status rc = finish_batch(ctx, *bt);
    if (rc != PDC_OK) return rc;
    Buffers *b = bt->buf;
    hipStream_t cs = ctx->copy_stream;  // copies wait for this batch only
    HIP_TRY(ctx, hipStreamWaitEvent(cs, b->ev_end, 0));
    const uint64_t total = b->host_state->total;
    const float E = ctx->dets[bt->det].p.photon_adu;
    const uint64_t n_out = std::min<uint64_t>(total, dst_capacity);
    if (n_out > 0) {
        if (dst_is_device) {
            HIP_TRY(ctx, launch_format_hits(b->hits, b->frame_offset, bt->n_frames, 0, n_out, E,
                                            reinterpret_cast<HitRecord *>(dst), cs));
        } else {
            const uint64_t chunk = (uint64_t)1 << 24;
            if (!ctx->fmt_buf) HIP_TRY(ctx, grow(&ctx->fmt_buf, ctx->fmt_cap, std::min(chunk, n_out)));
            if (ctx->fmt_cap < std::min(chunk, n_out))
                HIP_TRY(ctx, grow(&ctx->fmt_buf, ctx->fmt_cap, std::min(chunk, n_out)));
            for (uint64_t first = 0; first < n_out; first += ctx->fmt_cap) {
                uint64_t n = std::min(ctx->fmt_cap, n_out - first);
                HIP_TRY(ctx, launch_format_hits(b->hits, b->frame_offset, bt->n_frames, first, n, E,
                                                ctx->fmt_buf, cs));
                HIP_TRY(ctx, hipMemcpyAsync(dst + first, ctx->fmt_buf, n * sizeof(pdc_hit),
                                            hipMemcpyDeviceToHost, cs));
                HIP_TRY(ctx, hipStreamSynchronize(cs));
            }
        }
    }
    if (per_frame_hits && bt->n_frames)
        HIP_TRY(ctx, hipMemcpyAsync(per_frame_hits, b->frame_hits, bt->n_frames * sizeof(uint32_t),
                                    hipMemcpyDeviceToHost, cs));
    if (per_frame_photons && bt->n_frames)
        HIP_TRY(ctx, hipMemcpyAsync(per_frame_photons, b->frame_photons, bt->n_frames * sizeof(uint64_t),
                                    hipMemcpyDeviceToHost, cs));
    HIP_TRY(ctx, hipStreamSynchronize(cs));
    if (n_hits_total) *n_hits_total = total;
    return total > dst_capacity ? PDC_WARN_TRUNCATED : PDC_OK;
}

pdc_status pdc_get_corrected(pdc_ctx *ctx, uint64_t batch, float *dst, int32_t dst_is_device)
{
    if (!ctx) return fail(nullptr, PDC_EINVAL, "ctx is NULL");
    Batch *bt = find_batch(ctx, batch);
    if (!bt) return fail(ctx, PDC_ESTATE, "unknown batch %llu", (unsigned long long)batch);
    if (!bt->keep) return fail(ctx, PDC_ESTATE, "batch was not processed with PDC_KEEP_CORRECTED");
    const Detector &d = ctx->dets[bt->det];
    const uint64_t n = bt->n_frames * (uint64_t)d.g.n_tiles * d.g.rows * d.g.cols;
    if (n > 0 && !dst) return fail(ctx, PDC_EINVAL, "dst is NULL");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    pdc_status rc = finish_batch(ctx, *bt);
    if (rc != PDC_OK) return rc;
    hipStream_t cs = ctx->copy_stream;
    HIP_TRY(ctx, hipStreamWaitEvent(cs, bt->buf->ev_end, 0));
    if (n > 0)
        HIP_TRY(ctx, hipMemcpyAsync(dst, bt->buf->corrected, n * sizeof(float),
                                    dst_is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                                    cs));
    HIP_TRY(ctx, hipStreamSynchronize(cs));
    return PDC_OK;
}

pdc_status pdc_release_batch(pdc_ctx *ctx, uint64_t batch)
{
    if (!ctx) return fail(nullptr, PDC_EINVAL, "ctx is NULL");
    Batch *bt = find_batch(ctx, batch);
    if (!bt) return fail(ctx, PDC_ESTATE, "unknown batch %llu", (unsigned long long)batch);
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, hipEventSynchronize(bt->buf->ev_state));
    if (bt->buf->used) HIP_TRY(ctx, hipEventSynchronize(bt->buf->ev_use));
    bt->buf->used = false;
    int32_t det = bt->det;
    if (bt->graph)
        bt->graph->batch[bt->gitem] = 0;  // the buffers stay with the graph
    else
        ctx->spare.push_back(bt->buf);
    ctx->batches.erase(batch);
    ctx->dets[det].pending -= 1;
    maybe_free_detector(ctx, det);
    return PDC_OK;
}

pdc_status pdc_stream_read(pdc_ctx *ctx, const void *src_dev, uint64_t bytes, void *hip_stream, float *ms_out)
{
    if (!ctx) return fail(nullptr, PDC_EINVAL, "ctx is NULL");
    if (!src_dev || bytes == 0 || bytes % 16 || ((uintptr_t)src_dev & 15))
        return fail(ctx, PDC_EINVAL, "stream_read: src must be 16-byte aligned and bytes a nonzero multiple of 16");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t s = hip_stream ? (hipStream_t)hip_stream : ctx->stream;
    uint32_t *out = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    pdc_status rc = PDC_OK;
    if (hipMalloc((void **)&out, sizeof(uint32_t)) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
        hipEventCreate(&e1) != hipSuccess)
        rc = fail(ctx, PDC_ENOMEM, "stream_read: no memory for its result or events");
    if (rc == PDC_OK && (launch_fill_u32(out, 1, s) != hipSuccess || hipEventRecord(e0, s) != hipSuccess ||
                         launch_stream_read(src_dev, bytes, out, (uint32_t)ctx->n_cu, s) != hipSuccess ||
                         hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess))
        rc = fail(ctx, PDC_EDEVICE, "stream_read: launch failed");
    float ms = 0;
    if (rc == PDC_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = fail(ctx, PDC_EDEVICE, "stream_read: timing");
    if (rc == PDC_OK && ms_out) *ms_out = ms;
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    hipFree(out);
    return rc;
}

pdc_status pdc_batch_timing(pdc_ctx *ctx, uint64_t batch, float *main_ms, float *total_ms)
{
    if (!ctx) return fail(nullptr, PDC_EINVAL, "ctx is NULL");
    Batch *bt = find_batch(ctx, batch);
    if (!bt) return fail(ctx, PDC_ESTATE, "unknown batch %llu", (unsigned long long)batch);
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, hipEventSynchronize(bt->buf->ev_end));
    float a = 0, t = 0;
    HIP_TRY(ctx, hipEventElapsedTime(&a, bt->buf->ev_cm, bt->buf->ev_main));
    HIP_TRY(ctx, hipEventElapsedTime(&t, bt->buf->ev_start, bt->buf->ev_end));
    if (main_ms) *main_ms = a;
    if (total_ms) *total_ms = t;
    return PDC_OK;
}

// ---------------------------------------------------------------------------
// graph capture of a batch
// ---------------------------------------------------------------------------

// Capture items[0..n) into one graph: one item on the capture stream itself,
// several on the mixed-batch streams forked from it and joined back.
static pdc_status graph_capture(pdc_ctx *ctx, const pdc_mixed_item *items, int32_t n_items, pdc_graph **out)
{
    if (!ctx || !out || !items || n_items < 1 || n_items > 64)
        return fail(ctx, PDC_EINVAL, "ctx, items and out must be non-NULL, 1 <= n_items <= 64");
    *out = nullptr;
    for (int i = 0; i < n_items; ++i) {
        const int32_t det = items[i].det;
        if (det < 0 || det >= (int32_t)ctx->dets.size() || !ctx->dets[det].live || ctx->dets[det].release_requested)
            return fail(ctx, PDC_ESTATE, "item %d: unknown detector %d", i, det);
        if (!items[i].frames_dev || items[i].n_frames < 1 || items[i].n_frames > ((uint64_t)1 << 31))
            return fail(ctx, PDC_EINVAL, "item %d: frames_dev must be non-NULL and 1 <= n_frames <= 2^31", i);
    }
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    if (!ctx->capture_stream) HIP_TRY(ctx, hipStreamCreateWithFlags(&ctx->capture_stream, hipStreamNonBlocking));
    const int n_str = n_items > 1 ? std::min(n_items, 8) : 0;
    while ((int)ctx->mix_streams.size() < n_str) {
        hipStream_t st = nullptr;
        HIP_TRY(ctx, hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
        ctx->mix_streams.push_back(st);
    }
    while ((int)ctx->mix_events.size() < n_str + 1) {
        hipEvent_t ev = nullptr;
        HIP_TRY(ctx, hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        ctx->mix_events.push_back(ev);
    }
    std::unique_ptr<pdc_graph> g(new (std::nothrow) pdc_graph);
    if (!g) return fail(ctx, PDC_ENOMEM, "host allocation failed");
    g->ctx = ctx;
    g->proto.resize(n_items);
    g->buf.assign(n_items, nullptr);
    g->batch.assign(n_items, 0);
    auto drop = [&]() {
        for (Buffers *b : g->buf) free_buffers(b);
    };
    double work = 0.0;
    for (int i = 0; i < n_items; ++i) {
        const pdc_geometry &gg = ctx->dets[items[i].det].g;
        work += (double)items[i].n_frames * gg.n_tiles * gg.rows * gg.cols;
    }
    std::vector<int32_t> mix_dets;
    for (int i = 0; i < n_items; ++i) mix_dets.push_back(items[i].det);
    const int fg_more = mix_one_launch(ctx, mix_dets) ? kMixFgMore : 1;
    for (int i = 0; i < n_items; ++i) {
        const Detector &d = ctx->dets[items[i].det];
        Batch &bt = g->proto[i];
        bt.det = items[i].det;
        bt.gitem = i;
        bt.fg_more = fg_more;
        bt.frames = items[i].frames_dev;
        bt.n_frames = items[i].n_frames;
        const double px = (double)items[i].n_frames * d.g.n_tiles * d.g.rows * d.g.cols;
        bt.share = n_items > 1 && ctx->mix_share && work > 0.0 ? std::min(1.0, px / work) : 1.0;
        set_path(d, bt, d.v2_ok ? 2 : 1);
        bt.keep = (d.p.flags & PDC_KEEP_CORRECTED) != 0;
        bt.meds = (d.p.flags & PDC_KEEP_MEDIANS) != 0;
        const uint64_t hc = items[i].hit_capacity;
        bt.pool_cap = ctx->tight_pool ? hc : pool_capacity(d, bt.path, hc, batch_grid(d, bt));
        g->buf[i] = new (std::nothrow) Buffers;
        if (!g->buf[i]) {
            drop();
            return fail(ctx, PDC_ENOMEM, "host allocation failed");
        }
        pdc_status rc = ensure_buffers(ctx, g->buf[i], bt.n_units, bt.n_frames, bt.pool_cap, corr_floats(d, bt),
                                       cm_floats(d, bt), meds_floats(d, bt));
        if (rc != PDC_OK) {
            drop();
            return rc;
        }
        bt.buf = g->buf[i];
        bt.capture = true;
        bt.stream = n_str ? ctx->mix_streams[i % n_str] : ctx->capture_stream;
    }
    hipStream_t cs = ctx->capture_stream;
    // relaxed: the launch helpers may set kernel attributes while capturing
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess) {
        drop();
        return fail(ctx, PDC_EDEVICE, "hipStreamBeginCapture: %s", hipGetErrorString(e));
    }
    pdc_status rc = PDC_OK;
    // the forked streams join the capture by waiting for an event recorded in
    // it, and are joined back (enqueue_mixed joins them also after a failed
    // enqueue, so that no stream is left capturing)
    if (n_str) {
        std::vector<Batch *> ptrs;
        for (Batch &bt : g->proto) ptrs.push_back(&bt);
        const std::vector<hipStream_t> streams(ctx->mix_streams.begin(), ctx->mix_streams.begin() + n_str);
        rc = enqueue_mixed(ctx, ptrs, cs, streams, ctx->mix_events);
    } else {
        for (int i = 0; rc == PDC_OK && i < n_items; ++i) rc = enqueue(ctx, g->proto[i]);
    }
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(cs, &graph);
    if (rc == PDC_OK && e != hipSuccess) rc = fail(ctx, PDC_EDEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
    if (rc == PDC_OK) {
        e = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
        if (e != hipSuccess) rc = fail(ctx, PDC_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
    }
    if (rc != PDC_OK) {
        if (graph) hipGraphDestroy(graph);
        drop();
        return rc;
    }
    g->graph = graph;
    for (Batch &bt : g->proto) {
        bt.capture = false;
        bt.stream = nullptr;
        ctx->dets[bt.det].pending += 1;  // the graph holds the detector's planes
    }
    ctx->graphs.insert(g.get());
    *out = g.release();
    return PDC_OK;
}

pdc_status pdc_graph_create(pdc_ctx *ctx, int32_t det, const uint16_t *frames_dev, uint64_t n_frames,
                            uint64_t hit_capacity, pdc_graph **out)
{
    const pdc_mixed_item item{det, frames_dev, n_frames, hit_capacity};
    return graph_capture(ctx, &item, 1, out);
}

pdc_status pdc_graph_create_mixed(pdc_ctx *ctx, const pdc_mixed_item *items, int32_t n_items, pdc_graph **out)
{
    return graph_capture(ctx, items, n_items, out);
}

int32_t pdc_graph_items(const pdc_graph *g)
{
    return g ? (int32_t)g->proto.size() : 0;
}

pdc_status pdc_graph_launch(pdc_graph *g, void *hip_stream, uint64_t *batch_out)
{
    if (!g || !batch_out) return fail(g ? g->ctx : nullptr, PDC_EINVAL, "graph and batch_out must be non-NULL");
    pdc_ctx *ctx = g->ctx;
    if (g->busy()) return fail(ctx, PDC_ESTATE, "a batch of this graph is not released");
    const int n = (int)g->proto.size();
    if ((int)ctx->batches.size() + n > kMaxOutstandingBatches)
        return fail(ctx, PDC_ESTATE, "too many outstanding batches (release some)");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t s = hip_stream ? (hipStream_t)hip_stream : ctx->stream;
    // the graph holds kernels only: events and the state copies go around it
    for (int i = 0; i < n; ++i) {
        HIP_TRY(ctx, hipEventRecord(g->buf[i]->ev_start, s));
        HIP_TRY(ctx, hipEventRecord(g->buf[i]->ev_cm, s));
    }
    HIP_TRY(ctx, hipGraphLaunch(g->exec, s));
    for (int i = 0; i < n; ++i) {
        HIP_TRY(ctx, hipEventRecord(g->buf[i]->ev_main, s));
        pdc_status rc = record_end(ctx, g->buf[i], s);
        if (rc != PDC_OK) return rc;
    }
    for (int i = 0; i < n; ++i) {
        Batch bt = g->proto[i];
        bt.id = ctx->next_batch++;
        bt.stream = s;
        bt.buf = g->buf[i];
        bt.graph = g;
        ctx->dets[bt.det].pending += 1;
        ctx->batches[bt.id] = bt;
        g->batch[i] = bt.id;
        batch_out[i] = bt.id;
    }
    return PDC_OK;
}

pdc_status pdc_graph_destroy(pdc_graph *g)
{
    if (!g) return PDC_OK;
    pdc_ctx *ctx = g->ctx;
    if (g->busy()) return fail(ctx, PDC_ESTATE, "a batch of this graph is not released");
    // released batches have finished with the buffers (pdc_release_batch waits)
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipGraphExecDestroy(g->exec);
    hipGraphDestroy(g->graph);
    for (Buffers *b : g->buf) free_buffers(b);
    ctx->graphs.erase(g);
    std::vector<int32_t> dets;
    for (const Batch &bt : g->proto) dets.push_back(bt.det);
    delete g;
    for (int32_t det : dets) {
        ctx->dets[det].pending -= 1;
        maybe_free_detector(ctx, det);
    }
    return PDC_OK;
}

// ---------------------------------------------------------------------------
// subpixel stage
// ---------------------------------------------------------------------------

}  // extern "C"

namespace {

// The network's input scale 1/photon_adu, rounded once to binary32.
float inv_adu_of(float photon_adu) { return (float)(1.0 / (double)photon_adu); }

// Where a batch's Frames2 values are formed again from (kept medians or
// thresholded-mean stage values).
PatchSrc patch_src(const Detector &d, const Batch &bt)
{
    PatchSrc ps{};
    ps.frames = bt.frames;
    ps.ped = d.d_ped;
    ps.k = d.d_k;
    ps.T = d.g.n_tiles;
    ps.H = d.g.rows;
    ps.W = d.g.cols;
    ps.B = d.g.bank_cols;
    ps.nb = d.g.cols / d.g.bank_cols;
    ps.gain_mode = d.g.gain_mode;
    ps.meds = d.p.cm_mode ? nullptr : bt.buf->meds;
    ps.cm = d.p.cm_mode ? bt.buf->cm : nullptr;
    ps.cm_regions = d.cm_regions;
    ps.cm_tile = d.p.cm_mode == PDC_CM_TILE_MEAN;
    return ps;
}

// Patches (float32, patches != NULL) or network inputs (bf16 words) of the
// batch's first min(total, capacity) hits.
pdc_status capture(pdc_ctx *ctx, uint64_t batch, float *patches, uint16_t *inputs, float inv_adu, uint64_t capacity,
                   uint64_t *n_out)
{
    Batch *bt = find_batch(ctx, batch);
    if (!bt) return fail(ctx, PDC_ESTATE, "unknown batch %llu", (unsigned long long)batch);
    if (!bt->keep && !bt->meds)
        return fail(ctx, PDC_ESTATE, "batch was processed with neither PDC_KEEP_CORRECTED nor PDC_KEEP_MEDIANS");
    if (capacity > 0 && !patches && !inputs) return fail(ctx, PDC_EINVAL, "output pointer is NULL with capacity > 0");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    pdc_status rc = finish_batch(ctx, *bt);
    if (rc != PDC_OK) return rc;
    const Detector &d = ctx->dets[bt->det];
    Buffers *b = bt->buf;
    hipStream_t cs = ctx->copy_stream;
    HIP_TRY(ctx, hipStreamWaitEvent(cs, b->ev_end, 0));
    const uint64_t n = std::min<uint64_t>(b->host_state->total, capacity);
    if (bt->keep) {
        HIP_TRY(ctx, launch_capture_patches(b->corrected, b->hits, b->frame_offset, bt->n_frames, n, d.g.n_tiles,
                                            d.g.rows, d.g.cols, patches, inputs, inv_adu, cs));
    } else {
        HIP_TRY(ctx, launch_patches_from_frames(patch_src(d, *bt), b->hits, b->frame_offset, bt->n_frames, n, patches,
                                                inputs, inv_adu, cs));
    }
    HIP_TRY(ctx, hipStreamSynchronize(cs));
    if (n_out) *n_out = n;
    return PDC_OK;
}

}  // namespace

extern "C" {

pdc_status pdc_capture_patches(pdc_ctx *ctx, uint64_t batch, float *patches_dev, uint64_t capacity, uint64_t *n_out)
{
    if (!ctx) return fail(nullptr, PDC_EINVAL, "ctx is NULL");
    if (capacity > 0 && !patches_dev) return fail(ctx, PDC_EINVAL, "patches_dev is NULL with capacity > 0");
    return capture(ctx, batch, patches_dev, nullptr, 0.0f, capacity, n_out);
}

pdc_status pdc_capture_inputs(pdc_ctx *ctx, uint64_t batch, float photon_adu, uint16_t *inputs_dev, uint64_t capacity,
                              uint64_t *n_out)
{
    if (!ctx) return fail(nullptr, PDC_EINVAL, "ctx is NULL");
    if (capacity > 0 && !inputs_dev) return fail(ctx, PDC_EINVAL, "inputs_dev is NULL with capacity > 0");
    if (!finite_in(photon_adu, 0x1p-24f, 0x1p24f)) return fail(ctx, PDC_EINVAL, "photon_adu must be in [2^-24, 2^24]");
    return capture(ctx, batch, nullptr, inputs_dev, inv_adu_of(photon_adu), capacity, n_out);
}

pdc_status pdc_capture_centroids(pdc_ctx *ctx, uint64_t batch, float t_nb, const float *eta_dev, int32_t nbins,
                                 float *positions_dev, uint64_t capacity, int32_t only_implausible, uint64_t *n_out)
{
    if (!ctx) return fail(nullptr, PDC_EINVAL, "ctx is NULL");
    if (capacity > 0 && !positions_dev) return fail(ctx, PDC_EINVAL, "positions_dev is NULL with capacity > 0");
    if (!std::isfinite(t_nb)) return fail(ctx, PDC_EINVAL, "t_nb must be finite");
    if (eta_dev && (nbins < 1 || nbins > 65536)) return fail(ctx, PDC_EINVAL, "nbins must be in [1, 65536]");
    Batch *bt = find_batch(ctx, batch);
    if (!bt) return fail(ctx, PDC_ESTATE, "unknown batch %llu", (unsigned long long)batch);
    if (!bt->keep && !bt->meds)
        return fail(ctx, PDC_ESTATE, "batch was processed with neither PDC_KEEP_CORRECTED nor PDC_KEEP_MEDIANS");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    pdc_status rc = finish_batch(ctx, *bt);
    if (rc != PDC_OK) return rc;
    const Detector &d = ctx->dets[bt->det];
    Buffers *b = bt->buf;
    hipStream_t cs = ctx->copy_stream;
    HIP_TRY(ctx, hipStreamWaitEvent(cs, b->ev_end, 0));
    const uint64_t n = std::min<uint64_t>(b->host_state->total, capacity);
    HIP_TRY(ctx, launch_centroids(patch_src(d, *bt), bt->keep ? b->corrected : nullptr, b->hits, b->frame_offset,
                                  bt->n_frames, n, t_nb, eta_dev, nbins, only_implausible ? 1 : 0, positions_dev, cs));
    HIP_TRY(ctx, hipStreamSynchronize(cs));
    if (n_out) *n_out = n;
    return PDC_OK;
}

pdc_status pdc_mlp_make_inputs(pdc_ctx *ctx, const float *patches_dev, uint64_t n, float photon_adu,
                               uint16_t *inputs_dev, void *hip_stream)
{
    if (!ctx) return fail(nullptr, PDC_EINVAL, "ctx is NULL");
    if (n > 0 && (!patches_dev || !inputs_dev)) return fail(ctx, PDC_EINVAL, "device pointers must be non-NULL");
    if (!finite_in(photon_adu, 0x1p-24f, 0x1p24f)) return fail(ctx, PDC_EINVAL, "photon_adu must be in [2^-24, 2^24]");
    if (n > ((uint64_t)1 << 36)) return fail(ctx, PDC_EINVAL, "n too large");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t s = hip_stream ? (hipStream_t)hip_stream : ctx->stream;
    HIP_TRY(ctx, launch_make_inputs(patches_dev, n, inv_adu_of(photon_adu), inputs_dev, s));
    return PDC_OK;
}

pdc_status pdc_centroid(pdc_ctx *ctx, const float *patches_dev, uint64_t n, float t_nb, const float *eta_dev,
                        int32_t nbins, float *out_dev, void *hip_stream)
{
    if (!ctx) return fail(nullptr, PDC_EINVAL, "ctx is NULL");
    if (n > 0 && (!patches_dev || !out_dev)) return fail(ctx, PDC_EINVAL, "patches_dev and out_dev must be non-NULL");
    if (!std::isfinite(t_nb)) return fail(ctx, PDC_EINVAL, "t_nb must be finite");
    if (eta_dev && (nbins < 1 || nbins > 65536)) return fail(ctx, PDC_EINVAL, "nbins must be in [1, 65536]");
    if (n > ((uint64_t)1 << 36)) return fail(ctx, PDC_EINVAL, "n too large");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t s = hip_stream ? (hipStream_t)hip_stream : ctx->stream;
    HIP_TRY(ctx, launch_centroid_eta(patches_dev, n, t_nb, eta_dev, nbins, out_dev, s));
    return PDC_OK;
}

pdc_status pdc_eta_table(pdc_ctx *ctx, const float *patches_dev, uint64_t n, float t_nb, int32_t nbins,
                         uint32_t *workspace_dev, float *table_dev, void *hip_stream)
{
    if (!ctx) return fail(nullptr, PDC_EINVAL, "ctx is NULL");
    if ((n > 0 && !patches_dev) || !workspace_dev || !table_dev)
        return fail(ctx, PDC_EINVAL, "patches_dev, workspace_dev and table_dev must be non-NULL");
    if (!std::isfinite(t_nb)) return fail(ctx, PDC_EINVAL, "t_nb must be finite");
    if (nbins < 1 || nbins > 65536) return fail(ctx, PDC_EINVAL, "nbins must be in [1, 65536]");
    if (n > ((uint64_t)1 << 36)) return fail(ctx, PDC_EINVAL, "n too large");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t s = hip_stream ? (hipStream_t)hip_stream : ctx->stream;
    HIP_TRY(ctx, launch_eta_table(patches_dev, n, t_nb, nbins, workspace_dev, table_dev, s));
    return PDC_OK;
}

}  // extern "C"

struct pdc_mlp {
    pdc_ctx *ctx = nullptr;
    float *theta = nullptr, *m = nullptr, *v = nullptr;
    float *grad = nullptr;    // kMlpParams gradient + 1 loss sum
    float *slots = nullptr;   // per-wave partial gradients
    uint16_t *packed = nullptr;
    uint32_t max_grid = 0;
    int64_t step = 0;
    uint64_t last_n = 0;
    hipEvent_t done = nullptr;  // after the network's last enqueued work (calls on it are ordered)
};

namespace {

bool mlp_theta_ok(const float *theta)
{
    for (int i = 0; i < kMlpParams; ++i)
        if (!std::isfinite(theta[i])) return false;
    return true;
}

void mlp_free(pdc_mlp *net)
{
    hipFree(net->theta);
    hipFree(net->m);
    hipFree(net->v);
    hipFree(net->grad);
    hipFree(net->slots);
    hipFree(net->packed);
    if (net->done) hipEventDestroy(net->done);
    delete net;
}

pdc_status mlp_check_run(pdc_mlp *net, const float *patches_dev, const float *target_dev, bool need_target,
                         uint64_t n, float photon_adu)
{
    pdc_ctx *ctx = net->ctx;
    if (n > 0 && (!patches_dev || (need_target && !target_dev)))
        return fail(ctx, PDC_EINVAL, "device pointers must be non-NULL");
    if (!finite_in(photon_adu, 0x1p-24f, 0x1p24f)) return fail(ctx, PDC_EINVAL, "photon_adu must be in [2^-24, 2^24]");
    if (n > ((uint64_t)1 << 36)) return fail(ctx, PDC_EINVAL, "n too large");
    return PDC_OK;
}

}  // namespace

extern "C" {

pdc_status pdc_mlp_create(pdc_ctx *ctx, const float *theta_host, pdc_mlp **out)
{
    if (!ctx || !theta_host || !out) return fail(ctx, PDC_EINVAL, "ctx, theta_host and out must be non-NULL");
    if (!mlp_theta_ok(theta_host)) return fail(ctx, PDC_EINVAL, "theta has a non-finite value");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    pdc_mlp *net = new (std::nothrow) pdc_mlp;
    if (!net) return fail(ctx, PDC_ENOMEM, "host allocation failed");
    net->ctx = ctx;
    net->max_grid = (uint32_t)std::max(1, ctx->n_cu);
    const size_t pbytes = sizeof(float) * kMlpParams;
    hipError_t e = hipMalloc((void **)&net->theta, pbytes);
    if (e == hipSuccess) e = hipMalloc((void **)&net->m, pbytes);
    if (e == hipSuccess) e = hipMalloc((void **)&net->v, pbytes);
    if (e == hipSuccess) e = hipMalloc((void **)&net->grad, pbytes + sizeof(float));
    if (e == hipSuccess) e = hipMalloc((void **)&net->slots, sizeof(float) * kMlpSlotStride * 4 * (size_t)net->max_grid);
    if (e == hipSuccess) e = hipMalloc((void **)&net->packed, sizeof(uint16_t) * kPackElems);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&net->done, hipEventDisableTiming);
    if (e != hipSuccess) {
        mlp_free(net);
        return fail(ctx, e == hipErrorOutOfMemory ? PDC_ENOMEM : PDC_EDEVICE, "device allocation failed: %s",
                    hipGetErrorString(e));
    }
    pdc_status rc = pdc_mlp_set_params(net, theta_host);
    if (rc != PDC_OK) {
        mlp_free(net);
        return rc;
    }
    *out = net;
    return PDC_OK;
}

pdc_status pdc_mlp_destroy(pdc_mlp *net)
{
    if (!net) return PDC_OK;
    hipSetDevice(net->ctx->device);
    hipEventSynchronize(net->done);
    mlp_free(net);
    return PDC_OK;
}

pdc_status pdc_mlp_set_params(pdc_mlp *net, const float *theta_host)
{
    if (!net || !theta_host) return fail(net ? net->ctx : nullptr, PDC_EINVAL, "net and theta_host must be non-NULL");
    pdc_ctx *ctx = net->ctx;
    if (!mlp_theta_ok(theta_host)) return fail(ctx, PDC_EINVAL, "theta has a non-finite value");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    HIP_TRY(ctx, hipEventSynchronize(net->done));  // the network's earlier work, on whatever stream
    HIP_TRY(ctx, hipMemcpyAsync(net->theta, theta_host, sizeof(float) * kMlpParams, hipMemcpyHostToDevice, s));
    HIP_TRY(ctx, launch_fill_zero(net->m, kMlpParams, s));
    HIP_TRY(ctx, launch_fill_zero(net->v, kMlpParams, s));
    HIP_TRY(ctx, launch_mlp_pack(net->theta, net->packed, s));
    HIP_TRY(ctx, hipEventRecord(net->done, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    net->step = 0;
    net->last_n = 0;
    return PDC_OK;
}

pdc_status pdc_mlp_get_params(pdc_mlp *net, float *theta_host)
{
    if (!net || !theta_host) return fail(net ? net->ctx : nullptr, PDC_EINVAL, "net and theta_host must be non-NULL");
    pdc_ctx *ctx = net->ctx;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, hipEventSynchronize(net->done));
    HIP_TRY(ctx, hipMemcpy(theta_host, net->theta, sizeof(float) * kMlpParams, hipMemcpyDeviceToHost));
    return PDC_OK;
}

pdc_status pdc_mlp_infer(pdc_mlp *net, const float *patches_dev, uint64_t n, float photon_adu, float *out_dev,
                         void *hip_stream)
{
    if (!net) return fail(nullptr, PDC_EINVAL, "net is NULL");
    pdc_ctx *ctx = net->ctx;
    pdc_status rc = mlp_check_run(net, patches_dev, nullptr, false, n, photon_adu);
    if (rc != PDC_OK) return rc;
    if (n > 0 && !out_dev) return fail(ctx, PDC_EINVAL, "out_dev is NULL");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t s = hip_stream ? (hipStream_t)hip_stream : ctx->stream;
    HIP_TRY(ctx, launch_mlp_infer(patches_dev, n, inv_adu_of(photon_adu), net->theta, net->packed, out_dev,
                                  8u * (uint32_t)ctx->n_cu, s));
    HIP_TRY(ctx, hipEventRecord(net->done, s));
    return PDC_OK;
}

pdc_status pdc_mlp_infer_inputs(pdc_mlp *net, const uint16_t *inputs_dev, uint64_t n, float *out_dev,
                                void *hip_stream)
{
    if (!net) return fail(nullptr, PDC_EINVAL, "net is NULL");
    pdc_ctx *ctx = net->ctx;
    if (n > 0 && (!inputs_dev || !out_dev)) return fail(ctx, PDC_EINVAL, "device pointers must be non-NULL");
    if (n > ((uint64_t)1 << 36)) return fail(ctx, PDC_EINVAL, "n too large");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t s = hip_stream ? (hipStream_t)hip_stream : ctx->stream;
    HIP_TRY(ctx, launch_mlp_infer_inputs(inputs_dev, n, net->theta, net->packed, out_dev, 8u * (uint32_t)ctx->n_cu, s));
    HIP_TRY(ctx, hipEventRecord(net->done, s));
    return PDC_OK;
}

pdc_status pdc_mlp_gradient(pdc_mlp *net, const float *patches_dev, const float *target_dev, uint64_t n,
                            float photon_adu, float *grad_host, double *loss_host, void *hip_stream)
{
    if (!net) return fail(nullptr, PDC_EINVAL, "net is NULL");
    pdc_ctx *ctx = net->ctx;
    pdc_status rc = mlp_check_run(net, patches_dev, target_dev, true, n, photon_adu);
    if (rc != PDC_OK) return rc;
    if (n == 0) return fail(ctx, PDC_EINVAL, "n must be >= 1");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t s = hip_stream ? (hipStream_t)hip_stream : ctx->stream;
    HIP_TRY(ctx, launch_mlp_grad(patches_dev, target_dev, n, inv_adu_of(photon_adu), net->theta, net->packed,
                                 net->grad, net->slots, net->max_grid, s));
    std::vector<float> h(kMlpParams + 1);
    HIP_TRY(ctx, hipMemcpyAsync(h.data(), net->grad, sizeof(float) * h.size(), hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipEventRecord(net->done, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    if (grad_host) std::memcpy(grad_host, h.data(), sizeof(float) * kMlpParams);
    if (loss_host) *loss_host = (double)h[kMlpParams] / (2.0 * (double)n);
    return PDC_OK;
}

pdc_status pdc_mlp_train_step(pdc_mlp *net, const float *patches_dev, const float *target_dev, uint64_t n,
                              float photon_adu, float lr, void *hip_stream)
{
    if (!net) return fail(nullptr, PDC_EINVAL, "net is NULL");
    pdc_ctx *ctx = net->ctx;
    pdc_status rc = mlp_check_run(net, patches_dev, target_dev, true, n, photon_adu);
    if (rc != PDC_OK) return rc;
    if (n == 0) return fail(ctx, PDC_EINVAL, "n must be >= 1");
    if (!(std::isfinite(lr) && lr >= 0.0f)) return fail(ctx, PDC_EINVAL, "lr must be finite and >= 0");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t s = hip_stream ? (hipStream_t)hip_stream : ctx->stream;
    HIP_TRY(ctx, launch_mlp_train(patches_dev, target_dev, n, inv_adu_of(photon_adu), net->theta, net->m, net->v,
                                  net->packed, net->grad, net->slots, net->max_grid, lr, net->step + 1, s));
    HIP_TRY(ctx, hipEventRecord(net->done, s));
    net->step += 1;
    net->last_n = n;
    return PDC_OK;
}

pdc_status pdc_mlp_last_loss(pdc_mlp *net, double *loss)
{
    if (!net || !loss) return fail(net ? net->ctx : nullptr, PDC_EINVAL, "net and loss must be non-NULL");
    pdc_ctx *ctx = net->ctx;
    if (net->last_n == 0) return fail(ctx, PDC_ESTATE, "no training step yet");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, hipEventSynchronize(net->done));
    float l = 0.0f;
    HIP_TRY(ctx, hipMemcpy(&l, net->grad + kMlpParams, sizeof(float), hipMemcpyDeviceToHost));
    *loss = (double)l / (2.0 * (double)net->last_n);
    return PDC_OK;
}

// Test hook (not in pdc.h): one 16x32 by 32x16 bf16 MFMA product through the
// kernels' operand loads.  A, B (uint16 bf16 bits, row-major) and D (float32
// [16][16]) are host arrays.
pdc_status pdc_debug_mfma_probe(pdc_ctx *ctx, const uint16_t *A, const uint16_t *B, float *D)
{
    if (!ctx || !A || !B || !D) return fail(ctx, PDC_EINVAL, "NULL argument");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    uint16_t *dA = nullptr, *dB = nullptr;
    float *dD = nullptr;
    HIP_TRY(ctx, hipMalloc((void **)&dA, 2 * 16 * 32));
    HIP_TRY(ctx, hipMalloc((void **)&dB, 2 * 32 * 16));
    HIP_TRY(ctx, hipMalloc((void **)&dD, 4 * 16 * 16));
    hipStream_t s = ctx->stream;
    hipError_t e = hipMemcpyAsync(dA, A, 2 * 16 * 32, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(dB, B, 2 * 32 * 16, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = launch_mfma_probe(dA, dB, dD, s);
    if (e == hipSuccess) e = hipMemcpyAsync(D, dD, 4 * 16 * 16, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    hipFree(dA);
    hipFree(dB);
    hipFree(dD);
    if (e != hipSuccess) return fail(ctx, PDC_EDEVICE, "mfma probe: %s", hipGetErrorString(e));
    return PDC_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Summaries
// ---------------------------------------------------------------------------
namespace {

pdc_status check_bins(pdc_ctx *ctx, float lo, float hi, int32_t nbins, float *scale)
{
    if (nbins < 1 || nbins > (1 << 24)) return fail(ctx, PDC_EINVAL, "nbins must be in [1, 2^24]");
    if (!(std::isfinite(lo) && std::isfinite(hi) && lo < hi)) return fail(ctx, PDC_EINVAL, "need finite lo < hi");
    volatile float w = hi - lo;  // binary32
    volatile float sc = (float)nbins / w;
    if (!std::isfinite(w) || !(std::isfinite(sc) && sc > 0.0f))
        return fail(ctx, PDC_EINVAL, "nbins / (hi - lo) is not a finite positive binary32 value");
    *scale = sc;
    return PDC_OK;
}

}  // namespace

extern "C" {

pdc_status pdc_accumulate_hits(pdc_ctx *ctx, uint64_t batch, uint32_t *count_map_dev, uint32_t *spectrum_dev,
                               uint32_t *size_spectra_dev, float lo, float hi, int32_t nbins, void *hip_stream)
{
    if (!ctx) return fail(nullptr, PDC_EINVAL, "ctx is NULL");
    Batch *bt = find_batch(ctx, batch);
    if (!bt) return fail(ctx, PDC_ESTATE, "unknown batch %llu", (unsigned long long)batch);
    if (size_spectra_dev && !bt->keep)
        return fail(ctx, PDC_ESTATE, "size spectra need a batch processed with PDC_KEEP_CORRECTED");
    float scale = 1.0f;
    if (spectrum_dev || size_spectra_dev) {
        pdc_status rc = check_bins(ctx, lo, hi, nbins, &scale);
        if (rc != PDC_OK) return rc;
    }
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    pdc_status rc = finish_batch(ctx, *bt);
    if (rc != PDC_OK) return rc;
    const Detector &d = ctx->dets[bt->det];
    Buffers *b = bt->buf;
    hipStream_t s = hip_stream ? (hipStream_t)hip_stream : ctx->stream;
    HIP_TRY(ctx, hipStreamWaitEvent(s, b->ev_end, 0));
    AccumulateArgs a{};
    a.hits = b->hits;
    a.n = b->host_state->total;
    a.photon_adu = d.p.photon_adu;
    a.count_map = count_map_dev;
    a.spectrum = spectrum_dev;
    a.size_spectra = size_spectra_dev;
    a.lo = lo;
    a.scale = scale;
    a.nbins = (uint32_t)nbins;
    a.corrected = b->corrected;
    a.frame_offset = b->frame_offset;
    a.n_frames = bt->n_frames;
    a.T = d.g.n_tiles;
    a.H = d.g.rows;
    a.W = d.g.cols;
    a.t_nb = d.t_nb;
    HIP_TRY(ctx, launch_accumulate_hits(a, (uint32_t)ctx->n_cu * 8, s));
    HIP_TRY(ctx, hipEventRecord(b->ev_use, s));
    b->used = true;
    return PDC_OK;
}

pdc_status pdc_histogram_corrected(pdc_ctx *ctx, uint64_t batch, uint32_t *hist_dev, float lo, float hi,
                                   int32_t nbins, void *hip_stream)
{
    if (!ctx) return fail(nullptr, PDC_EINVAL, "ctx is NULL");
    Batch *bt = find_batch(ctx, batch);
    if (!bt) return fail(ctx, PDC_ESTATE, "unknown batch %llu", (unsigned long long)batch);
    if (!bt->keep) return fail(ctx, PDC_ESTATE, "batch was not processed with PDC_KEEP_CORRECTED");
    if (!hist_dev) return fail(ctx, PDC_EINVAL, "hist_dev is NULL");
    float scale = 1.0f;
    pdc_status rc = check_bins(ctx, lo, hi, nbins, &scale);
    if (rc != PDC_OK) return rc;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    rc = finish_batch(ctx, *bt);
    if (rc != PDC_OK) return rc;
    const Detector &d = ctx->dets[bt->det];
    Buffers *b = bt->buf;
    hipStream_t s = hip_stream ? (hipStream_t)hip_stream : ctx->stream;
    HIP_TRY(ctx, hipStreamWaitEvent(s, b->ev_end, 0));
    const uint64_t n = bt->n_frames * (uint64_t)d.g.n_tiles * d.g.rows * d.g.cols;
    HIP_TRY(ctx, launch_histogram(b->corrected, n, lo, scale, (uint32_t)nbins, hist_dev, (uint32_t)ctx->n_cu * 8, s));
    HIP_TRY(ctx, hipEventRecord(b->ev_use, s));
    b->used = true;
    return PDC_OK;
}

pdc_status pdc_dark_stats(pdc_ctx *ctx, const pdc_geometry *geom, const uint16_t *darks_dev, uint64_t n_frames,
                          float *pedestal_host, float *noise_host, void *hip_stream)
{
    if (!ctx) return fail(nullptr, PDC_EINVAL, "ctx is NULL");
    pdc_status rc = check_geometry(geom);
    if (rc != PDC_OK) return fail(ctx, rc, "%s", g_thread_error);
    if (n_frames < 2 || n_frames >= ((uint64_t)1 << 32)) return fail(ctx, PDC_EINVAL, "need 2 <= n_frames < 2^32");
    if (!darks_dev || !pedestal_host) return fail(ctx, PDC_EINVAL, "darks_dev and pedestal_host must be non-NULL");
    const uint64_t px = (uint64_t)geom->n_tiles * geom->rows * geom->cols;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t s = hip_stream ? (hipStream_t)hip_stream : ctx->stream;
    unsigned long long *sums = nullptr;
    HIP_TRY(ctx, hipMalloc((void **)&sums, 2 * px * sizeof(unsigned long long)));
    std::vector<uint64_t> s12(2 * px);
    hipError_t e = launch_dark_sums(darks_dev, n_frames, px, sums, sums + px, (uint32_t)ctx->n_cu, s);
    if (e == hipSuccess) e = hipMemcpyAsync(s12.data(), sums, 2 * px * sizeof(uint64_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    hipFree(sums);
    if (e != hipSuccess) return fail(ctx, PDC_EDEVICE, "dark sums: %s", hipGetErrorString(e));
    // pedestal = S1 / n and noise = sqrt((n S2 - S1^2) / (n (n - 1))): the
    // quotients and the root in IEEE double from exact integers, then binary32
    const double dn = (double)n_frames, dnn = (double)n_frames * (double)(n_frames - 1);
    for (uint64_t p = 0; p < px; ++p) {
        const uint64_t a = s12[p], q = s12[px + p];
        volatile double m = (double)a / dn;  // a < 2^46: exact operands
        pedestal_host[p] = (float)m;
        if (noise_host) {
            const unsigned __int128 num = (unsigned __int128)n_frames * q - (unsigned __int128)a * a;
            volatile double v = (double)num / dnn;
            noise_host[p] = (float)std::sqrt((double)v);
        }
    }
    return PDC_OK;
}

pdc_status pdc_calibrate_darks(pdc_ctx *ctx, const pdc_geometry *geom, const uint16_t *darks_dev, uint64_t n_frames,
                               const float *gain, const pdc_params *params, float *noise_host, int32_t *det_out)
{
    if (!ctx || !det_out) return fail(ctx, PDC_EINVAL, "ctx and det_out must be non-NULL");
    pdc_status rc = check_geometry(geom);
    if (rc != PDC_OK) return fail(ctx, rc, "%s", g_thread_error);
    rc = check_params(params, nullptr, nullptr);
    if (rc != PDC_OK) return fail(ctx, rc, "%s", g_thread_error);
    if (geom->gain_mode != 0)
        return fail(ctx, PDC_EINVAL, "calibration from darks takes single-range detectors (gain_mode 0)");
    const size_t px = (size_t)geom->n_tiles * geom->rows * geom->cols;
    std::vector<float> ped(px);
    rc = pdc_dark_stats(ctx, geom, darks_dev, n_frames, ped.data(), noise_host, nullptr);
    if (rc != PDC_OK) return rc;
    return pdc_calibrate(ctx, geom, ped.data(), gain, params, det_out);
}

pdc_status pdc_get_invalid_counts(pdc_ctx *ctx, uint64_t batch, uint32_t *per_frame_invalid)
{
    if (!ctx) return fail(nullptr, PDC_EINVAL, "ctx is NULL");
    Batch *bt = find_batch(ctx, batch);
    if (!bt) return fail(ctx, PDC_ESTATE, "unknown batch %llu", (unsigned long long)batch);
    if (!per_frame_invalid && bt->n_frames) return fail(ctx, PDC_EINVAL, "per_frame_invalid is NULL");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    pdc_status rc = finish_batch(ctx, *bt);
    if (rc != PDC_OK) return rc;
    if (bt->n_frames == 0) return PDC_OK;
    if (ctx->dets[bt->det].g.gain_mode == 0) {
        std::memset(per_frame_invalid, 0, bt->n_frames * sizeof(uint32_t));
        return PDC_OK;
    }
    hipStream_t cs = ctx->copy_stream;
    HIP_TRY(ctx, hipStreamWaitEvent(cs, bt->buf->ev_end, 0));
    HIP_TRY(ctx, hipMemcpyAsync(per_frame_invalid, bt->buf->invalid, bt->n_frames * sizeof(uint32_t),
                                hipMemcpyDeviceToHost, cs));
    HIP_TRY(ctx, hipStreamSynchronize(cs));
    return PDC_OK;
}

// Test hook: the kernel a batch ran on (1 general, 2 persistent), after any
// recomputation.  Waits for the batch.
pdc_status pdc_debug_batch_path(pdc_ctx *ctx, uint64_t batch, int32_t *path)
{
    if (!ctx || !path) return fail(ctx, PDC_EINVAL, "ctx and path must be non-NULL");
    Batch *bt = find_batch(ctx, batch);
    if (!bt) return fail(ctx, PDC_ESTATE, "unknown batch %llu", (unsigned long long)batch);
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    pdc_status rc = finish_batch(ctx, *bt);
    if (rc != PDC_OK) return rc;
    *path = bt->path == 2 && bt->fb == 1 ? 3 : bt->path;
    if (bt->path == 2 && bt->mix_one) *path += 2;
    return PDC_OK;
}

// Time the persistent kernel on the caller's frames with frame groups x 1, 2
// and 4 (each a whole number of rounds of the chip) and keep the fastest.
pdc_status pdc_autotune(pdc_ctx *ctx, int32_t det, const uint16_t *frames_dev, uint64_t n_frames,
                        uint64_t hit_capacity, void *hip_stream, int32_t *mult_out, float *ms_out)
{
    if (!ctx) return fail(nullptr, PDC_EINVAL, "ctx is NULL");
    if (det < 0 || det >= (int32_t)ctx->dets.size() || !ctx->dets[det].live || ctx->dets[det].release_requested)
        return fail(ctx, PDC_ESTATE, "unknown detector %d", det);
    if (n_frames < 1 || !frames_dev) return fail(ctx, PDC_EINVAL, "need frames_dev and n_frames >= 1");
    static const int kMults[3] = {1, 2, 4};
    float best_ms = 0.0f;
    int best = 1;
    for (int j = 0; j < 3; ++j) {
        ctx->dets[det].fg_mult = kMults[j];
        float ms = 0.0f;
        for (int rep = 0; rep < 3; ++rep) {  // one warm-up, then the faster of two
            uint64_t b = 0;
            pdc_status rc = pdc_process_frames(ctx, det, frames_dev, n_frames, hit_capacity, hip_stream, &b);
            if (rc != PDC_OK) {
                ctx->dets[det].fg_mult = 1;
                return rc;
            }
            float main_ms = 0.0f;
            rc = pdc_get_hits(ctx, b, nullptr, 0, 0, nullptr, nullptr, nullptr);
            if (rc >= 0) rc = pdc_batch_timing(ctx, b, &main_ms, nullptr);
            pdc_release_batch(ctx, b);
            if (rc < 0) {
                ctx->dets[det].fg_mult = 1;
                return rc;
            }
            if (rep == 1 || (rep == 2 && main_ms < ms)) ms = main_ms;
        }
        if (ms_out) ms_out[j] = ms;
        if (j == 0 || ms < best_ms) {
            best_ms = ms;
            best = kMults[j];
        }
    }
    ctx->dets[det].fg_mult = best;
    if (mult_out) *mult_out = best;
    return PDC_OK;
}

pdc_status pdc_autotune_strips(pdc_ctx *ctx, int32_t det, const uint16_t *frames_dev, uint64_t n_frames,
                               uint64_t hit_capacity, void *hip_stream, int32_t *rows_out, int32_t *mult_out,
                               float *ms_out, int32_t *n_tried)
{
    if (!ctx) return fail(nullptr, PDC_EINVAL, "ctx is NULL");
    if (det < 0 || det >= (int32_t)ctx->dets.size() || !ctx->dets[det].live || ctx->dets[det].release_requested)
        return fail(ctx, PDC_ESTATE, "unknown detector %d", det);
    if (n_frames < 1 || !frames_dev) return fail(ctx, PDC_EINVAL, "need frames_dev and n_frames >= 1");
    Detector &d = ctx->dets[det];
    if (!d.v2_ok) return fail(ctx, PDC_ESTATE, "the detector does not take the persistent kernel");
    if (d.pending) return fail(ctx, PDC_ESTATE, "the detector has outstanding batches or graphs");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    // own rows per strip: the most the lane layout holds, then 4 and 8 fewer
    d.strip_cap = 0;
    if (!plan_v2(ctx, d)) return fail(ctx, PDC_EDEVICE, "re-plan failed");
    const int full = kV2Waves * d.gmax / (d.g.cols / d.g.bank_cols) - 2;  // as plan_v2 allows
    int caps[3] = {full, full - 4, full - 8};
    int n_caps = 1;
    while (n_caps < 3 && caps[n_caps] >= 4) ++n_caps;
    float best_ms = 0.0f;
    int best_cap = full, best_mult = 1, tried = 0;
    for (int c = 0; c < n_caps; ++c) {
        d.strip_cap = caps[c];
        if (!plan_v2(ctx, d)) {
            d.strip_cap = 0;
            plan_v2(ctx, d);
            return fail(ctx, PDC_EDEVICE, "re-plan failed");
        }
        int mult = 1;
        float ms3[3] = {0.0f, 0.0f, 0.0f};
        const pdc_status rc = pdc_autotune(ctx, det, frames_dev, n_frames, hit_capacity, hip_stream, &mult, ms3);
        if (rc != PDC_OK) {
            d.strip_cap = 0;
            plan_v2(ctx, d);
            return rc;
        }
        const float ms = std::min(ms3[0], std::min(ms3[1], ms3[2]));
        for (int j = 0; j < 3; ++j)
            if (ms_out) ms_out[3 * c + j] = ms3[j];
        ++tried;
        if (c == 0 || ms < best_ms) {
            best_ms = ms;
            best_cap = caps[c];
            best_mult = mult;
        }
    }
    d.strip_cap = best_cap == full ? 0 : best_cap;
    if (!plan_v2(ctx, d)) return fail(ctx, PDC_EDEVICE, "re-plan failed");
    d.fg_mult = best_mult;
    if (rows_out) *rows_out = best_cap;
    if (mult_out) *mult_out = best_mult;
    if (n_tried) *n_tried = tried;
    return PDC_OK;
}

}  // extern "C"
