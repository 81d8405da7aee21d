// Serving loop: several detectors' frame streams arriving at their own times,
// processed with continuous batching on one GPU (one HIP stream per detector,
// so batches of different detectors overlap on the device), with admission
// control by a device-memory budget (each batch charged what the library
// reports for it), an optional subpixel stage on every hit, and per-frame
// latency records.  Built on the public C ABI of pdc.h only.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <deque>
#include <new>
#include <vector>

#include "pdc.h"

namespace {

using Clock = std::chrono::steady_clock;

uint64_t ns_since(Clock::time_point t0)
{
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(Clock::now() - t0).count();
}

struct InFlight {
    uint64_t batch = 0;
    uint64_t first = 0, n = 0;   // stream frame indices [first, first + n)
    uint64_t bytes = 0;          // admission charge
    hipEvent_t done = nullptr;
};

// Device bytes a hit's subpixel input takes: network inputs, or none for the
// centroid (computed from the batch directly).
uint64_t subpixel_bytes(int32_t subpixel)
{
    return subpixel == PDC_SERVE_SUBPIXEL_CENTROID ? 0 : PDC_MLP_INPUT_WORDS * sizeof(uint16_t);
}

struct StreamState {
    pdc_serve_stream *d = nullptr;
    hipStream_t hs = nullptr;
    hipStream_t ss = nullptr;    // subpixel work of completed batches
    void *patches = nullptr;     // device [cap][25] float32 patches, or [cap][32] bf16 network inputs
    float *pos = nullptr;        // device [cap][2]
    uint64_t cap = 0;
    uint64_t next_arrival = 0;   // next frame index not yet arrived
    std::deque<uint64_t> pending;  // arrived, not launched
    std::deque<InFlight> inflight;
    uint64_t pixels = 0;         // per frame
    uint64_t hits_written = 0;   // into d->hits
    std::vector<uint32_t> fh;
    std::vector<uint64_t> fp;
};

// Frames of the next launch: the run of consecutive stream frames at the
// front of the queue (a dropped arrival leaves a gap that ends it), at most
// max_batch of them and contiguous in the device pool (frame i is pool frame
// i mod pool_frames, so the run stops where the pool wraps).
template <typename Seq>
uint64_t next_batch_len(const Seq &pending, uint64_t n_pending, uint64_t max_batch, uint64_t pool_frames)
{
    if (n_pending == 0 || max_batch == 0 || pool_frames == 0) return 0;
    const uint64_t first = pending[0];
    const uint64_t lim = std::min<uint64_t>(std::min<uint64_t>(n_pending, max_batch), pool_frames - first % pool_frames);
    uint64_t n = 1;
    while (n < lim && pending[n] == first + n) ++n;
    return n;
}

}  // namespace

extern "C" {

pdc_status pdc_debug_serve_batch_len(const uint64_t *pending, uint64_t n_pending, uint64_t max_batch,
                                     uint64_t pool_frames, uint64_t *n_out)
{
    if (!n_out || (n_pending && !pending)) return PDC_EINVAL;
    for (uint64_t i = 1; i < n_pending; ++i)
        if (pending[i] <= pending[i - 1]) return PDC_EINVAL;
    *n_out = next_batch_len(pending, n_pending, max_batch, pool_frames);
    return PDC_OK;
}

pdc_status pdc_serve_run(pdc_ctx *ctx, pdc_serve_stream *streams, int32_t n_streams,
                         const pdc_serve_config *cfg, pdc_serve_summary *summary)
{
    if (!ctx || !streams || !cfg || n_streams < 1 || n_streams > 64) return PDC_EINVAL;
    if (cfg->max_batch < 1 || cfg->max_inflight < 1 || cfg->max_inflight > 64) return PDC_EINVAL;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return PDC_EDEVICE;
    std::vector<StreamState> S(n_streams);
    uint64_t total_frames = 0;
    for (int s = 0; s < n_streams; ++s) {
        pdc_serve_stream &d = streams[s];
        if (d.n_frames > 0 && (!d.pool_dev || d.pool_frames == 0 || !d.arrival_ns || !d.results)) return PDC_EINVAL;
        if (d.pixels_per_frame == 0) return PDC_EINVAL;
        if (d.subpixel < PDC_SERVE_SUBPIXEL_NONE || d.subpixel > PDC_SERVE_SUBPIXEL_MLP_FALLBACK) return PDC_EINVAL;
        if ((d.subpixel == PDC_SERVE_SUBPIXEL_MLP || d.subpixel == PDC_SERVE_SUBPIXEL_MLP_FALLBACK) && !cfg->net)
            return PDC_EINVAL;
        for (uint64_t i = 1; i < d.n_frames; ++i)
            if (d.arrival_ns[i] < d.arrival_ns[i - 1]) return PDC_EINVAL;
        S[s].d = &d;
        S[s].pixels = d.pixels_per_frame;
        S[s].fh.resize(cfg->max_batch);
        S[s].fp.resize(cfg->max_batch);
        total_frames += d.n_frames;
        for (uint64_t i = 0; i < d.n_frames; ++i) {
            pdc_serve_frame &r = d.results[i];
            std::memset(&r, 0, sizeof r);
            r.arrival_ns = d.arrival_ns[i];
        }
    }
    pdc_status rc = PDC_OK;
    for (int s = 0; s < n_streams && rc == PDC_OK; ++s) {
        if (hipStreamCreateWithFlags(&S[s].hs, hipStreamNonBlocking) != hipSuccess) rc = PDC_EDEVICE;
        if (rc == PDC_OK && streams[s].subpixel &&
            hipStreamCreateWithFlags(&S[s].ss, hipStreamNonBlocking) != hipSuccess)
            rc = PDC_EDEVICE;
    }

    uint64_t done_frames = 0, dropped = 0, launched_batches = 0, held_bytes = 0, peak_bytes = 0;
    const Clock::time_point t0 = Clock::now();
    auto finish = [&](StreamState &st, InFlight &b) -> pdc_status {
        uint64_t total = 0;
        pdc_hit *dst = nullptr;
        uint64_t cap = 0;
        if (st.d->hits && st.hits_written < st.d->hits_capacity) {
            dst = st.d->hits + st.hits_written;
            cap = st.d->hits_capacity - st.hits_written;
        }
        pdc_status r = pdc_get_hits(ctx, b.batch, dst, cap, 0, &total, st.fh.data(), st.fp.data());
        if (r < 0) return r;
        const uint64_t tdone = ns_since(t0);
        const uint64_t kept = std::min(total, cap);
        for (uint64_t j = 0; j < kept; ++j) dst[j].frame += (uint32_t)b.first;  // stream frame index
        if (st.d->subpixel && total > 0) {
            // positions of all the batch's hits; those of the kept hits are copied out.
            // The learned stage takes the network's inputs (64 bytes a hit); the
            // centroid is computed from the batch directly, and with the fallback
            // it replaces the network's implausible positions.
            const int32_t mode = st.d->subpixel;
            if (total > st.cap) {
                hipFree(st.patches);
                hipFree(st.pos);
                st.patches = nullptr;
                st.pos = nullptr;
                st.cap = 0;
                const uint64_t in_bytes = total * subpixel_bytes(mode);
                if ((in_bytes && hipMalloc(&st.patches, in_bytes) != hipSuccess) ||
                    hipMalloc((void **)&st.pos, total * 2 * sizeof(float)) != hipSuccess)
                    return PDC_ENOMEM;
                st.cap = total;
            }
            uint64_t np = 0;
            if (mode == PDC_SERVE_SUBPIXEL_CENTROID) {
                r = pdc_capture_centroids(ctx, b.batch, st.d->t_nb, cfg->eta_dev, cfg->eta_bins, st.pos, total, 0, &np);
                if (r < 0) return r;
            } else {
                r = pdc_capture_inputs(ctx, b.batch, st.d->photon_adu, static_cast<uint16_t *>(st.patches), total, &np);
                if (r < 0) return r;
                r = pdc_mlp_infer_inputs(cfg->net, static_cast<const uint16_t *>(st.patches), np, st.pos, st.ss);
                if (r < 0) return r;
                if (mode == PDC_SERVE_SUBPIXEL_MLP_FALLBACK) {
                    if (hipStreamSynchronize(st.ss) != hipSuccess) return PDC_EDEVICE;
                    r = pdc_capture_centroids(ctx, b.batch, st.d->t_nb, cfg->eta_dev, cfg->eta_bins, st.pos, np, 1,
                                              nullptr);
                    if (r < 0) return r;
                }
            }
            if (st.d->positions && kept > 0 &&
                hipMemcpyAsync(st.d->positions + 2 * st.hits_written, st.pos, kept * 2 * sizeof(float),
                               hipMemcpyDeviceToHost, st.ss) != hipSuccess)
                return PDC_EDEVICE;
            if (hipStreamSynchronize(st.ss) != hipSuccess) return PDC_EDEVICE;
        }
        st.hits_written += kept;
        for (uint64_t j = 0; j < b.n; ++j) {
            pdc_serve_frame &fr = st.d->results[b.first + j];
            fr.done_ns = tdone;
            fr.hits = st.fh[j];
            fr.photons = st.fp[j];
            fr.batch_frames = (uint32_t)b.n;
            fr.status = PDC_SERVE_DONE;
        }
        r = pdc_release_batch(ctx, b.batch);
        if (r < 0) return r;
        hipEventDestroy(b.done);
        held_bytes -= b.bytes;
        done_frames += b.n;
        return PDC_OK;
    };

    while (rc == PDC_OK && done_frames + dropped < total_frames) {
        const uint64_t now = ns_since(t0);
        bool progressed = false;
        for (int s = 0; s < n_streams && rc == PDC_OK; ++s) {
            StreamState &st = S[s];
            pdc_serve_stream &d = *st.d;
            // arrivals up to now; beyond the queue limit a frame is dropped
            while (st.next_arrival < d.n_frames && d.arrival_ns[st.next_arrival] <= now) {
                const uint64_t i = st.next_arrival++;
                if (cfg->max_queue && st.pending.size() >= cfg->max_queue) {
                    d.results[i].status = PDC_SERVE_DROPPED;
                    ++dropped;
                } else {
                    st.pending.push_back(i);
                }
                progressed = true;
            }
            // completions, in launch order
            while (!st.inflight.empty() && hipEventQuery(st.inflight.front().done) == hipSuccess) {
                rc = finish(st, st.inflight.front());
                st.inflight.pop_front();
                progressed = true;
                if (rc != PDC_OK) break;
            }
            // continuous batching: launch what has arrived while the stream has a
            // free slot and the device-memory budget admits the batch
            while (rc == PDC_OK && !st.pending.empty() && st.inflight.size() < (size_t)cfg->max_inflight) {
                const uint64_t first = st.pending.front();
                const uint64_t pool_i = first % d.pool_frames;
                const uint64_t n = next_batch_len(st.pending, st.pending.size(), cfg->max_batch, d.pool_frames);
                const uint64_t hit_cap = std::max<uint64_t>(1024, (uint64_t)(d.hit_fraction * (double)(st.pixels * n)));
                uint64_t bytes = 0;
                rc = pdc_batch_bytes(ctx, d.det, n, hit_cap, &bytes);
                if (rc != PDC_OK) break;
                if (d.subpixel) bytes += hit_cap * (subpixel_bytes(d.subpixel) + 2 * sizeof(float));  // and positions
                if (cfg->hbm_budget && held_bytes + bytes > cfg->hbm_budget && !st.inflight.empty()) break;
                InFlight b;
                b.first = first;
                b.n = n;
                b.bytes = bytes;
                const uint16_t *fr = d.pool_dev + pool_i * st.pixels;
                const uint64_t tl = ns_since(t0);
                pdc_status r = pdc_process_frames(ctx, d.det, fr, n, hit_cap, st.hs, &b.batch);
                if (r < 0) {
                    rc = r;
                    break;
                }
                if (hipEventCreateWithFlags(&b.done, hipEventDisableTiming) != hipSuccess ||
                    hipEventRecord(b.done, st.hs) != hipSuccess) {
                    rc = PDC_EDEVICE;
                    break;
                }
                for (uint64_t j = 0; j < n; ++j) d.results[first + j].launch_ns = tl;
                st.pending.erase(st.pending.begin(), st.pending.begin() + (ptrdiff_t)n);
                st.inflight.push_back(b);
                held_bytes += bytes;
                peak_bytes = std::max(peak_bytes, held_bytes);
                ++launched_batches;
                progressed = true;
            }
        }
        (void)progressed;  // a busy loop: arrivals and completions are polled
    }
    // drain on error
    for (int s = 0; s < n_streams; ++s) {
        for (InFlight &b : S[s].inflight) {
            pdc_release_batch(ctx, b.batch);
            if (b.done) hipEventDestroy(b.done);
        }
        if (S[s].hs) {
            hipStreamSynchronize(S[s].hs);
            hipStreamDestroy(S[s].hs);
        }
        if (S[s].ss) {
            hipStreamSynchronize(S[s].ss);
            hipStreamDestroy(S[s].ss);
        }
        hipFree(S[s].patches);
        hipFree(S[s].pos);
    }
    for (int s = 0; s < n_streams; ++s) streams[s].hits_kept = S[s].hits_written;
    if (summary) {
        summary->frames_done = done_frames;
        summary->frames_dropped = dropped;
        summary->batches = launched_batches;
        summary->peak_bytes = peak_bytes;
        summary->wall_ns = ns_since(t0);
    }
    return rc;
}

}  // extern "C"
