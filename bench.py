"""Throughput benchmark of the detector-correction and photon-finding path.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

One step = one pdc_process_frames call over a device-resident batch of
10,000 CSPAD-like frames (32 tiles of 185 x 388 uint16, 194-pixel common-mode
banks, 0.01 photons/pixel): 14-bit decode, dark, gain, bank median, common-mode
subtraction, seeds, 3x3 local maximum, masked charge sum, photon count and the
compacted raster-order hit list with per-frame counts and photon totals, all in
HBM.  pdc_release_batch waits for it.  The batch is 64 distinct synthetic
frames replicated on the device (45.9 GB, far larger than the on-chip caches).

Printed: ONE JSON line with the throughput (Mpixel/s), the roofline of the
dominant kernel (algorithmic HBM bytes / its event-timed duration against the
8 TB/s peak), the CPU oracle's rate on the 64-frame pool (which also checks the
GPU hits of that pool), single-frame latency percentiles, a four-detector
serving run (Poisson arrivals at 1 and 20 kHz per detector, p50/p99 latency),
a mixed batch of three detectors (ePix100, ePix10k-like and
Jungfrau-like with gain ranges, 4,000 frames each) enqueued together, the
thresholded-mean common mode of Fig. c (bank and tile regions, three
stacked stages) on the same batch, summaries (count map and charge spectrum of the batch's hits, the Frames2
histogram and per-cloud-size spectra of a kept 2,000-frame batch, pedestal
and noise from 1,000 dark frames), the learned subpixel estimator against
centroid + eta on 10 M simulated hits, and an occupancy sweep.

Other modes:
  --profile            short run for rocprofv3 (1 warm-up + --steps batches,
                       then a plain 2 GiB device copy used to scale counters)
  --ingest-pmc F W     turn two rocprofv3 --pmc counter CSVs (FETCH_SIZE, then
                       WRITE_SIZE) of a --profile run into
                       profiles/frame_kernel_cspad_traffic.json
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import csv
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Mpixel/s processed (% of HBM roofline), bit-exact hits; p99 frame latency"
HBM_PEAK_GBPS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "frame_kernel_cspad_traffic.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1903_06838_amd", "csrc", f)
                  for f in ("pdc_frame_v2.hip", "pdc_kernels.hip", "pdc_runtime.cpp", "pdc_internal.h",
                            "pdc_device.h", "pdc_exact.h")]
MAIN_KERNEL_PREFIX = "frame_kernel"
COPY_BYTES = 2 << 30


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


# ---------------------------------------------------------------------------
def make_batch(torch, synth, geom, ped, gain, occ_id, pool_frames, n_frames, dev):
    occ = synth.CSPAD_OCCUPANCIES[occ_id]
    t0 = time.time()
    pool = synth.make_frames(geom, ped, gain, pool_frames, occ, 1, occ_id)
    dpool = torch.from_numpy(pool).to(dev)
    frames = torch.empty((n_frames, *geom.shape), dtype=torch.int16, device=dev)
    for i in range(0, n_frames, pool_frames):
        n = min(pool_frames, n_frames - i)
        frames[i:i + n].copy_(dpool[:n])
    del dpool
    torch.cuda.synchronize()
    log("batch occ=%g: %d frames (%d distinct) ready in %.1f s" % (occ, n_frames, pool_frames, time.time() - t0))
    return pool, frames


def run_steps(torch, pdc, ctx, det, frames, n_frames, hit_cap, steps, warmup):
    """Returns (ms_per_step, main_ms list, total_ms list, hits per batch, per-frame hits)."""
    stream = torch.cuda.current_stream()
    b = pdc.process_frames(ctx, det, frames, n_frames, hit_cap, stream)
    _, total, fh, fp, _ = pdc.get_hits(ctx, b, n_frames, capacity=0)
    pdc.release_batch(ctx, b)
    hit_cap = int(total * 1.02) + 1024
    for _ in range(warmup):
        b = pdc.process_frames(ctx, det, frames, n_frames, hit_cap, stream)
        pdc.get_hits(ctx, b, n_frames, capacity=0)
        pdc.release_batch(ctx, b)
    mains, totals, step_ms = [], [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ts = time.perf_counter()
        b = pdc.process_frames(ctx, det, frames, n_frames, hit_cap, stream)
        # the step ends with the batch's final per-frame results: this also
        # runs any recomputation the batch needs (seed lists or staging full)
        pdc.get_hits(ctx, b, n_frames, capacity=0)
        m, t = pdc.batch_timing(ctx, b)
        mains.append(m)
        totals.append(t)
        pdc.release_batch(ctx, b)
        step_ms.append((time.perf_counter() - ts) * 1e3)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    run_steps.step_ms = step_ms
    return (t1 - t0) * 1e3 / steps, mains, totals, total, (fh, fp), hit_cap


def roofline(n_frames, npix, hits, main_ms):
    # algorithmic bytes of one launch: 2 B per raw pixel, 8 B per hit
    # (pixel index + charge), and the two float32 calibration planes once.
    alg = 2.0 * n_frames * npix + 8.0 * hits + 8.0 * npix
    avg_s = sum(main_ms) / len(main_ms) / 1e3
    achieved = alg / avg_s / 1e9
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as f:
            tr = json.load(f)
        if tr.get("kernel_hash") == kernel_hash() and tr.get("n_frames") == n_frames:
            traffic = tr.get("bytes_per_launch")
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": traffic,
            "kernel": "frame_kernel", "algorithmic_bytes_per_launch": alg,
            "avg_launch_ms": round(avg_s * 1e3, 4)}


def cpu_baseline(pool, ped, gain, bank_cols, gpu_fh, gpu_fp, gpu_hits_fn):
    """The oracle (test infrastructure) on the 64-frame pool with frame-parallel
    threads; also checks the GPU's per-frame counts and hit list for the pool."""
    import numpy as np

    from oracle import oracle

    o = oracle.load()
    P = pool.shape[0]
    threads = min(16, os.cpu_count() or 1, P)
    bounds = np.linspace(0, P, threads + 1).astype(int)
    parts = [(bounds[i], bounds[i + 1]) for i in range(threads) if bounds[i + 1] > bounds[i]]
    # repeated passes over the pool until at least min_s seconds of wall time
    # (the first pass's results are the ones compared with the GPU)
    min_s = 12.0
    passes = 0
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(len(parts)) as ex:
        while True:
            res = list(ex.map(lambda ab: o.process(pool[ab[0]:ab[1]], ped, gain, bank_cols), parts))
            if passes == 0:
                outs = res
            passes += 1
            wall = time.perf_counter() - t0
            if wall >= min_s:
                break
    fh = np.concatenate([r["frame_hits"] for r in outs])
    fp = np.concatenate([r["frame_photons"] for r in outs])
    hits = []
    for (a, _), r in zip(parts, outs):
        h = r["hits"].copy()
        h["frame"] += np.uint32(a)
        hits.append(h)
    hits = np.concatenate(hits)
    idx = np.arange(len(gpu_fh)) % P
    exact = bool(np.array_equal(gpu_fh, fh[idx]) and np.array_equal(gpu_fp, fp[idx]))
    g = gpu_hits_fn(int(fh.sum()))
    exact = exact and g is not None and np.array_equal(
        np.ascontiguousarray(g).view(np.uint32), np.ascontiguousarray(hits).view(np.uint32))
    rate = passes * pool.size / wall / 1e6
    return {"value": round(rate, 2), "unit": "Mpixel/s", "cores": len(parts), "kind": "oracle",
            "sample": "%d passes over %d CSPAD-like frames (32x185x388, occupancy 0.01), the distinct "
                      "frames the 10,000-frame GPU batch replicates: %d frames in %.1f s wall"
                      % (passes, P, passes * P, wall)}, exact


def stats_ms(xs):
    import numpy as np

    return {"mean": round(float(np.mean(xs)), 4), "median": round(float(np.median(xs)), 4),
            "min": round(float(np.min(xs)), 4), "max": round(float(np.max(xs)), 4), "n": len(xs)}


def pool_check(pool, ped, gain, bank_cols, gpu_fh, gpu_fp, gpu_hits_fn):
    """The oracle on the distinct frames of a replicated batch: True when the
    GPU's counts and photon totals of every batch frame, and its hit list of
    the pool, equal the oracle's bit for bit."""
    import numpy as np

    from oracle import oracle

    o = oracle.load()
    P = pool.shape[0]
    threads = min(16, os.cpu_count() or 1, P)
    bounds = np.linspace(0, P, threads + 1).astype(int)
    parts = [(bounds[i], bounds[i + 1]) for i in range(threads) if bounds[i + 1] > bounds[i]]
    with cf.ThreadPoolExecutor(len(parts)) as ex:
        outs = list(ex.map(lambda ab: o.process(pool[ab[0]:ab[1]], ped, gain, bank_cols), parts))
    fh = np.concatenate([r["frame_hits"] for r in outs])
    fp = np.concatenate([r["frame_photons"] for r in outs])
    hits = []
    for (a, _), r in zip(parts, outs):
        h = r["hits"].copy()
        h["frame"] += np.uint32(a)
        hits.append(h)
    hits = np.concatenate(hits)
    idx = np.arange(len(gpu_fh)) % P
    exact = bool(np.array_equal(gpu_fh, fh[idx]) and np.array_equal(gpu_fp, fp[idx]))
    g = gpu_hits_fn(int(fh.sum()))
    return exact and g is not None and np.array_equal(
        np.ascontiguousarray(g).view(np.uint32), np.ascontiguousarray(hits).view(np.uint32))


def latency(torch, pdc, ctx, det, frame, calls=10000, use_graph=False):
    """Small-batch process_frames (or a replay of its captured graph) + get_hits,
    host-observed and kernel-only."""
    import numpy as np

    n = frame.shape[0]
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    graph = pdc.graph_create(ctx, det, frame, n, 1 << 20) if use_graph else None
    host, kern = [], []
    for i in range(calls + 20):
        t0 = time.perf_counter()
        if graph is not None:
            b = pdc.graph_launch(ctx, graph, stream)
        else:
            b = pdc.process_frames(ctx, det, frame, n, 1 << 20, stream)
        pdc.get_hits(ctx, b, n)
        t1 = time.perf_counter()
        _, tk = pdc.batch_timing(ctx, b)
        pdc.release_batch(ctx, b)
        if i >= 20:
            host.append((t1 - t0) * 1e3)
            kern.append(tk)
    if graph is not None:
        pdc.graph_destroy(ctx, graph)
    q = lambda a, p: round(float(np.percentile(a, p)), 4)
    return {"frames": n, "graph": use_graph, "host_ms_p50": q(host, 50), "host_ms_p99": q(host, 99),
            "kernel_ms_p50": q(kern, 50), "kernel_ms_p99": q(kern, 99), "calls": calls}


def subpixel(torch, pdc, ctx, n_total=10_000_000, steps=4000, bs=2048, lr=2e-3, photon_adu=150.0, t_nb=9.0):
    """Learned subpixel positions against centroid + eta on simulated hits:
    10 M charge-sharing patches, 90/10 split; RMS error and hits/s, all
    through the C ABI on the torch stream."""
    import numpy as np

    from paper_1903_06838_amd import synth

    dev = torch.device("cuda:0")
    # a stream of our own: torch's default stream has handle 0, which the
    # library reads as "the context's stream", so events on it would time nothing
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    P, T = synth.make_patches(n_total, seed=31)
    n_tr = n_total * 9 // 10
    n_te = n_total - n_tr
    dP = torch.from_numpy(P).to(dev)
    dT = torch.from_numpy(T).to(dev)
    del P
    Pte, Tte = dP[n_tr:], T[n_tr:]
    ev = lambda: torch.cuda.Event(enable_timing=True)  # recorded on `stream` (current)
    # classical: eta table over the training split, centroid + eta on the test split
    nb = 1023
    table = torch.zeros((2, nb + 1), dtype=torch.float32, device=dev)
    ws = torch.zeros(2 * nb, dtype=torch.int32, device=dev)
    ce = torch.zeros((n_te, 2), dtype=torch.float32, device=dev)
    pdc.eta_table(ctx, dP, n_tr, t_nb, nb, ws, table, stream)
    pdc.centroid(ctx, Pte, n_te, t_nb, ce, eta_dev=table, nbins=nb, stream=stream)
    e0, e1 = ev(), ev()
    e0.record()
    for _ in range(5):
        pdc.centroid(ctx, Pte, n_te, t_nb, ce, eta_dev=table, nbins=nb, stream=stream)
    e1.record()
    torch.cuda.synchronize()
    ms_ce = e0.elapsed_time(e1) / 5
    # learned: He-uniform start, Adam on minibatches of the training split
    rng = np.random.default_rng(0)
    shapes = [(25, 64), (64,), (64, 64), (64,), (64, 2), (2,)]
    theta = np.concatenate([rng.uniform(-np.sqrt(6.0 / s[0]), np.sqrt(6.0 / s[0]), size=s).ravel()
                            if len(s) == 2 else np.zeros(s) for s in shapes]).astype(np.float32)
    net = pdc.mlp_create(ctx, theta)
    try:
        e0.record()
        for it in range(steps):
            o = (it * bs) % (n_tr - bs)
            pdc.mlp_train_step(net, dP[o:o + bs], dT[o:o + bs], bs, photon_adu, lr, stream)
        e1.record()
        torch.cuda.synchronize()
        ms_train = e0.elapsed_time(e1)
        loss = pdc.mlp_last_loss(net)
        y = torch.zeros((n_te, 2), dtype=torch.float32, device=dev)
        pdc.mlp_infer(net, Pte, n_te, photon_adu, y, stream)
        # throughput over all n_total patches (the held-out positions above
        # are the ones the RMS uses)
        y_all = torch.empty((n_total, 2), dtype=torch.float32, device=dev)
        pdc.mlp_infer(net, dP, n_total, photon_adu, y_all, stream)
        e0.record()
        for _ in range(5):
            pdc.mlp_infer(net, dP, n_total, photon_adu, y_all, stream)
        e1.record()
        torch.cuda.synchronize()
        ms_inf = e0.elapsed_time(e1) / 5
        # the same positions from the 64-byte network inputs
        x_all = torch.empty((n_total, pdc.MLP_INPUT_WORDS), dtype=torch.int16, device=dev)
        pdc.mlp_make_inputs(ctx, dP, n_total, photon_adu, x_all, stream)
        y_in = torch.empty((n_total, 2), dtype=torch.float32, device=dev)
        pdc.mlp_infer_inputs(net, x_all, n_total, y_in, stream)
        e0.record()
        for _ in range(5):
            pdc.mlp_infer_inputs(net, x_all, n_total, y_in, stream)
        e1.record()
        torch.cuda.synchronize()
        ms_inf16 = e0.elapsed_time(e1) / 5
        same_inputs = bool(torch.equal(y_in, y_all))
        del y_all, x_all, y_in
    finally:
        pdc.mlp_destroy(net)
    torch.cuda.set_stream(torch.cuda.default_stream())
    rms = lambda a: float(np.sqrt(np.mean((a.cpu().numpy() - Tte) ** 2)))
    inf_bytes = n_total * (25 * 4 + 2 * 4)
    inf_flop = n_total * 2 * (25 * 64 + 64 * 64 + 64 * 2)
    return {"hits": n_total, "train": n_tr, "test": n_te, "train_steps": steps, "batch": bs, "lr": lr,
            "rms_px_mlp": round(rms(y), 5), "rms_px_centroid_eta": round(rms(ce), 5),
            "final_train_loss": round(loss, 6),
            "mlp_infer_hits_per_s": round(n_total / (ms_inf / 1e3), 1),
            "mlp_infer_GBps": round(inf_bytes / (ms_inf / 1e3) / 1e9, 1),
            "mlp_infer_TFLOPs_bf16": round(inf_flop / (ms_inf / 1e3) / 1e12, 2),
            "mlp_infer_inputs_hits_per_s": round(n_total / (ms_inf16 / 1e3), 1),
            "mlp_infer_inputs_GBps": round(n_total * (2 * pdc.MLP_INPUT_WORDS + 2 * 4) / (ms_inf16 / 1e3) / 1e9, 1),
            "mlp_infer_inputs_same_positions": same_inputs,
            "centroid_eta_hits_per_s": round(n_te / (ms_ce / 1e3), 1),
            "train_hits_per_s": round(steps * bs / (ms_train / 1e3), 1),
            "data": "synthetic charge-sharing patches (uniform impact points, cloud sigma U(0.1, 0.4) px, "
                    "3 ADU noise, 150 ADU photons)"}


def he_uniform_mlp(seed):
    """Random-init weights of the 25-64-64-2 subpixel network (He-uniform,
    zero biases), packed in the library's theta layout."""
    import numpy as np

    rng = np.random.default_rng(seed)
    parts = []
    for fan_in, fan_out in ((25, 64), (64, 64), (64, 2)):
        lim = np.sqrt(6.0 / fan_in)
        parts += [rng.uniform(-lim, lim, size=(fan_in, fan_out)).ravel(), np.zeros(fan_out)]
    return np.concatenate(parts).astype(np.float32)


def serving(torch, pdc, ctx, rates=(1000.0, 5000.0, 10000.0, 20000.0), seconds=1.0, max_batch=64, max_inflight=2,
            hbm_budget=8 << 30):
    """Four detectors as Poisson frame streams: two ePix100 704x768, a CSPAD-like
    2.3 Mpixel one and a Jungfrau-like 512x1024 with three gain ranges, at
    occupancy 0.005, each frame resident in a 64-frame device pool, served with
    continuous batching, admission by an HBM budget charged with each batch's
    reported footprint, and the learned subpixel stage on every hit (random-init
    weights: its work does not depend on their values).  Latency = completion
    seen by the host, positions included, - arrival."""
    import numpy as np

    from paper_1903_06838_amd import synth

    dets = [("epix100_a", synth.EPIX100, 0), ("epix100_b", synth.EPIX100, 0), ("cspad", synth.CSPAD, 0),
            ("jungfrau_0.5M_multigain", synth.Geometry(1, 512, 1024, 256), 2)]
    pools, handles = [], []
    prm = pdc.params(3.0, 5.0, 3.0, 150.0, pdc.KEEP_MEDIANS)
    for j, (name, g, gm) in enumerate(dets):
        if gm:
            ped, gain = synth.make_calibration_multigain(g, 60 + j)
            # at occupancy 0.005 few pixels switch to the lower ranges: 1.1 % of
            # them (the multi-gain tests' setting for the mean modes)
            raw = synth.make_frames_multigain(g, ped, gain, 64, 0.005, 60 + j, gm, range_frac=(0.985, 0.008, 0.003),
                                              invalid_frac=0.01)
        else:
            ped, gain = synth.make_calibration(g, 60 + j)
            raw = synth.make_frames(g, ped, gain, 64, 0.005, 60 + j)
        pools.append(torch.from_numpy(raw).cuda())
        handles.append(pdc.calibrate(ctx, pdc.geometry(*g.shape, g.bank_cols, gain_mode=gm), ped, gain, prm))
    net = pdc.mlp_create(ctx, he_uniform_mlp(3))
    runs = []
    try:
        for rate_hz in rates:
            n = int(rate_hz * seconds)
            streams = []
            for j, ((name, g, gm), det, pool) in enumerate(zip(dets, handles, pools)):
                arr = np.cumsum(np.random.default_rng(90 + j).exponential(1e9 / rate_hz, size=n)).astype(np.uint64)
                streams.append(dict(det=det, pool=pool, arrival_ns=arr, hit_fraction=0.01,
                                    subpixel=pdc.SERVE_SUBPIXEL_MLP, photon_adu=150.0, t_nb=9.0))
            res, _, summ = pdc.serve_run(ctx, streams, max_batch=max_batch, max_inflight=max_inflight,
                                         hbm_budget=hbm_budget, net=net)
            out = {"rate_hz_per_detector": rate_hz, "seconds": seconds, "frames": summ["frames_done"],
                   "dropped": summ["frames_dropped"], "batches": summ["batches"],
                   "peak_batch_bytes": summ["peak_bytes"], "wall_s": round(summ["wall_ns"] / 1e9, 4),
                   "detectors": {}}
            px, hits = 0, 0
            lat_all = []
            for (name, g, gm), r in zip(dets, res):
                ok = r["status"] == 1
                lat = (r["done_ns"][ok] - r["arrival_ns"][ok]) / 1e6
                lat_all.append(lat)
                px += int(ok.sum()) * g.pixels
                hits += int(r["hits"][ok].sum())
                out["detectors"][name] = {"pixels": g.pixels, "frames": int(ok.sum()),
                                          "latency_ms_p50": round(float(np.percentile(lat, 50)), 4),
                                          "latency_ms_p99": round(float(np.percentile(lat, 99)), 4),
                                          "mean_batch": round(float(r["batch_frames"][ok].mean()), 2)}
            la = np.concatenate(lat_all)
            out["latency_ms_p50"] = round(float(np.percentile(la, 50)), 4)
            out["latency_ms_p99"] = round(float(np.percentile(la, 99)), 4)
            out["Mpixel_s"] = round(px / (summ["wall_ns"] / 1e9) / 1e6, 1)
            out["offered_Mpixel_s"] = round(sum(g.pixels for _, g, _ in dets) * rate_hz / 1e6, 1)
            out["hits_with_positions_per_s"] = round(hits / (summ["wall_ns"] / 1e9), 1)
            runs.append(out)
            log("serving at %.0f Hz per detector: %s Mpixel/s, p50 %s ms, p99 %s ms, dropped %d"
                % (rate_hz, out["Mpixel_s"], out["latency_ms_p50"], out["latency_ms_p99"], out["dropped"]))
    finally:
        pdc.mlp_destroy(net)
        for det in handles:
            pdc.release_detector(ctx, det)
    return runs


def mixed(torch, pdc, ctx, frames_each=4000, steps=3):
    """Mixed-geometry batch: ePix100 704x768 (single gain, 96-pixel banks),
    ePix10k-like 352x384 (three gain ranges, 96-pixel banks) and
    Jungfrau-like 512x1024 (three gain ranges, 256-pixel banks), 4,000 frames
    each at occupancies spread over 0.001..0.02, enqueued together with
    pdc_process_mixed (one launch of the persistent kernel over all three,
    frame groups sized for the whole chip per detector and again for each
    detector's share of it; and a launch per detector on forked streams),
    captured once into one graph and replayed, and the three processed one
    after another."""
    import numpy as np

    from paper_1903_06838_amd import synth

    dev = torch.device("cuda:0")
    spec = [("epix100", synth.EPIX100, 0), ("epix10k", synth.Geometry(1, 352, 384, 96), 1),
            ("jungfrau_0.5M", synth.Geometry(1, 512, 1024, 256), 2)]
    occs = (0.001, 0.007, 0.013, 0.02)
    frames, calib, px = [], [], 0
    for j, (name, g, gm) in enumerate(spec):
        parts = []
        if gm:
            ped, gain = synth.make_calibration_multigain(g, 70 + j)
        else:
            ped, gain = synth.make_calibration(g, 70 + j)
        for i, occ in enumerate(occs):
            if gm:
                parts.append(synth.make_frames_multigain(g, ped, gain, 4, occ, 70 + 10 * i + j, gm,
                                                         range_frac=(0.95, 0.03, 0.01), invalid_frac=0.01))
            else:
                parts.append(synth.make_frames(g, ped, gain, 4, occ, 70 + j, i))
        pool = torch.from_numpy(np.concatenate(parts)).to(dev)
        fr = torch.empty((frames_each, *g.shape), dtype=torch.int16, device=dev)
        for i in range(0, frames_each, pool.shape[0]):
            n = min(pool.shape[0], frames_each - i)
            fr[i:i + n].copy_(pool[:n])
        frames.append(fr)
        calib.append((ped, gain))
        px += frames_each * g.pixels
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()

    def setup(c):
        dets = [pdc.calibrate(c, pdc.geometry(*g.shape, g.bank_cols, gm), *calib[j], pdc.params())
                for j, (_, g, gm) in enumerate(spec)]
        items = [(d, f, frames_each, int(0.03 * frames_each * g.pixels) + 4096)
                 for d, f, (_, g, _) in zip(dets, frames, spec)]
        return dets, items

    def time_mixed(c, items):
        for k in range(steps + 1):  # one warm-up
            if k == 1:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
            for b, it in zip(pdc.process_mixed(c, items, stream), items):
                pdc.get_hits(c, b, it[2], capacity=0)
                pdc.release_batch(c, b)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / steps

    dets, items = setup(ctx)
    ms_mixed = time_mixed(ctx, items)
    # the same batches captured once into one graph and replayed
    graph = pdc.graph_create_mixed(ctx, items)
    for k in range(steps + 1):
        if k == 1:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
        for b, it in zip(pdc.graph_launch(ctx, graph, stream), items):
            pdc.get_hits(ctx, b, it[2], capacity=0)
            pdc.release_batch(ctx, b)
    torch.cuda.synchronize()
    ms_graph = (time.perf_counter() - t0) * 1e3 / steps
    pdc.graph_destroy(ctx, graph)
    alone = {}
    for i, (name, g, gm) in enumerate(spec):
        d, f, n, cap = items[i]
        for k in range(steps + 1):
            if k == 1:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
            b = pdc.process_frames(ctx, d, f, n, cap, stream)
            pdc.get_hits(ctx, b, n, capacity=0)
            pdc.release_batch(ctx, b)
        torch.cuda.synchronize()
        alone[name] = round((time.perf_counter() - t0) * 1e3 / steps, 3)
    for d in dets:
        pdc.release_detector(ctx, d)
    # the same with each launch sized to its share of the chip
    os.environ["PDC_MIX_SHARE"] = "1"
    try:
        c2 = pdc.create(0)
    finally:
        del os.environ["PDC_MIX_SHARE"]
    dets2, items2 = setup(c2)
    ms_share = time_mixed(c2, items2)
    for d in dets2:
        pdc.release_detector(c2, d)
    pdc.destroy(c2)
    # a launch per detector on forked streams
    os.environ["PDC_MIX_FORKED"] = "1"
    try:
        c3 = pdc.create(0)
    finally:
        del os.environ["PDC_MIX_FORKED"]
    dets3, items3 = setup(c3)
    ms_forked = time_mixed(c3, items3)
    for d in dets3:
        pdc.release_detector(c3, d)
    pdc.destroy(c3)
    del frames
    return {"frames_per_detector": frames_each, "pixels": px, "ms_mixed": round(ms_mixed, 3),
            "Mpixel_s_mixed": round(px / (ms_mixed / 1e3) / 1e6, 1),
            "ms_mixed_graph": round(ms_graph, 3), "ms_mixed_shared_chip": round(ms_share, 3),
            "ms_mixed_forked_launches": round(ms_forked, 3), "ms_alone": alone,
            "ms_alone_sum": round(sum(alone.values()), 3),
            "Mpixel_s_one_after_another": round(px / (sum(alone.values()) / 1e3) / 1e6, 1),
            "occupancies": list(occs), "gain_ranges": "95/3/1 % of pixels, 1 % invalid codes"}


def summaries(torch, pdc, ctx, geom, ped, gain, frames, n_frames, hit_cap, keep_frames=2000, dark_frames=1000):
    """Summaries over CSPAD-like batches: count map + charge spectrum of the
    headline batch's hits, Frames2 histogram and per-size spectra of a batch
    kept in HBM, and pedestal/noise from dark frames.  Event-timed on a stream
    of our own (torch's default stream reads as the context's stream)."""
    import numpy as np

    from paper_1903_06838_amd import synth

    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream()
    npix = geom.pixels
    nb = 1000
    out = {}
    ev = lambda: torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(stream):
        cmap = torch.zeros(npix, dtype=torch.int32, device=dev)
        spec = torch.zeros(nb + 2, dtype=torch.int32, device=dev)
        sizes = torch.zeros(9 * (nb + 2), dtype=torch.int32, device=dev)
        hist = torch.zeros(nb + 2, dtype=torch.int32, device=dev)
    det = pdc.calibrate(ctx, pdc.geometry(*geom.shape, geom.bank_cols), ped, gain, pdc.params())
    b = pdc.process_frames(ctx, det, frames, n_frames, hit_cap, stream)
    _, total, _, _, _ = pdc.get_hits(ctx, b, n_frames, capacity=0)
    pdc.accumulate_hits(ctx, b, cmap, spec, None, -50.0, 450.0, nb, stream)  # warm-up
    e0, e1 = ev(), ev()
    reps = 5
    e0.record(stream)
    for _ in range(reps):
        pdc.accumulate_hits(ctx, b, cmap, spec, None, -50.0, 450.0, nb, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    pdc.release_batch(ctx, b)
    pdc.release_detector(ctx, det)
    out["accumulate_hits"] = {"hits": total, "ms": round(ms, 4), "hits_per_s": round(total / (ms / 1e3), 1),
                              "GBps_hit_reads": round(8.0 * total / (ms / 1e3) / 1e9, 1),
                              "what": "count map (+= nphot per pixel) and 1000-bin charge spectrum"}
    # a kept batch: Frames2 histogram and spectra split by cloud size
    kdet = pdc.calibrate(ctx, pdc.geometry(*geom.shape, geom.bank_cols), ped, gain,
                         pdc.params(flags=pdc.KEEP_CORRECTED))
    b = pdc.process_frames(ctx, kdet, frames, keep_frames, hit_cap, stream)
    _, ktotal, _, _, _ = pdc.get_hits(ctx, b, keep_frames, capacity=0)
    pdc.histogram_corrected(ctx, b, hist, -50.0, 450.0, nb, stream)
    e0.record(stream)
    for _ in range(reps):
        pdc.histogram_corrected(ctx, b, hist, -50.0, 450.0, nb, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_h = e0.elapsed_time(e1) / reps
    e0.record(stream)
    for _ in range(reps):
        pdc.accumulate_hits(ctx, b, cmap, spec, sizes, -50.0, 450.0, nb, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_s = e0.elapsed_time(e1) / reps
    pdc.release_batch(ctx, b)
    pdc.release_detector(ctx, kdet)
    nval = keep_frames * npix
    out["histogram_frames2"] = {"values": nval, "ms": round(ms_h, 4),
                                "GBps": round(4.0 * nval / (ms_h / 1e3) / 1e9, 1),
                                "frac_of_hbm_peak": round(4.0 * nval / (ms_h / 1e3) / 1e9 / HBM_PEAK_GBPS, 4)}
    out["size_spectra"] = {"hits": ktotal, "ms": round(ms_s, 4), "hits_per_s": round(ktotal / (ms_s / 1e3), 1)}
    # darks: pedestal and noise
    dped, dgain = ped, gain
    pool = synth.make_frames(geom, dped, dgain, 16, 0.0, 1, 7)
    dpool = torch.from_numpy(pool).to(dev)
    darks = torch.empty((dark_frames, *geom.shape), dtype=torch.int16, device=dev)
    for i in range(0, dark_frames, 16):
        darks[i:i + 16].copy_(dpool[:min(16, dark_frames - i)])
    torch.cuda.synchronize()
    g = pdc.geometry(*geom.shape, geom.bank_cols)
    pdc.dark_stats(ctx, g, darks, dark_frames, stream)
    t0 = time.perf_counter()
    for _ in range(3):
        p_, n_ = pdc.dark_stats(ctx, g, darks, dark_frames, stream)
    ms_d = (time.perf_counter() - t0) * 1e3 / 3
    out["dark_stats"] = {"frames": dark_frames, "pixels": npix, "ms_wall": round(ms_d, 3),
                         "GBps_wall": round(2.0 * dark_frames * npix / (ms_d / 1e3) / 1e9, 1),
                         "noise_median_adu": round(float(np.median(n_)), 4),
                         "note": "synchronous call: device sums, 37 MB copy to the host, host finish"}
    del darks, dpool
    return out


# ---------------------------------------------------------------------------
def ingest_pmc(fetch_csv, write_csv):
    """Per-dispatch FETCH_SIZE / WRITE_SIZE (KiB) of the frame kernel, scaled by
    what the same counters read for the plain 2 GiB copy of a --profile run."""
    def rows(path, counter):
        out = []
        with open(path) as f:
            for r in csv.DictReader(f):
                name = r.get("Kernel_Name") or r.get("Kernel-Name") or ""
                if r.get("Counter_Name", counter) != counter:
                    continue
                out.append((name, float(r["Counter_Value"])))
        return out

    res = {}
    for key, path, counter in (("fetch", fetch_csv, "FETCH_SIZE"), ("write", write_csv, "WRITE_SIZE")):
        rs = rows(path, counter)
        main = [v for n, v in rs if MAIN_KERNEL_PREFIX in n and "pdc" in n]
        copy = [v for n, v in rs if "copy" in n.lower() or "elementwise" in n.lower()]
        copy = [v for v in copy if v > 0.5 * COPY_BYTES / 1024]
        if not main or not copy:
            raise SystemExit("no %s rows for the frame kernel or the copy kernel in %s" % (counter, path))
        kib_main = sorted(main)[len(main) // 2]
        kib_copy = sorted(copy)[len(copy) // 2]
        scale = COPY_BYTES / (kib_copy * 1024.0)
        res[key] = {"kib_per_dispatch": kib_main, "copy_kib": kib_copy, "scale": scale,
                    "bytes": kib_main * 1024.0 * scale}
    out = {"kernel_hash": kernel_hash(), "n_frames": 10000,
           "bytes_per_launch": res["fetch"]["bytes"] + res["write"]["bytes"],
           "fetch": res["fetch"], "write": res["write"],
           "note": "FETCH_SIZE and WRITE_SIZE from two rocprofv3 --pmc runs of "
                   "`python bench.py --profile --steps 2`, each scaled by the counter's "
                   "reading for a plain 2 GiB device copy in the same run"}
    os.makedirs(os.path.dirname(TRAFFIC_FILE), exist_ok=True)
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


# ---------------------------------------------------------------------------
def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--frames", type=int, default=10000)
    ap.add_argument("--pool", type=int, default=64)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--no-latency", action="store_true")
    ap.add_argument("--no-subpixel", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-summaries", action="store_true")
    ap.add_argument("--no-cm-mean", action="store_true")
    ap.add_argument("--phase-timers", action="store_true",
                    help="with the tracing build (PDC_LIB=.../libpdc_phase.so): per-phase cycles of the frame kernel")
    ap.add_argument("--serve-seconds", type=float, default=1.0,
                    help="seconds of Poisson arrivals per serving rate (the workload's own figure is 60)")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--profile", action="store_true")
    ap.add_argument("--ingest-pmc", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"))
    args = ap.parse_args()

    if args.ingest_pmc:
        ingest_pmc(*args.ingest_pmc)
        return
    if args.gpus != 1:
        print("bench.py: the benchmark runs on one GPU only (--gpus 1); frames shard across GPUs "
              "with no exchange between them, and no multi-GPU run is implemented", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1903_06838_amd import pdc, synth

    dev = torch.device("cuda:0")
    geom = synth.CSPAD
    npix = geom.pixels
    ped, gain = synth.make_calibration(geom, 1)
    ctx = pdc.create(0)
    det = pdc.calibrate(ctx, pdc.geometry(*geom.shape, geom.bank_cols), ped, gain, pdc.params())
    N = args.frames

    pool, frames = make_batch(torch, synth, geom, ped, gain, 1, args.pool, N, dev)
    est = int(0.01 * 1.2 * npix * N) + 4096
    # tile shape: strip height and frame-group count of the persistent launch,
    # tuned on this batch
    tune_rows, tune_mult, tune_ms = pdc.autotune_strips(ctx, det, frames, N, est, torch.cuda.current_stream())
    log("autotune: %d own rows per strip, frame groups x%d (frame kernel ms, rows by strip height, x1/x2/x4: %s)"
        % (tune_rows, tune_mult, [[round(float(x), 3) for x in row] for row in tune_ms]))
    phase_fn = None
    if args.phase_timers:
        import ctypes

        phase_fn = getattr(pdc._lib, "pdc_debug_phase_cycles", None)
        if phase_fn is None:
            sys.exit("--phase-timers needs the tracing build: PDC_PHASE_TIMERS=1 python -m paper_1903_06838_amd.build, "
                     "then PDC_LIB=paper_1903_06838_amd/libpdc_phase.so")
        phase_buf = (ctypes.c_ulonglong * (16 * 8))()
        phase_fn(phase_buf)  # clear what earlier launches left
    ms, mains, totals, hits, (fh, fp), hit_cap = run_steps(
        torch, pdc, ctx, det, frames, N, est, args.steps, args.warmup)
    step_ms = list(run_steps.step_ms)
    log("headline: %.3f ms/step, frame kernel %.3f ms, all kernels %.3f ms, %d hits"
        % (ms, sum(mains) / len(mains), sum(totals) / len(totals), hits))
    if phase_fn is not None:
        phase_fn(phase_buf)
        # each launch runs every strip-frame once on each wave index: CSPAD's
        # 5,920 rows make 198 strips of at most 30 own rows
        n_strips = -(-geom.n_tiles * geom.rows // 30)
        launches = args.steps + args.warmup
        names = ["A", "bar_AB", "medians", "seeds", "local_max", "hit_writes", "bar_BA"]
        rows = [[phase_buf[w * 8 + p] / (launches * N * n_strips) for p in range(7)] for w in range(16)]
        log("phase cycles per strip-frame per wave (s_memtime), %d launches of %d frames, %d strips:" % (
            launches, N, n_strips))
        log("wave " + " ".join("%10s" % n for n in names) + "      total")
        for w, r in enumerate(rows):
            log("%4d " % w + " ".join("%10.0f" % x for x in r) + " %10.0f" % sum(r))
        mean = [sum(r[p] for r in rows) / 16 for p in range(7)]
        log("mean " + " ".join("%10.0f" % x for x in mean) + " %10.0f" % sum(mean))
        print(json.dumps({"phase_timers": True, "frame_kernel_ms": sum(mains) / len(mains), "phases": names,
                          "cycles_per_strip_frame_per_wave": [[round(x, 1) for x in r] for r in rows]}))
        return

    if args.profile:
        src = torch.empty(COPY_BYTES // 2, dtype=torch.int16, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"profile_run": True, "ms_per_step": ms,
                          "frame_kernel_ms": sum(mains) / len(mains), "hits": hits}))
        pdc.destroy(ctx)
        return

    value = N * npix / (ms / 1e3) / 1e6
    out = {"metric": METRIC, "value": round(value, 1), "unit": "Mpixel/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": "CSPAD-like 32x185x388 uint16, 194-pixel banks, %d frames per "
                                  "batch (64 distinct, replicated in HBM), occupancy 0.01" % N,
                      "frames": N, "tiles": 32, "rows": 185, "cols": 388, "bank_cols": 194,
                      "occupancy": 0.01, "thresholds": "5 sigma seed, 3 sigma neighbours, sigma 3 ADU",
                      "tile_shape_autotuned": {"strip_rows": tune_rows, "frame_group_multiplier": tune_mult,
                                               "frame_kernel_ms_by_strip_rows_x1_x2_x4":
                                                   [[round(float(x), 3) for x in row] for row in tune_ms]}},
           "roofline": roofline(N, npix, hits, mains),
           "hits_per_step": hits,
           "all_kernels_ms": round(sum(totals) / len(totals), 4),
           "step_ms": stats_ms(step_ms), "frame_kernel_ms": stats_ms(mains)}

    # stream-copy context: achievable HBM bandwidth of a plain device copy
    src = torch.empty(COPY_BYTES // 2, dtype=torch.int16, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    out["copy_GBps"] = round(5 * 2 * COPY_BYTES / (time.perf_counter() - t0) / 1e9, 1)
    del src, dst
    # achievable HBM read bandwidth: a plain streaming read of the same batch
    nbytes = N * npix * 2
    pdc.stream_read(ctx, frames, nbytes, torch.cuda.current_stream())
    rd = [pdc.stream_read(ctx, frames, nbytes, torch.cuda.current_stream()) for _ in range(3)]
    rd_gbps = nbytes / (min(rd) / 1e3) / 1e9
    out["stream_read"] = {"bytes": nbytes, "ms_min": round(min(rd), 4), "GBps": round(rd_gbps, 1),
                          "frame_kernel_frac_of_stream_read": round(out["roofline"]["achieved"] / rd_gbps, 4)}
    log("stream read: %s" % out["stream_read"])

    if not args.no_cpu:
        def gpu_pool_hits(n):
            b = pdc.process_frames(ctx, det, frames, args.pool, n + 1024, torch.cuda.current_stream())
            h, total, _, _, _ = pdc.get_hits(ctx, b, args.pool)
            pdc.release_batch(ctx, b)
            return h if total == n else None
        cb, exact = cpu_baseline(pool, ped, gain, geom.bank_cols, fh, fp, gpu_pool_hits)
        out["cpu_baseline"] = cb
        out["bit_exact_vs_oracle"] = exact
        log("cpu baseline: %s; GPU bit-exact on the pool: %s" % (cb, exact))

    if not args.no_latency:
        lat = {"cspad_frame": latency(torch, pdc, ctx, det, frames[:1]),
               "cspad_frame_graph": latency(torch, pdc, ctx, det, frames[:1], use_graph=True),
               "cspad_16_frames": latency(torch, pdc, ctx, det, frames[:16]),
               "cspad_16_frames_graph": latency(torch, pdc, ctx, det, frames[:16], use_graph=True)}
        eg = synth.EPIX100
        eped, egain = synth.make_calibration(eg, 0)
        edet = pdc.calibrate(ctx, pdc.geometry(*eg.shape, eg.bank_cols), eped, egain, pdc.params())
        ef = torch.from_numpy(synth.make_frames(eg, eped, egain, 1, 0.01, 0)).to(dev)
        lat["epix100_frame"] = latency(torch, pdc, ctx, edet, ef)
        pdc.release_detector(ctx, edet)
        out["latency"] = lat
        log("latency: %s" % lat)

    if not args.no_serve:
        out["serving"] = serving(torch, pdc, ctx, seconds=args.serve_seconds)
        log("serving: %s" % out["serving"])

    if not args.no_cm_mean:
        cmr = []
        for mode, name in ((pdc.CM_BANK_MEAN, "bank"), (pdc.CM_TILE_MEAN, "tile")):
            cdet = pdc.calibrate(ctx, pdc.geometry(*geom.shape, geom.bank_cols), ped, gain,
                                 pdc.params(cm_mode=mode, cm_stages=3))
            ms_c, m_c, t_c, h_c, _, _ = run_steps(torch, pdc, ctx, cdet, frames, N, est, max(2, args.steps // 2), 1)
            pdc.release_detector(ctx, cdet)
            cmr.append({"region": name, "stages": 3, "ms_per_step": round(ms_c, 4),
                        "Mpixel_s": round(N * npix / (ms_c / 1e3) / 1e6, 1), "hits": h_c,
                        "frame_kernel_ms": round(sum(m_c) / len(m_c), 4),
                        "all_kernels_ms": round(sum(t_c) / len(t_c), 4),
                        "frame_kernel_roofline_frac": roofline(N, npix, h_c, m_c)["frac"]})
        out["cm_mean"] = cmr
        log("cm_mean: %s" % cmr)

    if not args.no_mixed:
        out["mixed"] = mixed(torch, pdc, ctx)
        log("mixed: %s" % out["mixed"])

    if not args.no_summaries:
        out["summaries"] = summaries(torch, pdc, ctx, geom, ped, gain, frames, N, hit_cap)
        log("summaries: %s" % out["summaries"])

    if not args.no_subpixel:
        out["subpixel"] = subpixel(torch, pdc, ctx)
        log("subpixel: %s" % out["subpixel"])

    if not args.no_sweep:
        sweep = [{"occupancy": 0.01, "Mpixel_s": out["value"], "frac": out["roofline"]["frac"],
                  "hits": hits}]
        del frames
        if "bit_exact_vs_oracle" in out:
            sweep[0]["bit_exact"] = out["bit_exact_vs_oracle"]
        for occ_id in (0, 2):
            pool2, fr = make_batch(torch, synth, geom, ped, gain, occ_id, args.pool, N, dev)
            occ = synth.CSPAD_OCCUPANCIES[occ_id]
            ms2, m2, _, h2, (fh2, fp2), _ = run_steps(torch, pdc, ctx, det, fr, N,
                                                      int(occ * 1.3 * npix * N) + 4096, max(2, args.steps // 3), 1)
            rf = roofline(N, npix, h2, m2)
            ent = {"occupancy": occ, "Mpixel_s": round(N * npix / (ms2 / 1e3) / 1e6, 1),
                   "frac": rf["frac"], "hits": h2, "ms_per_step": round(ms2, 4)}

            def pool_hits(n, fr=fr):
                b = pdc.process_frames(ctx, det, fr, args.pool, n + 1024, torch.cuda.current_stream())
                h, total, _, _, _ = pdc.get_hits(ctx, b, args.pool)
                pdc.release_batch(ctx, b)
                return h if total == n else None
            ent["bit_exact"] = pool_check(pool2, ped, gain, geom.bank_cols, fh2, fp2, pool_hits)
            log("sweep: %s" % ent)
            sweep.append(ent)
            del fr
        out["sweep"] = sorted(sweep, key=lambda s: s["occupancy"])
    pdc.destroy(ctx)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
