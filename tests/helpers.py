"""Shared helpers for the parity tests: run a batch through the C ABI, run the
oracle (frame-parallel threads; ctypes releases the GIL), compare bit for bit."""
from __future__ import annotations

import concurrent.futures as cf
import os

import numpy as np

from oracle import oracle


def oracle_threads(raw, ped, gain, bank_cols, threads=None, **kw):
    """Oracle over frame chunks in parallel threads; same output as one call."""
    o = oracle.load()
    N = raw.shape[0]
    if N == 0:
        return o.process(raw, ped, gain, bank_cols, **kw)
    threads = threads or min(16, os.cpu_count() or 1, N)
    bounds = np.linspace(0, N, threads + 1).astype(int)
    parts = [(bounds[i], bounds[i + 1]) for i in range(threads) if bounds[i + 1] > bounds[i]]
    with cf.ThreadPoolExecutor(len(parts)) as ex:
        outs = list(ex.map(lambda ab: o.process(raw[ab[0]:ab[1]], ped, gain, bank_cols, **kw), parts))
    hits = []
    for (a, _), r in zip(parts, outs):
        h = r["hits"].copy()
        h["frame"] += np.uint32(a)
        hits.append(h)
    res = dict(hits=np.concatenate(hits), frame_hits=np.concatenate([r["frame_hits"] for r in outs]),
               frame_photons=np.concatenate([r["frame_photons"] for r in outs]),
               total=sum(r["total"] for r in outs))
    if kw.get("keep_corrected"):
        res["corrected"] = np.concatenate([r["corrected"] for r in outs])
    return res


def hits_u32(h):
    return np.ascontiguousarray(h).view(np.uint32).reshape(-1, 4)


def assert_same(got, want, corrected=False):
    assert got["total"] == want["total"], (got["total"], want["total"])
    assert np.array_equal(got["frame_hits"], want["frame_hits"])
    assert np.array_equal(got["frame_photons"], want["frame_photons"])
    g, w = hits_u32(got["hits"]), hits_u32(want["hits"])
    assert len(g) == len(w) == got["total"], (len(g), len(w), got["total"])
    if not np.array_equal(g, w):
        bad = np.nonzero(np.any(g != w, axis=1))[0] if g.shape == w.shape else [0]
        raise AssertionError("hit lists differ (first differing record %s): got %s want %s" % (
            bad[0], g[bad[0]] if len(g) > bad[0] else None, w[bad[0]] if len(w) > bad[0] else None))
    if corrected:
        assert np.array_equal(got["corrected"].view(np.uint32), want["corrected"].view(np.uint32))


def run_pdc(ctx, raw, ped, gain, bank_cols, sigma=3.0, n_seed=5.0, n_nb=3.0, photon_adu=150.0,
            keep_corrected=False, hit_capacity=None, stream=None, frames_dev=None):
    """One batch through libpdc; returns the same dict layout as the oracle."""
    import torch

    from paper_1903_06838_amd import pdc

    N, T, H, W = raw.shape
    geom = pdc.geometry(T, H, W, bank_cols)
    prm = pdc.params(sigma, n_seed, n_nb, photon_adu, pdc.KEEP_CORRECTED if keep_corrected else 0)
    det = pdc.calibrate(ctx, geom, ped, gain, prm)
    try:
        if frames_dev is None:
            frames_dev = torch.from_numpy(np.ascontiguousarray(raw)).cuda()
        if hit_capacity is None:
            hit_capacity = max(1024, int(raw.size * 0.06))
        b = pdc.process_frames(ctx, det, frames_dev, N, hit_capacity, stream)
        hits, total, fh, fp, st = pdc.get_hits(ctx, b, N)
        out = dict(hits=hits, total=total, frame_hits=fh, frame_photons=fp, status=st, batch=b)
        if keep_corrected:
            corr = np.empty(raw.shape, dtype=np.float32)
            pdc.get_corrected(ctx, b, corr)
            out["corrected"] = corr
        pdc.release_batch(ctx, b)
    finally:
        pdc.release_detector(ctx, det)
    return out
