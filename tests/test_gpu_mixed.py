"""Mixed batches (pdc_process_mixed): several detectors with different
geometries, gain modes and common-mode settings enqueued at once, running
concurrently or in one launch of the persistent kernel; every batch equals
its oracle bit for bit and work enqueued afterwards on the caller's stream
sees all of them finished."""
import numpy as np
import pytest

from oracle import cm_mean as M
from oracle import multigain as G
from paper_1903_06838_amd import synth
from tests.helpers import assert_same, oracle_threads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1903_06838_amd import pdc

    c = pdc.create(0)
    yield c
    pdc.destroy(c)


FEW_LOW_GAIN = dict(range_frac=(0.95, 0.03, 0.01), invalid_frac=0.01)


def _detectors():
    """(geometry, gain_mode, cm_mode, raw, ped, gain, want)"""
    out = []
    g = synth.Geometry(1, 64, 768, 96)                 # ePix100-like rows, single gain, median
    ped, gain = synth.make_calibration(g, 41)
    raw = synth.make_frames(g, ped, gain, 5, 0.01, 41)
    out.append((g, 0, 0, raw, ped, gain, oracle_threads(raw, ped, gain, 96, keep_corrected=True)))
    g = synth.Geometry(2, 40, 388, 194)                # CSPAD-like, bank mean with 2 stages
    ped, gain = synth.make_calibration(g, 45)
    raw = synth.make_frames(g, ped, gain, 6, 0.01, 45)
    out.append((g, 0, 1, raw, ped, gain, M.process(raw, ped, gain, 194, M.BANK, 2, keep_corrected=True)))
    g = synth.Geometry(1, 64, 384, 96)                 # ePix10k-like, three gain ranges
    ped, gain = synth.make_calibration_multigain(g, 42)
    raw = synth.make_frames_multigain(g, ped, gain, 7, 0.02, 42, 1, **FEW_LOW_GAIN)
    out.append((g, 1, 0, raw, ped, gain, G.process(raw, ped, gain, 96, 1, keep_corrected=True)))
    g = synth.Geometry(1, 48, 1024, 256)               # Jungfrau-like, three gain ranges
    ped, gain = synth.make_calibration_multigain(g, 43)
    raw = synth.make_frames_multigain(g, ped, gain, 4, 0.005, 43, 2, **FEW_LOW_GAIN)
    out.append((g, 2, 0, raw, ped, gain, G.process(raw, ped, gain, 256, 2, keep_corrected=True)))
    return out


def test_mixed_batch_equals_oracle(ctx):
    import torch

    from paper_1903_06838_amd import pdc

    dets, items, devs = [], [], []
    cases = _detectors()
    try:
        for g, gm, cm, raw, ped, gain, _ in cases:
            prm = pdc.params(flags=pdc.KEEP_CORRECTED, cm_mode=cm, cm_stages=2)
            d = pdc.calibrate(ctx, pdc.geometry(*g.shape, g.bank_cols, gm), ped, gain, prm)
            dets.append(d)
            dev = torch.from_numpy(raw).cuda()
            devs.append(dev)
            items.append((d, dev, raw.shape[0], 1 << 16))
        stream = torch.cuda.Stream()
        batches = pdc.process_mixed(ctx, items, stream)
        # work enqueued after the call on the same stream waits for every batch
        flag = torch.zeros(1, device="cuda")
        with torch.cuda.stream(stream):
            flag += 1
        stream.synchronize()
        for b, (g, gm, cm, raw, ped, gain, want) in zip(batches, cases):
            hits, total, fh, fp, _ = pdc.get_hits(ctx, b, raw.shape[0])
            corr = np.empty(raw.shape, np.float32)
            pdc.get_corrected(ctx, b, corr)
            got = dict(hits=hits, total=total, frame_hits=fh, frame_photons=fp, corrected=corr)
            assert_same(got, want, corrected=True)
            assert pdc.debug_batch_path(ctx, b) == 2, (g, gm, cm)
            if gm:
                assert np.array_equal(pdc.get_invalid_counts(ctx, b, raw.shape[0]), want["invalid"])
            pdc.release_batch(ctx, b)
    finally:
        for d in dets:
            pdc.release_detector(ctx, d)


def _one_launch_detectors():
    """Median common mode, nothing kept: four lane layouts and gain modes of
    the one-launch kernel, with different frame counts."""
    out = []
    g = synth.Geometry(1, 64, 768, 96)                 # ePix100-like rows, 8 lanes per bank
    ped, gain = synth.make_calibration(g, 51)
    raw = synth.make_frames(g, ped, gain, 5, 0.01, 51)
    out.append((g, 0, raw, ped, gain, oracle_threads(raw, ped, gain, 96)))
    g = synth.Geometry(2, 40, 388, 194)                # CSPAD-like, 16 lanes per bank
    ped, gain = synth.make_calibration(g, 52)
    raw = synth.make_frames(g, ped, gain, 6, 0.02, 52)
    out.append((g, 0, raw, ped, gain, oracle_threads(raw, ped, gain, 194)))
    g = synth.Geometry(1, 64, 384, 96)                 # ePix10k-like, three gain ranges
    ped, gain = synth.make_calibration_multigain(g, 53)
    raw = synth.make_frames_multigain(g, ped, gain, 7, 0.02, 53, 1, **FEW_LOW_GAIN)
    out.append((g, 1, raw, ped, gain, G.process(raw, ped, gain, 96, 1)))
    g = synth.Geometry(1, 48, 1024, 256)               # Jungfrau-like, three gain ranges
    ped, gain = synth.make_calibration_multigain(g, 54)
    raw = synth.make_frames_multigain(g, ped, gain, 3, 0.01, 54, 2, **FEW_LOW_GAIN)
    out.append((g, 2, raw, ped, gain, G.process(raw, ped, gain, 256, 2)))
    return out


def test_mixed_one_launch_equals_oracle(ctx):
    """The four batches run as one launch (path 4, or 5 with overflowing
    units redone) and equal their oracles; a context with PDC_MIX_FORKED=1
    runs them as launches of their own (path 2 or 3) with the same results."""
    import os

    import torch

    from paper_1903_06838_amd import pdc

    cases = _one_launch_detectors()
    os.environ["PDC_MIX_FORKED"] = "1"
    try:
        forked = pdc.create(0)
    finally:
        del os.environ["PDC_MIX_FORKED"]
    try:
        got = {}
        for c, name in ((ctx, "one"), (forked, "forked")):
            dets, items, devs = [], [], []
            try:
                for g, gm, raw, ped, gain, _ in cases:
                    d = pdc.calibrate(c, pdc.geometry(*g.shape, g.bank_cols, gm), ped, gain, pdc.params())
                    dets.append(d)
                    dev = torch.from_numpy(raw).cuda()
                    devs.append(dev)
                    items.append((d, dev, raw.shape[0], 1 << 16))
                torch.cuda.synchronize()
                stream = torch.cuda.Stream()
                batches = pdc.process_mixed(c, items, stream)
                stream.synchronize()
                res = []
                for b, (g, gm, raw, ped, gain, want) in zip(batches, cases):
                    hits, total, fh, fp, _ = pdc.get_hits(c, b, raw.shape[0])
                    out = dict(hits=hits, total=total, frame_hits=fh, frame_photons=fp,
                               path=pdc.debug_batch_path(c, b))
                    if gm:
                        out["invalid"] = pdc.get_invalid_counts(c, b, raw.shape[0])
                    pdc.release_batch(c, b)
                    res.append(out)
                got[name] = res
            finally:
                for d in dets:
                    pdc.release_detector(c, d)
    finally:
        pdc.destroy(forked)
    for one, fk, (g, gm, raw, ped, gain, want) in zip(got["one"], got["forked"], cases):
        assert one["path"] in (4, 5) and fk["path"] in (2, 3), (g, one["path"], fk["path"])
        for r in (one, fk):
            assert_same(r, want)
            if gm:
                assert np.array_equal(r["invalid"], want["invalid"])


def test_mixed_one_launch_edge_items(ctx):
    """Two batches of one detector share the one launch (path 4 or 5); a mix
    with an empty item launches per batch (path 2 or 3); every non-empty batch
    equals its oracle."""
    import torch

    from paper_1903_06838_amd import pdc

    cases = _one_launch_detectors()
    g0, gm0, raw0, ped0, gain0, want0 = cases[0]
    g1, gm1, raw1, ped1, gain1, want1 = cases[3]
    d0 = pdc.calibrate(ctx, pdc.geometry(*g0.shape, g0.bank_cols, gm0), ped0, gain0, pdc.params())
    d1 = pdc.calibrate(ctx, pdc.geometry(*g1.shape, g1.bank_cols, gm1), ped1, gain1, pdc.params())
    try:
        dev0, dev1 = torch.from_numpy(raw0).cuda(), torch.from_numpy(raw1).cuda()
        torch.cuda.synchronize()
        for items, paths, wants in (
                ([(d0, dev0, raw0.shape[0], 1 << 16), (d0, dev0, raw0.shape[0], 1 << 16),
                  (d1, dev1, raw1.shape[0], 1 << 16)], (4, 5), (want0, want0, want1)),
                ([(d0, dev0, raw0.shape[0], 1 << 16), (d1, dev1, 0, 1 << 16)], (2, 3), (want0, None))):
            stream = torch.cuda.Stream()
            batches = pdc.process_mixed(ctx, items, stream)
            stream.synchronize()
            for b, it, want in zip(batches, items, wants):
                n = it[2]
                hits, total, fh, fp, _ = pdc.get_hits(ctx, b, max(n, 1))
                if want is None:
                    assert total == 0
                else:
                    assert pdc.debug_batch_path(ctx, b) in paths
                    assert_same(dict(hits=hits, total=total, frame_hits=fh, frame_photons=fp), want)
                pdc.release_batch(ctx, b)
    finally:
        pdc.release_detector(ctx, d0)
        pdc.release_detector(ctx, d1)


def test_mixed_rejects_bad_items(ctx):
    import torch

    from paper_1903_06838_amd import pdc

    g = synth.Geometry(1, 8, 16, 8)
    ped, gain = synth.make_calibration(g, 44)
    d = pdc.calibrate(ctx, pdc.geometry(*g.shape, 8), ped, gain, pdc.params())
    try:
        dev = torch.zeros((2, 1, 8, 16), dtype=torch.int16, device="cuda")
        torch.cuda.synchronize()  # torch fills on its stream, the library runs on its own
        with pytest.raises(pdc.PdcError) as e:
            pdc.process_mixed(ctx, [(d, dev, 2, 1024), (d + 100, dev, 2, 1024)])
        assert e.value.status == pdc.ESTATE
        with pytest.raises(pdc.PdcError):
            pdc.process_mixed(ctx, [(d, None, 2, 1024)])
        b = pdc.process_mixed(ctx, [(d, dev, 2, 1024)])[0]
        pdc.release_batch(ctx, b)
    finally:
        pdc.release_detector(ctx, d)
