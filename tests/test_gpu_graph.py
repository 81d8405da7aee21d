"""HIP graph capture of a batch (pdc_graph_create / pdc_graph_launch) through
the C ABI: every replay equals the eager batch of the same frames bit for bit
(and the oracle), with eager work and synchronizations between replays, new
frames written into the captured buffer before each launch, the seed-list
fallback and the staging-overflow recomputation on replayed batches, and the
one-batch-per-graph rule."""
import os

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


def _results(ctx, b, n, keep=True, shape=None, invalid=False):
    from paper_1903_06838_amd import pdc

    hits, total, fh, fp, _ = pdc.get_hits(ctx, b, n)
    out = dict(hits=hits, total=total, frame_hits=fh, frame_photons=fp, path=pdc.debug_batch_path(ctx, b))
    if keep:
        corr = np.empty(shape, np.float32)
        pdc.get_corrected(ctx, b, corr)
        out["corrected"] = corr
    if invalid:
        out["invalid"] = pdc.get_invalid_counts(ctx, b, n)
    return out


def _same(got, want, keep=True):
    assert_same(got, want, corrected=keep)
    if "invalid" in want:
        assert np.array_equal(got["invalid"], want["invalid"])


def test_graph_replays_match_eager_and_oracle(ctx):
    """Five replays over three frame sets (one with flood frames whose strips
    the general kernel redoes into the graph's buffers) on a caller stream."""
    import torch

    from paper_1903_06838_amd import pdc

    geom = synth.Geometry(2, 60, 388, 194)
    ped, gain = synth.make_calibration(geom, 61)
    n = 4
    sets = [synth.make_frames(geom, ped, gain, n, 0.01, 62),
            synth.make_frames(geom, ped, gain, n, 0.03, 63),
            np.concatenate([synth.make_frames(geom, ped, gain, 2, 0.4, 64),
                            synth.make_frames(geom, ped, gain, 2, 0.01, 65)])]
    wants = [oracle_threads(r, ped, gain, 194, keep_corrected=True) for r in sets]
    det = pdc.calibrate(ctx, pdc.geometry(*geom.shape, 194), ped, gain, pdc.params(flags=pdc.KEEP_CORRECTED))
    graph = None
    try:
        devs = [torch.from_numpy(r).cuda() for r in sets]
        eager = []
        for r, dv, w in zip(sets, devs, wants):
            b = pdc.process_frames(ctx, det, dv, n, 1 << 16)
            got = _results(ctx, b, n, shape=r.shape)
            pdc.release_batch(ctx, b)
            _same(got, w)
            eager.append(got)
        assert [e["path"] for e in eager] == [2, 2, 3]
        buf = torch.empty_like(devs[0])
        torch.cuda.synchronize()
        graph = pdc.graph_create(ctx, det, buf, n, 1 << 16)
        s = torch.cuda.Stream()
        other = torch.from_numpy(synth.make_frames(geom, ped, gain, 3, 0.02, 66)).cuda()
        for rep, k in enumerate([0, 1, 2, 0, 1]):
            with torch.cuda.stream(s):
                buf.copy_(devs[k])          # ordered before the launch on the same stream
            b = pdc.graph_launch(ctx, graph, s)
            got = _results(ctx, b, n, shape=sets[k].shape)
            assert got["path"] == eager[k]["path"], rep
            _same(got, eager[k])
            main_ms, total_ms = pdc.batch_timing(ctx, b)
            assert 0 < main_ms <= total_ms
            pdc.release_batch(ctx, b)
            # the program's own eager work between replays
            eb = pdc.process_frames(ctx, det, other, 3, 1 << 14)
            pdc.get_hits(ctx, eb, 3, capacity=0)
            pdc.release_batch(ctx, eb)
            (other.float() * 2).sum().item()
            torch.cuda.synchronize()
    finally:
        if graph is not None:
            pdc.graph_destroy(ctx, graph)
        pdc.release_detector(ctx, det)


def test_graph_one_batch_at_a_time_and_detector_lifetime(ctx):
    import torch

    from paper_1903_06838_amd import pdc

    geom = synth.Geometry(1, 40, 384, 96)
    ped, gain = synth.make_calibration(geom, 67)
    raw = synth.make_frames(geom, ped, gain, 3, 0.02, 67)
    want = oracle_threads(raw, ped, gain, 96)
    det = pdc.calibrate(ctx, pdc.geometry(*geom.shape, 96), ped, gain, pdc.params())
    buf = torch.from_numpy(raw).cuda()
    torch.cuda.synchronize()
    graph = pdc.graph_create(ctx, det, buf, 3, 1 << 14)
    b = pdc.graph_launch(ctx, graph)
    with pytest.raises(pdc.PdcError) as e:
        pdc.graph_launch(ctx, graph)
    assert e.value.status == pdc.ESTATE
    with pytest.raises(pdc.PdcError) as e:
        pdc.graph_destroy(ctx, graph)
    assert e.value.status == pdc.ESTATE
    # the graph holds the detector: its planes outlive pdc_release_detector
    pdc.release_detector(ctx, det)
    got = _results(ctx, b, 3, keep=False)
    assert_same(got, want)
    pdc.release_batch(ctx, b)
    for _ in range(2):
        b = pdc.graph_launch(ctx, graph)
        assert_same(_results(ctx, b, 3, keep=False), want)
        pdc.release_batch(ctx, b)
    pdc.graph_destroy(ctx, graph)
    with pytest.raises(pdc.PdcError):
        pdc.graph_create(ctx, det, buf, 3, 1024)
    with pytest.raises(pdc.PdcError) as e:
        pdc.graph_create(ctx, 12345, buf, 3, 1024)
    assert e.value.status == pdc.ESTATE


def test_graph_staging_overflow_moves_batch_off_graph():
    """With no staging slack and capacity 0 every replay overflows: the batch is
    recomputed on buffers of its own (so the graph may be launched again before
    the batch is released) and stays exact; eager batches agree."""
    import torch

    from paper_1903_06838_amd import pdc

    geom = synth.Geometry(2, 60, 194, 97)
    ped, gain = synth.make_calibration(geom, 68)
    raw = synth.make_frames(geom, ped, gain, 5, 0.05, 68)
    want = oracle_threads(raw, ped, gain, 97, keep_corrected=True)
    assert want["total"] > 100
    os.environ["PDC_DEBUG_TIGHT_POOL"] = "1"
    try:
        c = pdc.create(0)
    finally:
        del os.environ["PDC_DEBUG_TIGHT_POOL"]
    try:
        det = pdc.calibrate(c, pdc.geometry(*geom.shape, 97), ped, gain, pdc.params(flags=pdc.KEEP_CORRECTED))
        buf = torch.from_numpy(raw).cuda()
        torch.cuda.synchronize()
        b = pdc.process_frames(c, det, buf, 5, 0)
        _same(_results(c, b, 5, shape=raw.shape), want)
        pdc.release_batch(c, b)
        graph = pdc.graph_create(c, det, buf, 5, 0)
        b1 = pdc.graph_launch(c, graph)
        _same(_results(c, b1, 5, shape=raw.shape), want)
        b2 = pdc.graph_launch(c, graph)      # b1 no longer holds the graph's buffers
        _same(_results(c, b2, 5, shape=raw.shape), want)
        _same(_results(c, b1, 5, shape=raw.shape), want)  # b1 kept its own results
        pdc.release_batch(c, b1)
        pdc.release_batch(c, b2)
        b3 = pdc.graph_launch(c, graph)
        _same(_results(c, b3, 5, shape=raw.shape), want)
        pdc.release_batch(c, b3)
        pdc.graph_destroy(c, graph)
        pdc.release_detector(c, det)
    finally:
        pdc.destroy(c)


FEW_LOW_GAIN = dict(range_frac=(0.95, 0.03, 0.01), invalid_frac=0.01)


@pytest.mark.parametrize("gm,cm,stages", [(0, 2, 2), (2, 1, 3), (1, 2, 1)], ids=str)
def test_graph_common_mode_and_multigain(ctx, gm, cm, stages):
    """Graphs holding the common-mode pass and the invalid-count fill kernel;
    three replays, two frame sets, against the oracles."""
    import torch

    from paper_1903_06838_amd import pdc

    geom = synth.Geometry(2, 40, 388, 194)
    n = 3
    # a tile's mean cannot follow per-bank offsets: keep them small in tile mode
    sim = synth.SimParams(cm_sigma=1.0) if cm == 2 else synth.SimParams()
    sets, wants = [], []
    if gm:
        ped, gain = synth.make_calibration_multigain(geom, 69)
        for sd in (70, 71):
            r = synth.make_frames_multigain(geom, ped, gain, n, 0.02, sd, gm, sim=sim, **FEW_LOW_GAIN)
            sets.append(r)
            wants.append(G.process(r, ped, gain, 194, gm, cm, stages, keep_corrected=True))
    else:
        ped, gain = synth.make_calibration(geom, 69)
        for sd in (70, 71):
            r = synth.make_frames(geom, ped, gain, n, 0.02, sd, sim=sim)
            sets.append(r)
            wants.append(M.process(r, ped, gain, 194, cm, stages, keep_corrected=True))
    prm = pdc.params(flags=pdc.KEEP_CORRECTED, cm_mode=cm, cm_stages=stages)
    det = pdc.calibrate(ctx, pdc.geometry(*geom.shape, 194, gm), ped, gain, prm)
    graph = None
    try:
        devs = [torch.from_numpy(r).cuda() for r in sets]
        buf = torch.empty_like(devs[0])
        torch.cuda.synchronize()
        graph = pdc.graph_create(ctx, det, buf, n, 1 << 16)
        s = torch.cuda.Stream()
        for k in (0, 1, 0):
            with torch.cuda.stream(s):
                buf.copy_(devs[k])
            b = pdc.graph_launch(ctx, graph, s)
            got = _results(ctx, b, n, shape=sets[k].shape, invalid=bool(gm))
            pdc.release_batch(ctx, b)
            _same(got, wants[k])
            torch.cuda.synchronize()
    finally:
        if graph is not None:
            pdc.graph_destroy(ctx, graph)
        pdc.release_detector(ctx, det)


def test_mixed_graph_replays_equal_oracle(ctx):
    """One graph over three detectors (ePix100-like rows with the median,
    CSPAD-like with the 2-stage bank mean, Jungfrau-like with three gain
    ranges): each of three replays, with new frames written into the captured
    buffers and eager work in between, equals the oracles for every detector;
    the graph takes no launch while one of its batches is outstanding."""
    import torch

    from paper_1903_06838_amd import pdc

    n = 3
    specs = []
    g = synth.Geometry(1, 64, 768, 96)
    ped, gain = synth.make_calibration(g, 81)
    sets = [synth.make_frames(g, ped, gain, n, 0.01, sd) for sd in (81, 82)]
    specs.append((g, 0, 0, 1, ped, gain, sets, [oracle_threads(r, ped, gain, 96, keep_corrected=True) for r in sets]))
    g = synth.Geometry(2, 40, 388, 194)
    ped, gain = synth.make_calibration(g, 83)
    sets = [synth.make_frames(g, ped, gain, n, 0.02, sd) for sd in (83, 84)]
    specs.append((g, 0, 1, 2, ped, gain, sets, [M.process(r, ped, gain, 194, M.BANK, 2, keep_corrected=True)
                                                for r in sets]))
    g = synth.Geometry(1, 48, 1024, 256)
    ped, gain = synth.make_calibration_multigain(g, 85)
    sets = [synth.make_frames_multigain(g, ped, gain, n, 0.01, sd, 2, **FEW_LOW_GAIN) for sd in (85, 86)]
    specs.append((g, 2, 0, 1, ped, gain, sets, [G.process(r, ped, gain, 256, 2, keep_corrected=True) for r in sets]))

    dets, graph = [], None
    try:
        for g, gm, cm, st, ped, gain, _, _ in specs:
            prm = pdc.params(flags=pdc.KEEP_CORRECTED, cm_mode=cm, cm_stages=st)
            dets.append(pdc.calibrate(ctx, pdc.geometry(*g.shape, g.bank_cols, gm), ped, gain, prm))
        devs = [[torch.from_numpy(r).cuda() for r in sp[6]] for sp in specs]
        bufs = [torch.empty_like(dv[0]) for dv in devs]
        torch.cuda.synchronize()
        graph = pdc.graph_create_mixed(ctx, [(d, b, n, 1 << 18) for d, b in zip(dets, bufs)])
        s = torch.cuda.Stream()
        other = devs[0][1]
        for k in (0, 1, 0):
            with torch.cuda.stream(s):
                for b, dv in zip(bufs, devs):
                    b.copy_(dv[k])
            batches = pdc.graph_launch(ctx, graph, s)
            assert len(batches) == len(specs)
            with pytest.raises(pdc.PdcError) as e:
                pdc.graph_launch(ctx, graph, s)
            assert e.value.status == pdc.ESTATE
            for b, sp in zip(batches, specs):
                got = _results(ctx, b, n, shape=sp[6][k].shape, invalid=bool(sp[1]))
                pdc.release_batch(ctx, b)
                _same(got, sp[7][k])
            # the program's own eager work between replays
            eb = pdc.process_frames(ctx, dets[0], other, n, 1 << 16)
            pdc.get_hits(ctx, eb, n, capacity=0)
            pdc.release_batch(ctx, eb)
            (other.float() + 1).sum().item()
            torch.cuda.synchronize()
    finally:
        if graph is not None:
            pdc.graph_destroy(ctx, graph)
        for d in dets:
            pdc.release_detector(ctx, d)


def test_mixed_graph_one_launch_replays_equal_oracle(ctx):
    """A graph of three detectors whose frame kernels are one launch
    (median, nothing kept: ePix100-like rows, CSPAD-like, Jungfrau-like with
    three gain ranges): each of three replays with new frames equals the
    oracles, and each batch reports the one-launch path."""
    import torch

    from paper_1903_06838_amd import pdc

    n = 3
    specs = []
    g = synth.Geometry(1, 64, 768, 96)
    ped, gain = synth.make_calibration(g, 91)
    sets = [synth.make_frames(g, ped, gain, n, 0.01, sd) for sd in (91, 92)]
    specs.append((g, 0, ped, gain, sets, [oracle_threads(r, ped, gain, 96) for r in sets]))
    g = synth.Geometry(2, 40, 388, 194)
    ped, gain = synth.make_calibration(g, 93)
    sets = [synth.make_frames(g, ped, gain, n, 0.02, sd) for sd in (93, 94)]
    specs.append((g, 0, ped, gain, sets, [oracle_threads(r, ped, gain, 194) for r in sets]))
    g = synth.Geometry(1, 48, 1024, 256)
    ped, gain = synth.make_calibration_multigain(g, 95)
    sets = [synth.make_frames_multigain(g, ped, gain, n, 0.01, sd, 2, **FEW_LOW_GAIN) for sd in (95, 96)]
    specs.append((g, 2, ped, gain, sets, [G.process(r, ped, gain, 256, 2) for r in sets]))

    dets, graph = [], None
    try:
        for g, gm, ped, gain, _, _ in specs:
            dets.append(pdc.calibrate(ctx, pdc.geometry(*g.shape, g.bank_cols, gm), ped, gain, pdc.params()))
        devs = [[torch.from_numpy(r).cuda() for r in sp[4]] for sp in specs]
        bufs = [torch.empty_like(dv[0]) for dv in devs]
        torch.cuda.synchronize()
        graph = pdc.graph_create_mixed(ctx, [(d, b, n, 1 << 18) for d, b in zip(dets, bufs)])
        s = torch.cuda.Stream()
        for k in (0, 1, 0):
            with torch.cuda.stream(s):
                for b, dv in zip(bufs, devs):
                    b.copy_(dv[k])
            batches = pdc.graph_launch(ctx, graph, s)
            for b, sp in zip(batches, specs):
                got = _results(ctx, b, n, keep=False, invalid=bool(sp[1]))
                pdc.release_batch(ctx, b)
                assert got["path"] in (4, 5), got["path"]
                _same(got, sp[5][k], keep=False)
            (devs[0][1].float() + 1).sum().item()
            torch.cuda.synchronize()
    finally:
        if graph is not None:
            pdc.graph_destroy(ctx, graph)
        for d in dets:
            pdc.release_detector(ctx, d)


def test_mixed_graph_items_move_off_graph_on_overflow():
    """No staging slack and capacity 0: every item of a two-detector graph
    overflows and is recomputed on buffers of its own, each item freeing its
    place in the graph, so the graph launches again before those batches are
    released; every result equals the oracle."""
    import torch

    from paper_1903_06838_amd import pdc

    n = 3
    g1 = synth.Geometry(2, 40, 388, 194)
    p1, k1 = synth.make_calibration(g1, 91)
    r1 = synth.make_frames(g1, p1, k1, n, 0.03, 91)
    g2 = synth.Geometry(1, 30, 192, 96)
    p2, k2 = synth.make_calibration(g2, 92)
    r2 = synth.make_frames(g2, p2, k2, n, 0.05, 92)
    w1 = oracle_threads(r1, p1, k1, 194)
    w2 = oracle_threads(r2, p2, k2, 96)
    os.environ["PDC_DEBUG_TIGHT_POOL"] = "1"
    try:
        c = pdc.create(0)
    finally:
        del os.environ["PDC_DEBUG_TIGHT_POOL"]
    try:
        d1 = pdc.calibrate(c, pdc.geometry(*g1.shape, 194), p1, k1, pdc.params())
        d2 = pdc.calibrate(c, pdc.geometry(*g2.shape, 96), p2, k2, pdc.params())
        f1, f2 = torch.from_numpy(r1).cuda(), torch.from_numpy(r2).cuda()
        torch.cuda.synchronize()
        graph = pdc.graph_create_mixed(c, [(d1, f1, n, 0), (d2, f2, n, 0)])
        first = pdc.graph_launch(c, graph)
        for b, w in zip(first, (w1, w2)):
            assert_same(_results(c, b, n, keep=False), w)
        second = pdc.graph_launch(c, graph)  # both items left the graph's buffers
        for b, w in zip(second, (w1, w2)):
            assert_same(_results(c, b, n, keep=False), w)
        for b, w in zip(first, (w1, w2)):  # the first batches kept their own results
            assert_same(_results(c, b, n, keep=False), w)
        for b in first + second:
            pdc.release_batch(c, b)
        pdc.graph_destroy(c, graph)
        pdc.release_detector(c, d1)
        pdc.release_detector(c, d2)
    finally:
        pdc.destroy(c)
