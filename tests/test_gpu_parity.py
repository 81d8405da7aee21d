"""Parity of the HIP path (through the C ABI) with the CPU oracle, bit for bit:
hit lists (frame, pixel, charge bits, count), per-frame hit counts and photon
totals, and Frames2 where requested."""
import numpy as np
import pytest

from paper_1903_06838_amd import synth
from tests.helpers import assert_same, hits_u32, oracle_threads, run_pdc

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1903_06838_amd import pdc

    c = pdc.create(0)
    yield c
    pdc.destroy(c)


def _case(geom, occ, n_frames, cfg_id):
    ped, gain = synth.make_calibration(geom, cfg_id)
    raw = synth.make_frames(geom, ped, gain, n_frames, occ, cfg_id)
    return raw, ped, gain


def test_epix100_full_batch(ctx):
    """ePix100 704x768, 96-pixel banks, 100 frames at 0.01 photons/pixel: every
    hit, every count and every corrected pixel."""
    geom = synth.EPIX100
    raw, ped, gain = _case(geom, 0.01, 100, 0)
    want = oracle_threads(raw, ped, gain, geom.bank_cols, keep_corrected=True)
    got = run_pdc(ctx, raw, ped, gain, geom.bank_cols, keep_corrected=True)
    assert want["total"] > 400000
    assert_same(got, want, corrected=True)


RAGGED = [
    # (T, H, W, B, occupancy, frames)
    (1, 1, 1, 1, 0.5, 3),
    (1, 3, 5, 5, 0.3, 2),
    (3, 17, 40, 8, 0.05, 3),
    (2, 13, 388, 194, 0.05, 2),
    (1, 7, 96, 96, 0.1, 4),
    (4, 30, 64, 32, 0.05, 2),
    (1, 50, 100, 25, 0.05, 2),
    (1, 2, 1024, 1024, 0.02, 2),
    (2, 185, 388, 194, 0.05, 2),
    (1, 33, 2048, 128, 0.01, 1),
    (1, 9, 2048, 1, 0.05, 1),
]


@pytest.mark.parametrize("T,H,W,B,occ,n", RAGGED, ids=lambda x: str(x))
def test_ragged_geometries(ctx, T, H, W, B, occ, n):
    geom = synth.Geometry(T, H, W, B)
    raw, ped, gain = _case(geom, occ, n, 100 + T * 7 + H)
    want = oracle_threads(raw, ped, gain, B, keep_corrected=True)
    got = run_pdc(ctx, raw, ped, gain, B, keep_corrected=True)
    assert_same(got, want, corrected=True)


def test_adversarial_ties(ctx):
    """Integer frames with unit gain and integer dark: dense plateaus and exact
    ties in the median and the local maximum, thresholds hit exactly."""
    rng = np.random.default_rng(5)
    T, H, W, B = 2, 24, 60, 12
    ped = rng.integers(1000, 1010, size=(T, H, W)).astype(np.float32)
    gain = np.ones((T, H, W), np.float32)
    raw = (ped[None] + rng.choice([0, 0, 0, 9, 15, 16, 30, 30, 45], size=(5, T, H, W))).astype(np.uint16)
    for n_nb in (3.0, 0.0, 5.0):
        want = oracle_threads(raw, ped, gain, B, n_nb=n_nb, keep_corrected=True)
        got = run_pdc(ctx, raw, ped, gain, B, n_nb=n_nb, keep_corrected=True)
        assert want["total"] > 100
        assert_same(got, want, corrected=True)


def test_power_of_two_gains_and_gain_bits(ctx):
    """Gain bits 14-15 set in the raw words are ignored; gains of 2^j."""
    rng = np.random.default_rng(6)
    geom = synth.Geometry(1, 20, 96, 48)
    ped, _ = synth.make_calibration(geom, 3)
    gain = (2.0 ** rng.integers(-2, 3, size=geom.shape)).astype(np.float32)
    raw = synth.make_frames(geom, ped, gain, 3, 0.05, 3)
    raw |= (rng.integers(0, 4, size=raw.shape).astype(np.uint16) << 14)
    want = oracle_threads(raw, ped, gain, geom.bank_cols, keep_corrected=True)
    got = run_pdc(ctx, raw, ped, gain, geom.bank_cols, keep_corrected=True)
    assert_same(got, want, corrected=True)


def test_empty_batch(ctx):
    geom = synth.Geometry(1, 8, 16, 8)
    ped, gain = synth.make_calibration(geom, 1)
    raw = np.zeros((0, *geom.shape), np.uint16)
    import torch

    fz = torch.zeros(1, dtype=torch.int16, device="cuda")
    torch.cuda.synchronize()
    got = run_pdc(ctx, raw, ped, gain, 8, frames_dev=fz)
    assert got["total"] == 0 and len(got["hits"]) == 0


def test_dark_frames_no_hits(ctx):
    """Noise truncated below 2.5 sigma: no pixel exceeds a 5 sigma seed."""
    rng = np.random.default_rng(8)
    T, H, W, B = 2, 40, 96, 48
    ped = rng.normal(1500, 50, size=(T, H, W)).round().astype(np.float32)
    gain = np.ones((T, H, W), np.float32)
    noise = np.clip(rng.normal(0, 3, size=(6, T, H, W)), -7.4, 7.4)
    cm = rng.normal(0, 10, size=(6, T, H, W // B)).repeat(B, axis=3)
    raw = np.rint(ped[None] + cm + noise).astype(np.uint16)
    got = run_pdc(ctx, raw, ped, gain, B)
    assert got["total"] == 0


def test_overflow_recompute_and_truncation(ctx):
    """A hit capacity of 0 forces the staging pool to overflow; the batch is
    recomputed with exact sizes and still matches.  A small destination gets
    the first hits in raster order and a truncation status."""
    import torch

    from paper_1903_06838_amd import pdc

    geom = synth.Geometry(2, 60, 194, 97)
    raw, ped, gain = _case(geom, 0.08, 6, 9)
    want = oracle_threads(raw, ped, gain, geom.bank_cols)
    got = run_pdc(ctx, raw, ped, gain, geom.bank_cols, hit_capacity=0)
    assert_same(got, want)

    det = pdc.calibrate(ctx, pdc.geometry(*geom.shape, geom.bank_cols), ped, gain, pdc.params())
    frames = torch.from_numpy(raw).cuda()
    b = pdc.process_frames(ctx, det, frames, raw.shape[0], 0, None)
    cap = want["total"] // 3
    hits, total, fh, fp, st = pdc.get_hits(ctx, b, raw.shape[0], capacity=cap)
    assert st == pdc.WARN_TRUNCATED and total == want["total"] and len(hits) == cap
    assert np.array_equal(hits_u32(hits), hits_u32(want["hits"][:cap]))
    # device destination
    dst = torch.zeros(want["total"] * 4, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    _, total2, _, _, st2 = pdc.get_hits(ctx, b, raw.shape[0], capacity=want["total"], dst_dev=dst)
    assert st2 == pdc.OK and total2 == want["total"]
    assert np.array_equal(dst.cpu().numpy().view(np.uint32).reshape(-1, 4), hits_u32(want["hits"]))
    pdc.release_batch(ctx, b)
    pdc.release_detector(ctx, det)


def test_streams_and_determinism(ctx):
    """Same batch on a side stream, twice: identical; each frame alone gives the
    same result as inside the batch."""
    import torch

    geom = synth.Geometry(4, 37, 388, 194)
    raw, ped, gain = _case(geom, 0.03, 5, 11)
    want = oracle_threads(raw, ped, gain, geom.bank_cols)
    s = torch.cuda.Stream()
    a = run_pdc(ctx, raw, ped, gain, geom.bank_cols, stream=s)
    b = run_pdc(ctx, raw, ped, gain, geom.bank_cols, stream=s)
    assert_same(a, want)
    assert_same(b, want)
    for i in (0, 3):
        one = run_pdc(ctx, raw[i:i + 1], ped, gain, geom.bank_cols)
        mine = want["hits"][want["hits"]["frame"] == i].copy()
        mine["frame"] = 0
        assert np.array_equal(hits_u32(one["hits"]), hits_u32(mine))


def test_two_detectors_one_context(ctx):
    from paper_1903_06838_amd import pdc
    import torch

    g1, g2 = synth.Geometry(1, 64, 192, 96), synth.Geometry(3, 30, 194, 97)
    r1, p1, k1 = _case(g1, 0.02, 2, 21)
    r2, p2, k2 = _case(g2, 0.02, 3, 22)
    d1 = pdc.calibrate(ctx, pdc.geometry(*g1.shape, 96), p1, k1, pdc.params())
    d2 = pdc.calibrate(ctx, pdc.geometry(*g2.shape, 97), p2, k2, pdc.params(n_seed=4.0))
    f1, f2 = torch.from_numpy(r1).cuda(), torch.from_numpy(r2).cuda()
    b1 = pdc.process_frames(ctx, d1, f1, 2, 10000, None)
    b2 = pdc.process_frames(ctx, d2, f2, 3, 10000, None)
    h2 = pdc.get_hits(ctx, b2, 3)
    h1 = pdc.get_hits(ctx, b1, 2)
    w1 = oracle_threads(r1, p1, k1, 96)
    w2 = oracle_threads(r2, p2, k2, 97, n_seed=4.0)
    assert np.array_equal(hits_u32(h1[0]), hits_u32(w1["hits"]))
    assert np.array_equal(hits_u32(h2[0]), hits_u32(w2["hits"]))
    for b in (b1, b2):
        pdc.release_batch(ctx, b)
    pdc.release_detector(ctx, d1)
    pdc.release_detector(ctx, d2)


@pytest.mark.parametrize("occ_id", [0, 1, 2], ids=lambda i: "occupancy_%g" % synth.CSPAD_OCCUPANCIES[i])
def test_cspad_full_batch(ctx, occ_id):
    """CSPAD-like 32 x 185 x 388, 194-pixel banks, 10,000 frames in one batch
    (64 distinct frames replicated on the device), at each occupancy the
    benchmark sweeps (0.001, 0.01, 0.05 photons per pixel; at 0.05 about 920 M
    hits).  Every frame's counts and photon totals, and every hit record of
    every frame, against the oracle's result for its pool frame: the records
    are written to device memory and compared there, one 64-frame replica of
    the pool at a time."""
    import torch

    from paper_1903_06838_amd import pdc

    geom = synth.CSPAD
    occ = synth.CSPAD_OCCUPANCIES[occ_id]
    P, N = 64, 10000
    print("full batch: occupancy %g, %d frames" % (occ, N), flush=True)
    ped, gain = synth.make_calibration(geom, 1)
    pool = synth.make_frames(geom, ped, gain, P, occ, 1, occ_id)
    want = oracle_threads(pool, ped, gain, geom.bank_cols)
    dpool = torch.from_numpy(pool).cuda()
    frames = torch.empty((N, *geom.shape), dtype=torch.int16, device="cuda")
    for i in range(0, N, P):
        n = min(P, N - i)
        frames[i:i + n].copy_(dpool[:n])
    torch.cuda.synchronize()  # torch's copies run on its stream, the library on the context's
    del dpool
    idx = np.arange(N) % P
    total_want = int(want["frame_hits"][idx].sum())
    det = pdc.calibrate(ctx, pdc.geometry(*geom.shape, geom.bank_cols), ped, gain, pdc.params())
    b = pdc.process_frames(ctx, det, frames, N, int(total_want * 1.05) + 1, None)
    recs = torch.empty((total_want + 1, 4), dtype=torch.int32, device="cuda")
    _, total, fh, fp, st = pdc.get_hits(ctx, b, N, capacity=total_want + 1, dst_dev=recs)
    pdc.release_batch(ctx, b)
    pdc.release_detector(ctx, det)
    del frames
    assert st == pdc.OK
    assert np.array_equal(fh, want["frame_hits"][idx])
    assert np.array_equal(fp, want["frame_photons"][idx])
    assert total == total_want
    # one replica of the pool: its hits with frame indices rebased, compared
    # record by record on the device
    ref = torch.from_numpy(hits_u32(want["hits"]).view(np.int32).copy()).cuda()
    pool_frame = ref[:, 0].clone()
    per = int(want["total"])
    for r, f0 in enumerate(range(0, N, P)):
        nf = min(P, N - f0)
        nh = int(want["frame_hits"][:nf].sum())
        got = recs[r * per:r * per + nh]
        exp = ref[:nh].clone()
        exp[:, 0] = pool_frame[:nh] + f0
        if not torch.equal(got, exp):
            bad = int(torch.nonzero(torch.any(got != exp, dim=1))[0, 0])
            raise AssertionError("replica %d (frames %d..): record %d is %s, want %s" % (
                r, f0, r * per + bad, got[bad].tolist(), exp[bad].tolist()))
    del recs


@pytest.fixture(scope="module")
def ctx_general():
    """A context whose batches all take the general kernel (PDC_FORCE_GENERAL=1)."""
    import os

    from paper_1903_06838_amd import pdc

    os.environ["PDC_FORCE_GENERAL"] = "1"
    try:
        c = pdc.create(0)
    finally:
        del os.environ["PDC_FORCE_GENERAL"]
    yield c
    pdc.destroy(c)


@pytest.mark.parametrize("geom", [synth.Geometry(2, 50, 388, 194), synth.Geometry(1, 64, 768, 96),
                                  synth.Geometry(3, 21, 256, 128), synth.Geometry(1, 40, 512, 256)],
                         ids=lambda g: "%dx%dx%d_B%d" % (g.n_tiles, g.rows, g.cols, g.bank_cols))
def test_general_and_persistent_kernels_agree(ctx, ctx_general, geom):
    """The same batch through the persistent kernel and the general kernel:
    both equal the oracle, corrected frames included."""
    raw, ped, gain = _case(geom, 0.03, 4, 31)
    want = oracle_threads(raw, ped, gain, geom.bank_cols, keep_corrected=True)
    assert_same(run_pdc(ctx, raw, ped, gain, geom.bank_cols, keep_corrected=True), want, corrected=True)
    assert_same(run_pdc(ctx_general, raw, ped, gain, geom.bank_cols, keep_corrected=True), want, corrected=True)


def test_flood_frame_falls_back_exactly(ctx):
    """A frame where a third of the pixels carry photons has more seed pixels per
    strip than the persistent kernel holds on chip; the batch is recomputed by
    the general kernel and still matches."""
    import torch

    from paper_1903_06838_amd import pdc

    geom = synth.Geometry(2, 60, 388, 194)
    ped, gain = synth.make_calibration(geom, 41)
    raw = synth.make_frames(geom, ped, gain, 2, 0.4, 41)
    raw = np.concatenate([raw, synth.make_frames(geom, ped, gain, 3, 0.01, 42)])  # flood and ordinary frames
    want = oracle_threads(raw, ped, gain, geom.bank_cols, keep_corrected=True)
    assert want["total"] > 1000
    det = pdc.calibrate(ctx, pdc.geometry(*geom.shape, 194), ped, gain, pdc.params(flags=pdc.KEEP_CORRECTED))
    try:
        b = pdc.process_frames(ctx, det, torch.from_numpy(raw).cuda(), raw.shape[0], 1 << 14)
        hits, total, fh, fp, _ = pdc.get_hits(ctx, b, raw.shape[0])
        corr = np.empty(raw.shape, np.float32)
        pdc.get_corrected(ctx, b, corr)
        # only the flood frames' strips are redone by the general kernel
        assert pdc.debug_batch_path(ctx, b) == 3
        pdc.release_batch(ctx, b)
    finally:
        pdc.release_detector(ctx, det)
    assert_same(dict(hits=hits, total=total, frame_hits=fh, frame_photons=fp, corrected=corr), want,
                corrected=True)


def test_strips_across_tile_edges(ctx):
    """Two 40-row tiles are cut into strips of 26-27 rows, so one strip holds
    rows of both tiles: photons on either side of the edge, in the same and
    adjacent columns, are not neighbours (each tile's pixel is its own hit),
    and a flood frame makes that strip overflow its seed list, so the general
    kernel redoes it, edge included.  Every result matches the oracle."""
    import torch

    from paper_1903_06838_amd import pdc

    geom = synth.Geometry(2, 40, 388, 194)
    ped, gain = synth.make_calibration(geom, 51)
    raw = synth.make_frames(geom, ped, gain, 4, 0.01, 51)
    for c in range(3, 380, 9):  # tile 0's last row against tile 1's first row
        raw[:2, 0, 39, c] = np.minimum(raw[:2, 0, 39, c].astype(np.int32) + 900, 0x3FFF)
        raw[:2, 1, 0, c + (c % 2)] = np.minimum(raw[:2, 1, 0, c + (c % 2)].astype(np.int32) + 1500, 0x3FFF)
    raw = np.concatenate([raw, synth.make_frames(geom, ped, gain, 1, 0.45, 52)])
    want = oracle_threads(raw, ped, gain, 194, keep_corrected=True)
    h = want["hits"]
    edge = h[(h["frame"] < 2) & (((h["pixel"] // 388) == 39) | ((h["pixel"] // 388) == 40))]
    assert len(edge) >= 80  # both sides of the edge hold hits in the same columns
    det = pdc.calibrate(ctx, pdc.geometry(*geom.shape, 194), ped, gain, pdc.params(flags=pdc.KEEP_CORRECTED))
    try:
        b = pdc.process_frames(ctx, det, torch.from_numpy(raw).cuda(), raw.shape[0], 1 << 16)
        hits, total, fh, fp, _ = pdc.get_hits(ctx, b, raw.shape[0])
        corr = np.empty(raw.shape, np.float32)
        pdc.get_corrected(ctx, b, corr)
        assert pdc.debug_batch_path(ctx, b) == 3
        pdc.release_batch(ctx, b)
    finally:
        pdc.release_detector(ctx, det)
    assert_same(dict(hits=hits, total=total, frame_hits=fh, frame_photons=fp, corrected=corr), want,
                corrected=True)


def test_median_with_outliers_and_plateaus(ctx):
    """Banks whose median sits on a long run of equal values, banks with far
    outliers on one side, and banks of identical values."""
    rng = np.random.default_rng(12)
    T, H, W, B = 1, 24, 388, 194
    ped = np.full((T, H, W), 1000.0, np.float32)
    gain = np.ones((T, H, W), np.float32)
    raw = np.full((3, T, H, W), 1000, np.int64)
    raw[0, 0, :8] += rng.integers(0, 3, size=(8, W))            # plateaus of 0/1/2
    raw[0, 0, 8:16] += rng.integers(0, 2, size=(8, W)) * 9000   # two far clusters
    raw[1, 0, :, :97] += 15000 - 1000                            # one side saturates
    raw[2] += rng.integers(-3, 4, size=(T, H, W))
    raw[2, 0, 5, 10:20] += 300
    raw = np.clip(raw, 0, 16383).astype(np.uint16)
    want = oracle_threads(raw, ped, gain, B, keep_corrected=True)
    assert_same(run_pdc(ctx, raw, ped, gain, B, keep_corrected=True), want, corrected=True)


def test_median_brackets_straddling_zero(ctx):
    """Banks whose values spread widely on both sides of zero (and whose lane
    estimate is pulled away by bright pixels), so the median search widens its
    bracket across zero before converging."""
    rng = np.random.default_rng(21)
    T, H, W, B = 2, 30, 388, 194
    ped = np.full((T, H, W), 2000.0, np.float32)
    gain = rng.uniform(0.95, 1.05, size=(T, H, W)).astype(np.float32)
    raw = 2000 + rng.normal(0, 40, size=(4, T, H, W))
    hot = rng.random(size=raw.shape) < 0.15
    raw[hot] += 400
    raw = np.clip(np.rint(raw), 0, 16383).astype(np.uint16)
    want = oracle_threads(raw, ped, gain, B, keep_corrected=True)
    assert_same(run_pdc(ctx, raw, ped, gain, B, keep_corrected=True), want, corrected=True)
    eg = synth.Geometry(1, 40, 768, 96)
    rawe = np.clip(np.rint(2000 + rng.normal(0, 40, size=(4, *eg.shape))
                           + (rng.random(size=(4, *eg.shape)) < 0.15) * 400), 0, 16383).astype(np.uint16)
    pe = np.full(eg.shape, 2000.0, np.float32)
    ge = rng.uniform(0.95, 1.05, size=eg.shape).astype(np.float32)
    want = oracle_threads(rawe, pe, ge, 96, keep_corrected=True)
    assert_same(run_pdc(ctx, rawe, pe, ge, 96, keep_corrected=True), want, corrected=True)


def test_autotune_keeps_results(ctx):
    """The frame-group autotuner picks one of its multipliers and the batches
    after it still equal the oracle bit for bit."""
    import torch

    from paper_1903_06838_amd import pdc

    geom = synth.Geometry(2, 40, 388, 194)
    raw, ped, gain = _case(geom, 0.02, 64, 51)
    want = oracle_threads(raw, ped, gain, geom.bank_cols)
    det = pdc.calibrate(ctx, pdc.geometry(*geom.shape, 194), ped, gain, pdc.params())
    try:
        dev = torch.from_numpy(raw).cuda()
        mult, ms = pdc.autotune(ctx, det, dev, raw.shape[0], 1 << 16)
        assert mult in (1, 2, 4) and np.all(ms > 0)
        b = pdc.process_frames(ctx, det, dev, raw.shape[0], 1 << 16)
        hits, total, fh, fp, _ = pdc.get_hits(ctx, b, raw.shape[0])
        pdc.release_batch(ctx, b)
    finally:
        pdc.release_detector(ctx, det)
    assert_same(dict(hits=hits, total=total, frame_hits=fh, frame_photons=fp), want)


def test_strip_heights_keep_results(ctx):
    """The strip-height autotuner times three strip heights and keeps one;
    batches with each height (forced at pdc_create) and after the tuner equal
    the oracle bit for bit; the tuner refuses while a batch is outstanding."""
    import os

    import torch

    from paper_1903_06838_amd import pdc

    geom = synth.Geometry(2, 40, 388, 194)
    raw, ped, gain = _case(geom, 0.02, 24, 53)
    want = oracle_threads(raw, ped, gain, geom.bank_cols)
    dev = torch.from_numpy(raw).cuda()
    torch.cuda.synchronize()
    det = pdc.calibrate(ctx, pdc.geometry(*geom.shape, 194), ped, gain, pdc.params())
    try:
        b = pdc.process_frames(ctx, det, dev, raw.shape[0], 1 << 16)
        with pytest.raises(pdc.PdcError) as e:
            pdc.autotune_strips(ctx, det, dev, raw.shape[0], 1 << 16)
        assert e.value.status == pdc.ESTATE
        pdc.release_batch(ctx, b)
        rows, mult, ms = pdc.autotune_strips(ctx, det, dev, raw.shape[0], 1 << 16)
        assert rows in (30, 26, 22) and mult in (1, 2, 4) and ms.shape == (3, 3) and np.all(ms > 0)
        b = pdc.process_frames(ctx, det, dev, raw.shape[0], 1 << 16)
        hits, total, fh, fp, _ = pdc.get_hits(ctx, b, raw.shape[0])
        assert pdc.debug_batch_path(ctx, b) in (2, 3)
        pdc.release_batch(ctx, b)
    finally:
        pdc.release_detector(ctx, det)
    assert_same(dict(hits=hits, total=total, frame_hits=fh, frame_photons=fp), want)
    for r in (26, 22, 5):
        os.environ["PDC_STRIP_ROWS"] = str(r)
        try:
            c = pdc.create(0)
        finally:
            del os.environ["PDC_STRIP_ROWS"]
        try:
            d = pdc.calibrate(c, pdc.geometry(*geom.shape, 194), ped, gain, pdc.params())
            b = pdc.process_frames(c, d, dev, raw.shape[0], 1 << 16)
            hits, total, fh, fp, _ = pdc.get_hits(c, b, raw.shape[0])
            assert pdc.debug_batch_path(c, b) in (2, 3), r
            pdc.release_batch(c, b)
            pdc.release_detector(c, d)
        finally:
            pdc.destroy(c)
        assert_same(dict(hits=hits, total=total, frame_hits=fh, frame_photons=fp), want)
