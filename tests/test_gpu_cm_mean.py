"""Thresholded-mean common mode (Fig. c, stacked stages) on the GPU through the
C ABI against oracle/cm_mean.py, bit for bit: hit lists, per-frame counts and
photon totals, and Frames2, for bank and tile regions, 1 to 3 stages, on the
persistent kernel (both lane layouts) and the general kernel.  The oracle's
sum is the exact sum rounded once, so these also check that no order of
summation shows through."""
import os

import numpy as np
import pytest

from oracle import cm_mean as M
from paper_1903_06838_amd import synth
from tests.helpers import assert_same

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1903_06838_amd import pdc

    c = pdc.create(0)
    yield c
    pdc.destroy(c)


def _run(ctx, raw, ped, gain, bank_cols, mode, stages, keep=True, n_cm=3.0):
    import torch

    from paper_1903_06838_amd import pdc

    N, T, H, W = raw.shape
    prm = pdc.params(3.0, 5.0, 3.0, 150.0, pdc.KEEP_CORRECTED if keep else 0, cm_mode=mode, cm_stages=stages,
                     n_cm=n_cm)
    det = pdc.calibrate(ctx, pdc.geometry(T, H, W, bank_cols), ped, gain, prm)
    try:
        b = pdc.process_frames(ctx, det, torch.from_numpy(raw).cuda(), N, max(1024, raw.size // 10))
        hits, total, fh, fp, _ = pdc.get_hits(ctx, b, N)
        out = dict(hits=hits, total=total, frame_hits=fh, frame_photons=fp, path=pdc.debug_batch_path(ctx, b))
        if keep:
            corr = np.empty(raw.shape, np.float32)
            pdc.get_corrected(ctx, b, corr)
            out["corrected"] = corr
        pdc.release_batch(ctx, b)
    finally:
        pdc.release_detector(ctx, det)
    return out


CASES = [
    # geometry, occupancy, frames, region, stages
    (synth.Geometry(2, 40, 388, 194), 0.02, 5, M.BANK, 1),
    (synth.Geometry(2, 40, 388, 194), 0.02, 5, M.BANK, 3),
    (synth.Geometry(2, 40, 388, 194), 0.02, 4, M.TILE, 3),
    (synth.Geometry(1, 64, 768, 96), 0.02, 3, M.BANK, 2),    # ePix100-like rows, 8 lanes per bank
    (synth.Geometry(1, 64, 768, 96), 0.05, 3, M.TILE, 3),
    (synth.Geometry(1, 24, 1024, 512), 0.02, 3, M.BANK, 3),  # banks beyond the persistent kernel
    (synth.Geometry(3, 17, 40, 8), 0.03, 7, M.BANK, 3),      # small banks, ragged strips
    (synth.Geometry(1, 9, 2048, 1), 0.05, 1, M.BANK, 2),     # one-pixel banks
    (synth.Geometry(1, 33, 2048, 128), 0.01, 2, M.TILE, 1),
    (synth.Geometry(1, 1, 1, 1), 0.5, 3, M.TILE, 3),
    (synth.Geometry(2, 12, 96, 48), 0.03, 37, M.BANK, 3),    # several frame groups and a ragged one
    (synth.Geometry(2, 12, 96, 48), 0.03, 19, M.TILE, 2),
    (synth.Geometry(1, 200, 512, 128), 0.02, 2, M.TILE, 3),  # a tile beyond one workgroup's LDS: a pass per stage
]


@pytest.mark.parametrize("geom,occ,n,region,stages", CASES, ids=lambda x: str(x))
def test_cm_mean_parity(ctx, geom, occ, n, region, stages):
    # a tile's mean cannot follow per-bank offsets: with the default 10 ADU
    # offsets about a third of the pixels become seeds and the busiest strips
    # overflow their lists (that case has its own test below), so the tile
    # cases that check for the persistent kernel keep the offsets small
    small = region == M.TILE and geom.bank_cols in (194, 96)
    sim = synth.SimParams(cm_sigma=1.0) if small else synth.SimParams()
    ped, gain = synth.make_calibration(geom, 21)
    raw = synth.make_frames(geom, ped, gain, n, occ, 21, sim=sim)
    want = M.process(raw, ped, gain, geom.bank_cols, region, stages, keep_corrected=True)
    got = _run(ctx, raw, ped, gain, geom.bank_cols, region, stages)
    assert want["total"] > 0
    if geom.bank_cols in (194, 96):
        assert got["path"] == 2  # the persistent kernel
    assert_same(got, want, corrected=True)


def test_tile_mean_overflow_redoes_units(ctx):
    """Large per-bank offsets that a tile's mean cannot follow leave many
    pixels above threshold: strip-frames whose seed lists overflow are redone
    by the general kernel from the pass's values, bit for bit."""
    geom = synth.Geometry(2, 60, 388, 194)
    ped, gain = synth.make_calibration(geom, 25)
    raw = synth.make_frames(geom, ped, gain, 3, 0.01, 25, sim=synth.SimParams(cm_sigma=50.0))
    want = M.process(raw, ped, gain, 194, M.TILE, 2, keep_corrected=True)
    got = _run(ctx, raw, ped, gain, 194, M.TILE, 2)
    assert got["path"] == 3
    assert_same(got, want, corrected=True)


@pytest.mark.parametrize("region", [M.BANK, M.TILE])
def test_cm_mean_wide_window(ctx, region):
    """One pixel's dark of 2^-60 gives its Frames1 bits far below the ADC's
    unit (raw 0 there makes a tiny negative noise value), which widens every
    sum's window past two binary64 limbs: the separate pass takes the general
    way (unit 2^-149), and with bank regions the persistent kernel hands its
    units to the general kernel, which reads the pass's values."""
    geom = synth.Geometry(2, 40, 388, 194)
    ped, gain = synth.make_calibration(geom, 26)
    ped[0, 3, 5] = 2.0 ** -60
    ped[1, 30, 200] = -(2.0 ** -40)
    sim = synth.SimParams(cm_sigma=1.0) if region == M.TILE else synth.SimParams()
    raw = synth.make_frames(geom, ped, gain, 3, 0.02, 26, sim=sim)
    raw[1, 0, 3, 5] = 0
    raw[2, 1, 30, 200] = 0
    want = M.process(raw, ped, gain, 194, region, 3, keep_corrected=True)
    got = _run(ctx, raw, ped, gain, 194, region, 3)
    if region == M.BANK:
        assert got["path"] == 3  # every unit redone by the general kernel
    assert_same(got, want, corrected=True)


def test_cm_mean_guard_at_high_occupancy(ctx):
    """At 1.5 photons per pixel most banks have fewer noise pixels than
    sqrt(bank_cols): the guard sets the denominator."""
    geom = synth.Geometry(1, 32, 388, 194)
    ped, gain = synth.make_calibration(geom, 22)
    raw = synth.make_frames(geom, ped, gain, 3, 1.5, 22)
    from oracle import oracle as C

    f1 = C.load().dark_gain(raw[0], ped, gain)
    _, n0 = M.region_cm(M._regions(f1, M.BANK, 194), np.float32(9.0))
    assert np.count_nonzero(n0 < np.sqrt(194)) > 5
    want = M.process(raw, ped, gain, 194, M.BANK, 3, keep_corrected=True)
    got = _run(ctx, raw, ped, gain, 194, M.BANK, 3)
    assert_same(got, want, corrected=True)


def test_cm_mean_general_kernel():
    """A context whose batches take the general kernel gives the same bits."""
    import torch

    from paper_1903_06838_amd import pdc

    assert torch.cuda.is_available()
    geom = synth.Geometry(2, 40, 388, 194)
    ped, gain = synth.make_calibration(geom, 23)
    raw = synth.make_frames(geom, ped, gain, 4, 0.02, 23)
    want = M.process(raw, ped, gain, 194, M.BANK, 3, keep_corrected=True)
    os.environ["PDC_FORCE_GENERAL"] = "1"
    try:
        c = pdc.create(0)
    finally:
        del os.environ["PDC_FORCE_GENERAL"]
    try:
        got = _run(c, raw, ped, gain, 194, M.BANK, 3)
        got_t = _run(c, raw, ped, gain, 194, M.TILE, 2)
    finally:
        pdc.destroy(c)
    assert got["path"] == got_t["path"] == 1
    assert_same(got, want, corrected=True)
    assert_same(got_t, M.process(raw, ped, gain, 194, M.TILE, 2, keep_corrected=True), corrected=True)


def test_cm_mean_without_keep_and_bad_params(ctx):
    from paper_1903_06838_amd import pdc

    geom = synth.Geometry(1, 40, 388, 194)
    ped, gain = synth.make_calibration(geom, 24)
    raw = synth.make_frames(geom, ped, gain, 6, 0.02, 24)
    want = M.process(raw, ped, gain, 194, M.BANK, 2)
    got = _run(ctx, raw, ped, gain, 194, M.BANK, 2, keep=False)
    assert_same(got, want)
    g = pdc.geometry(*geom.shape, 194)
    for kw in (dict(cm_mode=3), dict(cm_mode=1, cm_stages=0), dict(cm_mode=2, cm_stages=4),
               dict(cm_mode=1, n_cm=-1.0), dict(cm_mode=1, n_cm=float("nan"))):
        with pytest.raises(pdc.PdcError) as e:
            pdc.calibrate(ctx, g, ped, gain, pdc.params(**kw))
        assert e.value.status == pdc.EINVAL, kw
