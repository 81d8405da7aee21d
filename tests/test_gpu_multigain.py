"""Auto-ranging (multi-gain) detectors on the GPU through the C ABI against
oracle/multigain.py, bit for bit: hit lists, per-frame counts, photon totals,
Frames2 and per-frame invalid-code counts, for both gain-code tables, the
median and thresholded-mean common modes, on the persistent and general
kernels."""
import os

import numpy as np
import pytest

from oracle import multigain as G
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


def _run(ctx, raw, ped, gain, bank_cols, gain_mode, cm_mode=0, stages=1, keep=True):
    import torch

    from paper_1903_06838_amd import pdc

    N, T, H, W = raw.shape
    prm = pdc.params(3.0, 5.0, 3.0, 150.0, pdc.KEEP_CORRECTED if keep else 0, cm_mode=cm_mode, cm_stages=stages)
    det = pdc.calibrate(ctx, pdc.geometry(T, H, W, bank_cols, gain_mode), ped, gain, prm)
    try:
        b = pdc.process_frames(ctx, det, torch.from_numpy(raw).cuda(), N, max(1024, raw.size // 10))
        hits, total, fh, fp, _ = pdc.get_hits(ctx, b, N)
        out = dict(hits=hits, total=total, frame_hits=fh, frame_photons=fp, path=pdc.debug_batch_path(ctx, b),
                   invalid=pdc.get_invalid_counts(ctx, b, N))
        if keep:
            corr = np.empty(raw.shape, np.float32)
            pdc.get_corrected(ctx, b, corr)
            out["corrected"] = corr
        pdc.release_batch(ctx, b)
    finally:
        pdc.release_detector(ctx, det)
    return out


def _case(geom, gain_mode, n, occ, seed, **kw):
    ped, gain = synth.make_calibration_multigain(geom, seed)
    raw = synth.make_frames_multigain(geom, ped, gain, n, occ, seed, gain_mode, **kw)
    return raw, ped, gain


CASES = [
    # geometry, gain_mode, cm_mode, stages, occupancy, frames, kernel (2 persistent, 1 general)
    (synth.Geometry(1, 64, 384, 96), 1, 0, 1, 0.02, 3, 2),       # ePix10k-like, 8 lanes per bank
    (synth.Geometry(1, 48, 1024, 256), 2, 0, 1, 0.02, 3, 2),     # Jungfrau-like
    (synth.Geometry(2, 40, 388, 194), 1, 0, 1, 0.03, 3, 2),
    (synth.Geometry(2, 40, 388, 194), 2, 1, 3, 0.02, 3, 2),      # bank mean, 3 stages
    (synth.Geometry(1, 64, 384, 96), 1, 2, 2, 0.02, 3, 2),       # tile mean (small bank offsets)
    (synth.Geometry(1, 24, 1024, 512), 2, 0, 1, 0.02, 2, 1),     # banks beyond the persistent kernel
]
# The thresholded mean is pulled far down by the noisy low-gain pixels, so
# the mean-mode cases use fewer of them: with 20 % of pixels in the lower
# ranges their seeds overflow the persistent kernel's on-chip lists and the
# batch is recomputed on the general kernel (still bit-exact).  With 1.1 % the
# oracle's busiest 27-row strip of the bank-mean case holds about 2,200 seeds,
# inside the list (about 2,700 for that strip height).
FEW_LOW_GAIN = dict(range_frac=(0.985, 0.008, 0.003), invalid_frac=0.01)


@pytest.mark.parametrize("geom,gm,cm,stages,occ,n,path", CASES, ids=lambda x: str(x))
def test_multigain_parity(ctx, geom, gm, cm, stages, occ, n, path):
    kw = dict(FEW_LOW_GAIN) if cm else {}
    if cm == 2:  # a tile's mean cannot follow per-bank offsets: keep them small
        kw["sim"] = synth.SimParams(cm_sigma=1.0)
    raw, ped, gain = _case(geom, gm, n, occ, 31, **kw)
    want = G.process(raw, ped, gain, geom.bank_cols, gm, cm, stages, keep_corrected=True)
    got = _run(ctx, raw, ped, gain, geom.bank_cols, gm, cm, stages)
    assert got["path"] == path
    assert want["total"] > 0 and want["invalid"].sum() > 0
    assert np.array_equal(got["invalid"], want["invalid"])
    assert_same(got, want, corrected=True)


def test_mean_mode_overflow_falls_back_bit_exact(ctx):
    """Many low-gain pixels under the thresholded mean: seed lists overflow,
    the general kernel redoes those strip-frames (with the mean pass, which
    the persistent kernel had computed inline) and the results are exact."""
    geom = synth.Geometry(2, 40, 388, 194)
    raw, ped, gain = _case(geom, 2, 3, 0.02, 31)
    want = G.process(raw, ped, gain, 194, 2, 1, 3, keep_corrected=True)
    got = _run(ctx, raw, ped, gain, 194, 2, 1, 3)
    assert got["path"] == 3
    assert np.array_equal(got["invalid"], want["invalid"])
    assert_same(got, want, corrected=True)


@pytest.mark.parametrize("cm", [0, 1])
def test_mostly_invalid_banks(ctx, cm):
    """90 % invalid codes on 8-pixel banks: many banks with one or no valid
    pixel (median 0, all Frames2 zero)."""
    geom = synth.Geometry(2, 20, 64, 8)
    raw, ped, gain = _case(geom, 1, 3, 0.05, 32, range_frac=(0.05, 0.03, 0.02), invalid_frac=0.9)
    r, _ = G.decode(raw, 1)
    assert np.any(np.all(r.reshape(3, 2, 20, 8, 8) < 0, axis=-1))
    want = G.process(raw, ped, gain, 8, 1, cm, 2, keep_corrected=True)
    got = _run(ctx, raw, ped, gain, 8, 1, cm, 2)
    assert np.array_equal(got["invalid"], want["invalid"])
    assert_same(got, want, corrected=True)


def test_multigain_general_kernel():
    import torch

    from paper_1903_06838_amd import pdc

    assert torch.cuda.is_available()
    geom = synth.Geometry(2, 40, 388, 194)
    raw, ped, gain = _case(geom, 2, 3, 0.02, 33)
    os.environ["PDC_FORCE_GENERAL"] = "1"
    try:
        c = pdc.create(0)
    finally:
        del os.environ["PDC_FORCE_GENERAL"]
    try:
        for cm, st in ((0, 1), (2, 3)):
            want = G.process(raw, ped, gain, 194, 2, cm, st, keep_corrected=True)
            got = _run(c, raw, ped, gain, 194, 2, cm, st)
            assert got["path"] == 1
            assert np.array_equal(got["invalid"], want["invalid"])
            assert_same(got, want, corrected=True)
    finally:
        pdc.destroy(c)


def test_single_range_reports_no_invalid_and_bad_modes(ctx):
    from paper_1903_06838_amd import pdc

    geom = synth.Geometry(1, 16, 32, 16)
    ped, gain = synth.make_calibration(geom, 34)
    raw = synth.make_frames(geom, ped, gain, 2, 0.02, 34)
    raw[:, 0, 0, :4] |= np.uint16(0xC000)  # gain bits are ignored in single-range mode
    got = _run(ctx, raw, ped, gain, 16, 0, keep=False)
    assert got["invalid"].tolist() == [0, 0]
    g = pdc.geometry(1, 16, 32, 16, 3)
    with pytest.raises(pdc.PdcError) as e:
        pdc.calibrate(ctx, g, np.stack([ped] * 3), np.stack([gain] * 3), pdc.params())
    assert e.value.status == pdc.EINVAL
    with pytest.raises(ValueError):  # one plane where three are needed
        pdc.calibrate(ctx, pdc.geometry(1, 16, 32, 16, 1), ped, gain, pdc.params())
