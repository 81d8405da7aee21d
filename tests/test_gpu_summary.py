"""Summaries on the GPU (through the C ABI) against oracle/summary.py, bit for
bit: photon-count maps and charge spectra accumulated over batches, spectra
split by cloud size, histograms of Frames2, and pedestal/noise from darks."""
import numpy as np
import pytest

from oracle import summary as S
from paper_1903_06838_amd import synth
from tests.helpers import oracle_threads

pytestmark = pytest.mark.gpu

T_NB = 9.0


@pytest.fixture(scope="module")
def ctx():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1903_06838_amd import pdc

    c = pdc.create(0)
    yield c
    pdc.destroy(c)


def _zeros(n):
    import torch

    t = torch.zeros(n, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()  # torch fills on its stream, the library runs on its own
    return t


def _host(t):
    import torch

    torch.cuda.synchronize()
    return t.cpu().numpy().view(np.uint32)


def _batches(ctx, geom, raw, ped, gain, keep, cuts):
    import torch

    from paper_1903_06838_amd import pdc

    prm = pdc.params(3.0, 5.0, 3.0, 150.0, pdc.KEEP_CORRECTED if keep else 0)
    det = pdc.calibrate(ctx, pdc.geometry(*geom.shape, geom.bank_cols), ped, gain, prm)
    dev = torch.from_numpy(raw).cuda()
    out = []
    for a, b in zip(cuts[:-1], cuts[1:]):
        out.append(pdc.process_frames(ctx, det, dev[a:b], b - a, 1 << 16))
    return det, dev, out


@pytest.mark.parametrize("nbins", [300, 20000])
def test_accumulate_hits(ctx, nbins):
    """Two batches accumulated into one map and spectra equal the oracle's over
    all frames; 300 bins are gathered in LDS, 20000 go straight to memory."""
    from paper_1903_06838_amd import pdc

    geom = synth.Geometry(2, 40, 388, 194)
    ped, gain = synth.make_calibration(geom, 5)
    raw = synth.make_frames(geom, ped, gain, 9, 0.03, 5)
    want = oracle_threads(raw, ped, gain, geom.bank_cols, keep_corrected=True)
    assert want["total"] > 2000
    lo, hi = -20.0, 280.0
    cmap, spec, sizes = _zeros(geom.pixels), _zeros(nbins + 2), _zeros(9 * (nbins + 2))
    det, dev, bs = _batches(ctx, geom, raw, ped, gain, True, [0, 4, 9])
    try:
        for b in bs:
            pdc.accumulate_hits(ctx, b, cmap, spec, sizes, lo, hi, nbins)
        for b in bs:
            pdc.release_batch(ctx, b)
    finally:
        pdc.release_detector(ctx, det)
    h = want["hits"]
    assert np.array_equal(_host(cmap), S.count_map(h, geom.pixels))
    assert np.array_equal(_host(spec), S.histogram(h["charge"], lo, hi, nbins))
    got = _host(sizes).reshape(9, nbins + 2)
    assert np.array_equal(got, S.size_spectra(want["corrected"], h, T_NB, lo, hi, nbins))
    assert got.sum() == want["total"] and got[1].sum() > 0 and got[2].sum() > 0


def test_size_spectra_many_sparse_frames(ctx):
    """600 small frames at about one photon each, many with no hit at all: the
    frame of each hit is found across runs of empty frames."""
    from paper_1903_06838_amd import pdc

    geom = synth.Geometry(1, 16, 32, 16)
    ped, gain = synth.make_calibration(geom, 12)
    raw = synth.make_frames(geom, ped, gain, 600, 0.002, 12)
    raw[200:450] = synth.make_frames(geom, ped, gain, 250, 0.0, 12, occ_id=3)  # 250 frames without photons
    want = oracle_threads(raw, ped, gain, geom.bank_cols, keep_corrected=True)
    assert np.count_nonzero(want["frame_hits"] == 0) > 300 and want["total"] > 100
    nb = 50
    sizes = _zeros(9 * (nb + 2))
    det, dev, bs = _batches(ctx, geom, raw, ped, gain, True, [0, 600])
    try:
        pdc.accumulate_hits(ctx, bs[0], None, None, sizes, 0.0, 300.0, nb)
        pdc.release_batch(ctx, bs[0])
    finally:
        pdc.release_detector(ctx, det)
    got = _host(sizes).reshape(9, nb + 2)
    assert np.array_equal(got, S.size_spectra(want["corrected"], want["hits"], T_NB, 0.0, 300.0, nb))


def test_accumulate_map_only_without_keep(ctx):
    from paper_1903_06838_amd import pdc

    geom = synth.EPIX100
    ped, gain = synth.make_calibration(geom, 6)
    raw = synth.make_frames(geom, ped, gain, 5, 0.02, 6)
    want = oracle_threads(raw, ped, gain, geom.bank_cols)
    cmap, spec = _zeros(geom.pixels), _zeros(1000 + 2)
    det, dev, bs = _batches(ctx, geom, raw, ped, gain, False, [0, 5])
    try:
        pdc.accumulate_hits(ctx, bs[0], cmap, spec, None, 0.0, 1000.0, 1000)
        with pytest.raises(pdc.PdcError) as e:  # size spectra need Frames2
            pdc.accumulate_hits(ctx, bs[0], None, None, _zeros(9 * 12), 0.0, 1.0, 10)
        assert e.value.status == pdc.ESTATE
        pdc.release_batch(ctx, bs[0])
    finally:
        pdc.release_detector(ctx, det)
    assert np.array_equal(_host(cmap), S.count_map(want["hits"], geom.pixels))
    assert np.array_equal(_host(spec), S.histogram(want["hits"]["charge"], 0.0, 1000.0, 1000))


@pytest.mark.parametrize("geom,n,nbins", [
    (synth.Geometry(1, 5, 9, 3), 3, 64),          # 135 values: a ragged tail of 3
    (synth.Geometry(2, 40, 388, 194), 6, 1000),
    (synth.Geometry(2, 40, 388, 194), 2, 13000),  # bins beyond LDS
])
def test_histogram_corrected(ctx, geom, n, nbins):
    from paper_1903_06838_amd import pdc

    ped, gain = synth.make_calibration(geom, 7)
    raw = synth.make_frames(geom, ped, gain, n, 0.02, 7)
    want = oracle_threads(raw, ped, gain, geom.bank_cols, keep_corrected=True)
    lo, hi = -10.0, 170.0
    hist = _zeros(nbins + 2)
    det, dev, bs = _batches(ctx, geom, raw, ped, gain, True, [0, n])
    try:
        pdc.histogram_corrected(ctx, bs[0], hist, lo, hi, nbins)
        pdc.histogram_corrected(ctx, bs[0], hist, lo, hi, nbins)  # accumulates
        pdc.release_batch(ctx, bs[0])
    finally:
        pdc.release_detector(ctx, det)
    one = S.histogram(want["corrected"], lo, hi, nbins)
    assert np.array_equal(_host(hist), 2 * one)
    assert one.sum() == raw.size
    if raw.size > 1000:
        assert one[0] > 0 and one[-1] > 0


def test_histogram_needs_keep_and_valid_bins(ctx):
    from paper_1903_06838_amd import pdc

    geom = synth.Geometry(1, 8, 16, 8)
    ped, gain = synth.make_calibration(geom, 8)
    raw = synth.make_frames(geom, ped, gain, 2, 0.02, 8)
    h = _zeros(16)
    for keep in (False, True):
        det, dev, bs = _batches(ctx, geom, raw, ped, gain, keep, [0, 2])
        try:
            if not keep:
                with pytest.raises(pdc.PdcError) as e:
                    pdc.histogram_corrected(ctx, bs[0], h, 0.0, 1.0, 10)
                assert e.value.status == pdc.ESTATE
            else:
                for lo, hi, nb in [(0.0, 1.0, 0), (1.0, 1.0, 4), (2.0, 1.0, 4), (0.0, float("inf"), 4),
                                   (-3e38, 3e38, 4), (0.0, 1e-38, 1 << 24)]:
                    with pytest.raises(pdc.PdcError) as e:
                        pdc.histogram_corrected(ctx, bs[0], h, lo, hi, nb)
                    assert e.value.status == pdc.EINVAL, (lo, hi, nb)
            pdc.release_batch(ctx, bs[0])
        finally:
            pdc.release_detector(ctx, det)


@pytest.mark.parametrize("geom,n", [
    (synth.EPIX100, 50),                    # 4 pixels a thread, 2 frame chunks
    (synth.Geometry(1, 7, 9, 3), 33),       # 63 pixels: one pixel a thread
])
def test_dark_stats(ctx, geom, n):
    import torch

    from paper_1903_06838_amd import pdc

    ped, gain = synth.make_calibration(geom, 9)
    darks = synth.make_frames(geom, ped, gain, n, 0.0, 9)
    darks[1::3] |= np.uint16(0xC000)  # gain bits are ignored
    g = pdc.geometry(*geom.shape, geom.bank_cols)
    p, s = pdc.dark_stats(ctx, g, torch.from_numpy(darks).cuda(), n)
    wp, ws = S.dark_stats(darks)
    assert np.array_equal(p.view(np.uint32), wp.view(np.uint32))
    assert np.array_equal(s.view(np.uint32), ws.view(np.uint32))


def test_dark_stats_long_run_at_full_scale(ctx):
    """2^18 + 5 frames of 8 pixels near the ADC maximum: S1 beyond 2^32 and S2
    near 2^46, summed over many frame chunks."""
    import torch

    from paper_1903_06838_amd import pdc

    n = (1 << 18) + 5
    rng = np.random.default_rng(10)
    darks = (np.uint16(16383) - rng.integers(0, 3, size=(n, 1, 1, 8)).astype(np.uint16)) | np.uint16(0x4000)
    g = pdc.geometry(1, 1, 8, 8)
    p, s = pdc.dark_stats(ctx, g, torch.from_numpy(darks).cuda(), n)
    wp, ws = S.dark_stats(darks.reshape(n, 1, 8))
    assert np.array_equal(p.reshape(-1), wp.reshape(-1)) and np.array_equal(s.reshape(-1), ws.reshape(-1))


def test_calibrate_darks_then_process(ctx):
    """A detector calibrated from its darks finds the same hits as the oracle
    given the oracle's pedestal."""
    import torch

    from paper_1903_06838_amd import pdc

    geom = synth.Geometry(1, 64, 192, 96)
    ped, gain = synth.make_calibration(geom, 11)
    darks = synth.make_frames(geom, ped, gain, 40, 0.0, 11, occ_id=5)
    raw = synth.make_frames(geom, ped, gain, 4, 0.02, 11)
    wped, wnoise = S.dark_stats(darks)
    want = oracle_threads(raw, wped, gain, geom.bank_cols)
    prm = pdc.params(3.0, 5.0, 3.0, 150.0)
    det, noise = pdc.calibrate_darks(ctx, pdc.geometry(*geom.shape, geom.bank_cols), torch.from_numpy(darks).cuda(),
                                     40, gain, prm)
    try:
        assert np.array_equal(noise, wnoise)
        b = pdc.process_frames(ctx, det, torch.from_numpy(raw).cuda(), 4, 1 << 16)
        hits, total, fh, fp, _ = pdc.get_hits(ctx, b, 4)
        pdc.release_batch(ctx, b)
    finally:
        pdc.release_detector(ctx, det)
    assert total == want["total"] > 50
    assert np.array_equal(hits.view(np.uint32), want["hits"].view(np.uint32))
    with pytest.raises(pdc.PdcError):
        pdc.dark_stats(ctx, pdc.geometry(*geom.shape, geom.bank_cols), torch.from_numpy(darks).cuda(), 1)
