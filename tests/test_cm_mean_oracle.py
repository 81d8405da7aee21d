"""Pins for the thresholded-mean common-mode oracle (oracle/cm_mean.py): closed
forms, the guard, the summation order worked by hand, stacked stages worked by
hand, and the float64 mean within its rounding bound.  CPU only."""
import numpy as np
import pytest

from oracle import cm_mean as M

F32 = np.float32
BIG = F32(2 ** 24)


def _bank(vals, B=None):
    v = np.asarray(vals, F32)
    B = B or len(v)
    return v.reshape(1, 1, B), B


def test_constant_region_is_its_own_mean():
    for B in (8, 96, 194, 1024):
        f1, _ = _bank(np.full(B, 5.0), B)
        f2, cms = M.common_mode(f1, M.BANK, B, 3, 9.0)
        assert cms[0].tolist() == [5.0, 0.0, 0.0] and np.all(f2 == 0.0)


def test_guard_limits_few_noise_pixels():
    # 196 pixels, three below the threshold: sum 28, N0 = 3 < sqrt(196) = 14
    v = np.full(196, 100.0, F32)
    v[[5, 70, 195]] = [7.0, 7.0, 14.0]
    f2, cms = M.common_mode(v.reshape(1, 1, 196), M.BANK, 196, 1, 18.0)
    assert cms[0, 0] == F32(2.0)
    assert f2[0, 0, 0] == F32(98.0)
    # with no pixel below the threshold the correction is 0 / guard = 0
    _, cms = M.common_mode(np.full((1, 1, 196), 50.0, F32), M.BANK, 196, 1, 18.0)
    assert cms[0, 0] == 0.0


def test_sum_order_interleaved_then_tree_bank():
    # B = 4: partials hold one pixel each; the tree adds (p0 + p1) + (p2 + p3):
    # fl(2^24 + 1) = 2^24 (tie to even), fl(1 - 2^24) = -(2^24 - 1), sum 1;
    # left to right would give 0, the exact sum is 2.
    f1, B = _bank([BIG, 1.0, 1.0, -BIG])
    _, cms = M.common_mode(f1, M.BANK, B, 1, 2.0 ** 25)
    assert cms[0, 0] == F32(1.0) / F32(4.0)
    # B = 128: pixel i goes to partial i mod 64; partial 0 = fl(2^24 + 1) = 2^24,
    # partial 1 = fl(1 - 2^24); sum 1, N = 128
    v = np.zeros(128, F32)
    v[0], v[64], v[1], v[65] = BIG, 1.0, 1.0, -BIG
    _, cms = M.common_mode(v.reshape(1, 1, 128), M.BANK, 128, 1, 2.0 ** 25)
    assert cms[0, 0] == F32(1.0 / 128)


def test_sum_order_tile_uses_256_partials():
    # a 2 x 256 tile: pixel (r, c) goes to partial c; the same pixels in a bank
    # region (one row each) give different sums
    v = np.zeros((1, 2, 256), F32)
    v[0, 0, 0], v[0, 1, 0], v[0, 0, 1], v[0, 1, 1] = BIG, 1.0, 1.0, -BIG
    _, cms = M.common_mode(v, M.TILE, 256, 1, 2.0 ** 25)
    assert cms[0, 0] == F32(1.0 / 512)
    _, cb = M.common_mode(v, M.BANK, 256, 1, 2.0 ** 25)
    # row 0: partial 0 = 2^24, partial 1 = 1 -> (2^24 + 1) = 2^24; row 1: 1 - 2^24
    assert cb[0, 0] == BIG / F32(256) and cb[1, 0] == F32(1.0 - 2.0 ** 24) / F32(256)


def test_stacked_stages_by_hand():
    # T = 16.  Stage 1: 29 is excluded, CM = 42 / 3 = 14 -> [15, 0, 0, 0].
    # Stage 2: 15 < 16 now counts, CM = 15 / 4 = 3.75 -> [11.25, -3.75 x 3].
    # Stage 3: (11.25 - 3.75) + (-3.75 - 3.75) = 0.
    f1, B = _bank([29.0, 14.0, 14.0, 14.0])
    f2, cms = M.common_mode(f1, M.BANK, B, 3, 16.0)
    assert cms[0].tolist() == [14.0, 3.75, 0.0]
    assert f2.ravel().tolist() == [11.25, -3.75, -3.75, -3.75]
    f2_1, _ = M.common_mode(f1, M.BANK, B, 1, 16.0)
    assert f2_1.ravel().tolist() == [15.0, 0.0, 0.0, 0.0]


def test_threshold_is_strict():
    f1, B = _bank([16.0, 0.0, 0.0, 0.0])
    _, cms = M.common_mode(f1, M.BANK, B, 1, 16.0)
    assert cms[0, 0] == 0.0  # 16 is not below 16
    _, cms = M.common_mode(f1, M.BANK, B, 1, float(np.nextafter(F32(16), F32(17))))
    assert cms[0, 0] == 4.0


@pytest.mark.parametrize("region,shape", [(M.BANK, (3, 40, 388)), (M.TILE, (2, 185, 388))])
def test_close_to_float64_mean(region, shape):
    rng = np.random.default_rng(4)
    f1 = rng.normal(7.0, 3.0, size=shape).astype(F32)
    f1[rng.random(shape) < 0.02] += 150.0  # photons, excluded by the threshold
    t = F32(9.0)
    _, cms = M.common_mode(f1, region, 194, 1, t)
    x = M._regions(f1, region, 194).astype(np.float64)
    m = x < t
    n0 = m.sum(axis=1)
    want = (x * m).sum(axis=1) / np.maximum(n0, np.sqrt(x.shape[1]))
    # rounding bound of a sum of n terms: about n * eps * sum |x|
    bound = x.shape[1] * 2.0 ** -23 * (np.abs(x) * m).sum(axis=1) / np.maximum(n0, 1) + 1e-6
    assert np.all(np.abs(cms[:, 0] - want) <= bound)
    assert np.max(np.abs(cms[:, 0] - want)) < 1e-4


def test_process_reduces_to_find_hits():
    """With the whole path: a frame whose only offsets are per-bank constants is
    corrected exactly, so the hits are those of the signal alone."""
    from oracle import oracle as C

    T, H, W, B = 1, 8, 16, 8
    rng = np.random.default_rng(5)
    sig = np.zeros((T, H, W), F32)
    sig[0, 3, 4], sig[0, 3, 5] = 120.0, 60.0
    sig[0, 6, 12] = 300.0
    off = np.repeat(rng.integers(-5, 6, size=(T, H, W // B)), B, axis=2).astype(F32)
    ped = np.full((T, H, W), 1000.0, F32)
    gain = np.ones((T, H, W), F32)
    raw = (1000.0 + sig + off).astype(np.uint16)[None]
    got = M.process(raw, ped, gain, B, M.BANK, 1, keep_corrected=True)
    # photon pixels are above 9 ADU, so each bank's mean is its offset exactly
    assert np.array_equal(got["corrected"][0], sig)
    h, ph = C.load().find_hits(sig, 15.0, 9.0, 150.0)
    assert np.array_equal(got["hits"], h) and got["frame_photons"][0] == ph
    assert got["total"] == 2 and sorted(got["hits"]["nphot"].tolist()) == [1, 2]
