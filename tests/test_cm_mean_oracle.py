"""Pins for the thresholded-mean common-mode oracle (oracle/cm_mean.py): closed
forms, the guard, exact sums worked by hand (where a left-to-right sum and a
tree of partial sums both differ from the exactly rounded one), ties of the
one rounding, order invariance, the integer method against Fractions with an
independent nearest-float search, stacked stages worked by hand, and the
float64 mean within two roundings.  CPU only."""
from fractions import Fraction

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


def test_exact_sum_by_hand():
    # [2^24, 1, 1, -2^24]: the exact sum is 2 (a left-to-right binary32 sum
    # gives 0, the tree (p0 + p1) + (p2 + p3) gives 1); CM = 2 / 4
    f1, B = _bank([BIG, 1.0, 1.0, -BIG])
    _, cms = M.common_mode(f1, M.BANK, B, 1, 2.0 ** 25)
    assert cms[0, 0] == F32(0.5)
    # [2^24, 1, 1/4, 1/4]: exact 2^24 + 1.5, rounded once to 2^24 + 2 (both
    # orders above give 2^24); CM = (2^24 + 2) / 4 = 2^22 + 1/2
    f1, B = _bank([BIG, 1.0, 0.25, 0.25])
    _, cms = M.common_mode(f1, M.BANK, B, 1, 2.0 ** 25)
    assert cms[0, 0] == F32(2.0 ** 22 + 0.5)


def test_one_rounding_ties_to_even():
    # 2^24 + 1 lies halfway between 2^24 and 2^24 + 2: the even one is 2^24;
    # 2^24 + 3 lies halfway between 2^24 + 2 and 2^24 + 4: the even one is 2^24 + 4
    assert M.exact_sums(np.array([[BIG, 1.0, 0.0, 0.0]], F32))[0] == BIG
    assert M.exact_sums(np.array([[BIG + F32(2.0), 1.0, 0.0, 0.0]], F32))[0] == F32(2.0 ** 24 + 4)
    # the same below zero, and a sum that cancels to +0
    assert M.exact_sums(np.array([[-BIG, -1.0]], F32))[0] == -BIG
    z = M.exact_sums(np.array([[3.5, -3.5, 0.0]], F32))[0]
    assert z == 0.0 and not np.signbit(z)


def test_sum_has_no_order():
    rng = np.random.default_rng(7)
    x = (rng.normal(0.0, 1.0, size=(40, 194)) * np.exp2(rng.integers(-30, 30, size=(40, 194)))).astype(F32)
    want = M.exact_sums(x)
    for _ in range(5):
        perm = rng.permutation(194)
        assert np.array_equal(M.exact_sums(x[:, perm]).view(np.uint32), want.view(np.uint32))
    # a tile's sum is the exact sum over all its rows, whatever the row split
    v = x.reshape(1, 20, 388)
    _, ct = M.common_mode(v, M.TILE, 194, 1, 1e30)
    assert ct[0, 0] == F32(M.exact_sums(x.reshape(1, -1))[0] / F32(40 * 194))


def _nearest_f32(q):
    """Nearest binary32 to the Fraction q, ties to even, by searching the
    neighbours of the double nearest to q (independent of the oracle)."""
    d = np.float32(float(q))
    cands = {d, np.nextafter(d, np.float32(np.inf)), np.nextafter(d, np.float32(-np.inf))}
    best = sorted(cands, key=lambda f: (abs(Fraction(float(f)) - q), int(np.float32(f).view(np.uint32)) & 1))
    return np.float32(best[0])


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_exact_sums_against_fractions(seed):
    rng = np.random.default_rng(seed)
    R, n = 30, 50
    mag = np.exp2(rng.integers(-149, 60, size=(R, n)).astype(np.float64))
    x = (rng.choice([-1.0, 1.0], size=(R, n)) * mag * rng.uniform(1.0, 2.0, size=(R, n))).astype(F32)
    x[rng.random((R, n)) < 0.2] = 0.0
    x[0, :] = np.float32(2.0 ** -149) * rng.integers(-5, 6, size=n).astype(F32)  # subnormals
    got = M.exact_sums(x)
    for r in range(R):
        q = sum(Fraction(float(v)) for v in x[r])
        assert got[r] == _nearest_f32(q), (r, got[r])


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
    # two roundings (the exact sum, then the quotient) and the float64 sum's
    # own error, far smaller
    assert np.all(np.abs(cms[:, 0] - want) <= 2.0 ** -22 * np.abs(want) + 1e-9)


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
