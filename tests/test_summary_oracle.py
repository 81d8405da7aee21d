"""Pins for the summaries oracle (oracle/summary.py).  CPU only."""
import numpy as np

from oracle import summary as S

F32 = np.float32


def test_histogram_hand_worked():
    # 4 bins of width 1 over [0, 4): below, [0,1), [1,2), [2,3), [3,4), at or above
    v = np.array([-1.0, 0.0, 0.5, 1.0, 3.999, 4.0, 100.0, np.nextafter(F32(0), F32(-1))], F32)
    assert S.histogram(v, 0.0, 4.0, 4).tolist() == [2, 2, 1, 0, 1, 2]


def test_histogram_bin_centres_and_total():
    rng = np.random.default_rng(0)
    lo, hi, nb = -50.0, 250.0, 300
    centres = lo + (np.arange(nb) + 0.5) * (hi - lo) / nb
    idx = rng.integers(0, nb, 5000)
    h = S.histogram(centres[idx].astype(F32), lo, hi, nb)
    assert np.array_equal(h[1:-1], np.bincount(idx, minlength=nb))
    assert h[0] == 0 and h[-1] == 0
    x = rng.normal(50, 80, 20000).astype(F32)
    assert S.histogram(x, lo, hi, nb).sum() == len(x)
    # away from bin edges it agrees with numpy's histogram
    edges = np.linspace(lo, hi, nb + 1)
    far = np.min(np.abs(x[:, None] - edges[None, :]), axis=1) > 1e-3
    want = np.histogram(x[far], bins=edges)[0]
    got = S.histogram(x[far], lo, hi, nb)
    assert np.array_equal(got[1:-1], want)
    assert got[0] == np.count_nonzero(x[far] < lo) and got[-1] == np.count_nonzero(x[far] >= hi)


def test_count_map():
    hits = np.zeros(5, [("pixel", "<u4"), ("nphot", "<u4")])
    hits["pixel"] = [3, 0, 3, 7, 3]
    hits["nphot"] = [1, 2, 0, 5, 4]
    assert S.count_map(hits, 8).tolist() == [2, 0, 0, 5, 0, 0, 0, 5]


def test_dark_stats_closed_forms():
    c = np.full((5, 3, 4), 1234, np.uint16)
    ped, noise = S.dark_stats(c)
    assert np.all(ped == 1234.0) and np.all(noise == 0.0)
    a = np.array([[[100, 7]]], np.uint16)
    b = np.array([[[103, 7]]], np.uint16)
    ped, noise = S.dark_stats(np.concatenate([a, b]))
    assert ped[0, 0] == F32(101.5) and noise[0, 0] == F32(3 / np.sqrt(2.0))
    assert noise[0, 1] == 0.0
    # gain bits above the 14-bit ADC word are ignored
    g = np.concatenate([a | 0x8000, b | 0x4000])
    assert np.array_equal(S.dark_stats(g)[0], ped)


def test_dark_stats_matches_float64_moments():
    rng = np.random.default_rng(3)
    d = np.clip(np.rint(rng.normal(1500, 3, size=(64, 20, 30))), 0, 16383).astype(np.uint16)
    ped, noise = S.dark_stats(d)
    x = d.astype(np.float64)
    assert np.array_equal(ped, x.mean(axis=0).astype(F32))
    want = x.std(axis=0, ddof=1)
    assert np.max(np.abs(noise - want) / want) <= 2 ** -23


def test_cloud_sizes_hand_worked():
    # one frame, two 3x4 tiles; t_nb = 10
    v = np.zeros((1, 2, 3, 4), F32)
    v[0, 0] = [[50, 11, 0, 0],
               [10, 12, 0, 9],
               [0, 0, 0, 99]]
    v[0, 1] = [[0, 0, 0, 0],
               [0, 40, 40, 0],
               [11, 11, 11, 0]]
    hits = np.zeros(4, [("frame", "<u4"), ("pixel", "<u4"), ("charge", "<f4")])
    hits["pixel"] = [0, 11, 12 + 5, 12 + 6]
    hits["charge"] = [73, 99, 113, 113]
    # corner (0,0): 50, 11, 12 above (10 is not); (2,3) of tile 0: only 99 (the
    # window stops at the tile edge, tile 1 below is not counted); tile 1 (1,1):
    # 40, 40, 11, 11, 11; (1,2): 40, 40, 11, 11
    assert S.cloud_sizes(v, hits, 10.0).tolist() == [3, 1, 5, 4]
    sp = S.size_spectra(v, hits, 10.0, 0.0, 200.0, 2)
    assert sp.shape == (9, 4)
    assert sp[2].tolist() == [0, 1, 0, 0] and sp[0].tolist() == [0, 1, 0, 0]
    assert sp[4].tolist() == [0, 0, 1, 0] and sp[3].tolist() == [0, 0, 1, 0]
    assert sp.sum() == 4
