"""Pins for the multi-gain oracle (oracle/multigain.py): the decode tables,
range selection and the valid-only median worked by hand, and reduction to
the single-gain C oracle when every pixel reports range 0.  CPU only."""
import numpy as np

from oracle import multigain as G
from oracle import oracle as C
from paper_1903_06838_amd import synth

F32 = np.float32


def test_decode_tables():
    words = np.array([5, (1 << 14) | 6, (2 << 14) | 7, (3 << 14) | 8], np.uint16)
    r1, adc = G.decode(words, 1)
    assert r1.tolist() == [0, 1, 2, -1] and adc.tolist() == [5, 6, 7, 8]
    r2, _ = G.decode(words, 2)
    assert r2.tolist() == [0, 1, -1, 2]


def test_range_planes_by_hand():
    ped = np.array([[[[100.0, 100.0]]], [[[40.0, 40.0]]], [[[10.0, 10.0]]]], F32)  # [3, 1, 1, 2]
    gain = np.array([[[[1.0, 1.0]]], [[[0.25, 0.25]]], [[[0.5, 0.5]]]], F32)
    raw = np.array([[[(1 << 14) | 50, (2 << 14) | 12]]], np.uint16)
    # mode 1: (50 - 40) / 0.25 = 40 and (12 - 10) / 0.5 = 4
    assert G.frames1(raw, ped, gain, 1).tolist() == [[[40.0, 4.0]]]
    # mode 2: code 2 is invalid
    f = G.frames1(raw, ped, gain, 2)
    assert f[0, 0, 0] == 40.0 and np.isinf(f[0, 0, 1])


def test_valid_only_median_by_hand():
    inf = np.inf
    f1 = np.array([[[3.0, inf, 1.0, inf, 2.0, 9.0, 8.0, inf, inf, 7.0]]], F32)  # two banks of 5
    f2, m = G.median_cm(f1, 5)
    # bank 0 valid [3, 1, 2] -> median 2; bank 1 valid [9, 8, 7] -> 8
    assert m.ravel().tolist() == [2.0, 8.0]
    assert f2.ravel().tolist() == [1.0, 0.0, -1.0, 0.0, 0.0, 1.0, 0.0, 0.0, 0.0, -1.0]
    # a bank with no valid pixel: m = 0 and Frames2 all zero; even counts take the lower median
    f2, m = G.median_cm(np.array([[[inf, inf, 4.0, 6.0]]], F32), 2)
    assert m.ravel().tolist() == [0.0, 4.0] and f2.ravel().tolist() == [0.0, 0.0, 0.0, 2.0]


def test_all_high_gain_reduces_to_single_gain_oracle():
    geom = synth.Geometry(2, 20, 96, 48)
    ped, gain = synth.make_calibration(geom, 3)
    raw = synth.make_frames(geom, ped, gain, 3, 0.03, 3)
    want = C.load().process(raw, ped, gain, 48, keep_corrected=True)
    ped3 = np.stack([ped, ped + 7, ped - 7]).astype(F32)
    gain3 = np.stack([gain, gain * 2, gain * 3]).astype(F32)
    for mode in (1, 2):
        got = G.process(raw, ped3, gain3, 48, mode, keep_corrected=True)
        assert np.array_equal(got["hits"], want["hits"]) and got["total"] == want["total"] > 20
        assert np.array_equal(got["corrected"].view(np.uint32), want["corrected"].view(np.uint32))
        assert got["invalid"].tolist() == [0, 0, 0]


def test_generated_ranges_and_invalid_counts():
    geom = synth.Geometry(1, 40, 96, 48)
    ped, gain = synth.make_calibration_multigain(geom, 4)
    raw = synth.make_frames_multigain(geom, ped, gain, 2, 0.02, 4, gain_mode=2)
    r, _ = G.decode(raw, 2)
    frac = [np.mean(r == k) for k in (0, 1, 2, -1)]
    assert abs(frac[0] - 0.80) < 0.03 and abs(frac[3] - 0.02) < 0.01 and frac[2] > 0.04
    got = G.process(raw, ped, gain, 48, 2, keep_corrected=True)
    assert got["invalid"].tolist() == [int(np.sum(r[0] < 0)), int(np.sum(r[1] < 0))]
    assert np.all(got["corrected"][r < 0] == 0.0)
    assert got["total"] > 10
