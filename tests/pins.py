"""Pins for the CPU oracle: checks against facts that do not come from the oracle.

Each ``pin_*`` function takes an oracle handle (``oracle.oracle.Oracle``) and
raises AssertionError when the oracle disagrees with

* hand-worked fixtures in tests/golden/ (each cites the passage it follows),
* closed forms (integer pedestals with unit or power-of-two gains are exact),
* a float64 evaluation of the same definitions within a derived error bound,
* brute force on tiny inputs, written differently from the oracle (rank
  counting for the median, a lexicographic arg-max for the local maximum),
* invariants of the method (injected noise-free photons, dark frames, constant
  per-bank offsets, translation, batch composition).

The same checks run against mutated copies of the oracle in
test_oracle_mutants.py, which shows that each planted mistake fails at least
one of them.
"""
from __future__ import annotations

import json
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
F32 = np.float32


def _golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def _hits_tuple(hits):
    return [(int(h["pixel"]), float(h["charge"]), int(h["nphot"])) for h in hits]


# --------------------------------------------------------------------------
# steps 1-3: decode, dark, gain
# --------------------------------------------------------------------------
def pin_adc_mask(o):
    """Only the low 14 bits are the ADC value; bits 14-15 (gain bits) are ignored."""
    rng = np.random.default_rng(11)
    adc = rng.integers(0, 1 << 14, size=(1, 8, 16)).astype(np.uint16)
    dark = np.zeros(adc.shape, F32)
    gain = np.ones(adc.shape, F32)
    base = o.dark_gain(adc, dark, gain)
    assert np.array_equal(base, adc.astype(F32))
    for top in (1, 2, 3):
        tagged = (adc | np.uint16(top << 14)).astype(np.uint16)
        assert np.array_equal(o.dark_gain(tagged, dark, gain).view(np.uint32), base.view(np.uint32))


def pin_dark_gain_exact(o):
    """Integer dark with gain 1 or a power of two: Frames1 = (adc - dark) / gain exactly."""
    rng = np.random.default_rng(12)
    adc = rng.integers(0, 1 << 14, size=(2, 8, 32)).astype(np.uint16)
    dark = rng.integers(1000, 2000, size=adc.shape).astype(F32)
    for g in (1.0, 2.0, 0.25, 8.0):
        gain = np.full(adc.shape, g, F32)
        want = (adc.astype(np.float64) - dark.astype(np.float64)) / g   # exact in binary32
        got = o.dark_gain(adc, dark, gain)
        assert np.array_equal(got.astype(np.float64), want), g


def pin_dark_gain_bound(o):
    """Realistic planes: |Frames1 - (adc - dark)/gain| within three binary32 roundings."""
    rng = np.random.default_rng(13)
    shape = (2, 16, 64)
    dark = rng.normal(1500, 50, size=shape).astype(F32)
    gain = rng.uniform(0.5, 2.0, size=shape).astype(F32)
    adc = np.clip(np.rint(dark + rng.normal(0, 200, size=shape)), 0, 16383).astype(np.uint16)
    exact = (adc.astype(np.float64) - dark.astype(np.float64)) / gain.astype(np.float64)
    got = o.dark_gain(adc, dark, gain).astype(np.float64)
    eps = 2.0 ** -24
    # t = fl(a - d) (|err| <= eps|t|), k = fl(1/g) (<= eps/g), u = fl(t k) (<= eps|u|)
    bound = 3.01 * eps * np.abs(exact) + 1e-30
    assert np.all(np.abs(got - exact) <= bound)


# --------------------------------------------------------------------------
# step 4-5: bank median and common-mode subtraction
# --------------------------------------------------------------------------
def _rank_ok(bank, m):
    """Brute-force rank test: m is in the bank, #{x < m} <= k < #{x <= m}, k = (B-1)//2."""
    k = (len(bank) - 1) // 2
    below = sum(1 for x in bank if x < m)
    below_eq = sum(1 for x in bank if x <= m)
    return (m in list(bank)) and below <= k < below_eq


def pin_median_handworked(o):
    for case in _golden("median_small.json")["cases"]:
        bank = np.array(case["bank"], F32)
        med = o.bank_medians(bank.reshape(1, 1, -1), len(bank))
        assert med.shape == (1, 1, 1)
        assert med[0, 0, 0] == F32(case["median"]), (case, med)


def pin_median_rank_bruteforce(o):
    """Random banks (many ties; B odd and even; several banks per row and tiles)."""
    rng = np.random.default_rng(14)
    for B, nb, T, H in ((1, 3, 1, 2), (2, 2, 2, 3), (5, 3, 1, 4), (6, 4, 2, 3), (7, 2, 1, 2),
                        (96, 2, 1, 2), (194, 2, 2, 2)):
        W = B * nb
        f1 = rng.integers(-4, 5, size=(T, H, W)).astype(F32) * F32(0.5)
        med = o.bank_medians(f1, B)
        for t in range(T):
            for r in range(H):
                for b in range(nb):
                    bank = f1[t, r, b * B:(b + 1) * B]
                    assert _rank_ok(bank.tolist(), float(med[t, r, b])), (B, t, r, b)


def pin_common_mode_invariants(o):
    """Post-CM bank median is exactly +0; Frames2 = Frames1 - median pixel by pixel."""
    rng = np.random.default_rng(15)
    T, H, B, nb = 2, 3, 10, 3
    W = B * nb
    f1 = rng.normal(0, 5, size=(T, H, W)).astype(F32)
    f1 += rng.normal(0, 10, size=(T, H, nb)).repeat(B, axis=2).astype(F32)
    f2 = o.common_mode(f1, B)
    for t in range(T):
        for r in range(H):
            for b in range(nb):
                bank1 = f1[t, r, b * B:(b + 1) * B]
                bank2 = f2[t, r, b * B:(b + 1) * B]
                # the median of Frames1 by rank counting (independent of the oracle)
                m = [x for x in bank1.tolist() if _rank_ok(bank1.tolist(), x)][0]
                assert np.array_equal(bank2, (bank1 - F32(m)).astype(F32))
                zero = [x for x in bank2.tolist() if _rank_ok(bank2.tolist(), x)]
                assert zero and zero[0] == 0.0 and np.signbit(F32(zero[0])) == False


# --------------------------------------------------------------------------
# steps 6-8 on fixed corrected frames
# --------------------------------------------------------------------------
def _golden_hits(o, name):
    g = _golden(name)
    fr = np.array(g["frame"], F32)
    if fr.ndim == 2:
        fr = fr[None]
    hits, _ = o.find_hits(fr, F32(g["t_seed"]), F32(g["t_nb"]), F32(g["photon_adu"]))
    want = [(h["pixel"], float(F32(h["charge"])), h["nphot"]) for h in g["hits"]]
    assert _hits_tuple(hits) == want, (name, _hits_tuple(hits), want)


def pin_golden_charge_sum_order(o):
    _golden_hits(o, "charge_sum_order.json")


def pin_golden_mask_threshold(o):
    _golden_hits(o, "mask_and_threshold.json")


def pin_golden_photon_rounding(o):
    _golden_hits(o, "photon_rounding.json")


def pin_golden_plateau(o):
    _golden_hits(o, "plateau_ties.json")


def pin_golden_tile_edge(o):
    _golden_hits(o, "tile_edge.json")


def brute_hits(v, t_seed, t_nb, photon_adu):
    """Independent brute force: p is a hit iff v[p] > t_seed and (v[p], -p) is the
    lexicographic maximum over its in-tile 3x3 window.  Charge: binary32 sum of
    the masked window in row-major order; count rint(q / E) in binary32."""
    T, H, W = v.shape
    out = []
    for t in range(T):
        for r in range(H):
            for c in range(W):
                vp = v[t, r, c]
                if not vp > t_seed:
                    continue
                p = (t * H + r) * W + c
                window = [(v[t, rr, cc], -((t * H + rr) * W + cc))
                          for rr in range(max(r - 1, 0), min(r + 2, H))
                          for cc in range(max(c - 1, 0), min(c + 2, W))]
                if max(window) != (vp, -p):
                    continue
                q = F32(0.0)
                for rr in range(max(r - 1, 0), min(r + 2, H)):
                    for cc in range(max(c - 1, 0), min(c + 2, W)):
                        x = v[t, rr, cc]
                        q = F32(q + (x if x > t_nb else F32(0.0)))
                n = int(np.rint(F32(q / F32(photon_adu))))
                out.append((p, float(q), n))
    return out


def pin_hits_bruteforce(o):
    """Tiny integer-valued frames (dense ties) and small-noise frames, 1-3 tiles."""
    rng = np.random.default_rng(16)
    for trial in range(12):
        T = 1 + trial % 3
        H = 2 + (trial * 3) % 7
        W = 3 + (trial * 5) % 11
        if trial % 2 == 0:
            v = rng.integers(-2, 6, size=(T, H, W)).astype(F32) * F32(8.0)
        else:
            v = rng.normal(0, 3, size=(T, H, W)).astype(F32)
            k = rng.integers(0, v.size, size=3)
            v.reshape(-1)[k] += F32(150.0)
        for (ts, tn) in ((15.0, 9.0), (0.0, 0.0), (16.0, 16.0)):
            hits, ph = o.find_hits(v, F32(ts), F32(tn), F32(150.0))
            want = brute_hits(v, F32(ts), F32(tn), 150.0)
            assert _hits_tuple(hits) == want, (trial, ts, tn)
            assert ph == sum(w[2] for w in want)


# --------------------------------------------------------------------------
# whole pipeline on raw frames: invariants
# --------------------------------------------------------------------------
def _flat_setup(T=2, H=12, W=24, B=12, dark_value=1000):
    dark = np.full((T, H, W), dark_value, F32)
    gain = np.ones((T, H, W), F32)
    return dark, gain, B


def pin_injected_photons(o):
    """Noise-free delta photons, integer dark, unit gain, no common mode:
    one hit per injected pixel, q = 150 k exactly, n = k."""
    dark, gain, B = _flat_setup()
    T, H, W = dark.shape
    raw = np.full((1, T, H, W), 1000, np.uint16)
    spots = [(0, 2, 2, 1), (0, 2, 6, 2), (0, 7, 10, 3), (1, 4, 4, 1), (1, 9, 20, 5), (1, 5, 15, 1)]
    for (t, r, c, k) in spots:
        raw[0, t, r, c] += 150 * k
    res = o.process(raw, dark, gain, B, sigma=3.0, n_seed=5.0, n_nb=3.0, photon_adu=150.0)
    want = sorted(((t * H + r) * W + c, 150.0 * k, k) for (t, r, c, k) in spots)
    assert _hits_tuple(res["hits"]) == want
    assert int(res["frame_photons"][0]) == sum(s[3] for s in spots)
    assert int(res["frame_hits"][0]) == len(spots)


def pin_dark_frames_no_hits(o):
    """Noise truncated to |n| < 2.5 sigma, integer dark, unit gain, per-bank offsets:
    every v = rint(cm + n) - rint(cm + n') <= 15 = 5 sigma, so a strict 5-sigma
    seed threshold finds nothing."""
    rng = np.random.default_rng(17)
    T, H, W, B = 2, 16, 48, 16
    dark = rng.normal(1500, 50, size=(T, H, W)).astype(F32).round()
    gain = np.ones((T, H, W), F32)
    n = rng.normal(0, 3, size=(4, T, H, W))
    n = np.clip(n, -7.4, 7.4)
    cm = rng.normal(0, 10, size=(4, T, H, W // B)).repeat(B, axis=3)
    raw = np.rint(dark[None] + cm + n).astype(np.uint16)
    res = o.process(raw, dark, gain, B, sigma=3.0, n_seed=5.0, n_nb=3.0)
    assert res["total"] == 0 and len(res["hits"]) == 0


def pin_cm_offset_removal(o):
    """Integer raw and dark, unit gain: adding an integer per bank changes nothing."""
    rng = np.random.default_rng(18)
    T, H, W, B = 2, 10, 40, 10
    dark = rng.integers(1400, 1600, size=(T, H, W)).astype(F32)
    gain = np.ones((T, H, W), F32)
    raw = (dark[None] + rng.integers(-6, 7, size=(3, T, H, W))).astype(np.int64)
    raw[0, 0, 3, 5] += 300
    raw[1, 1, 7, 33] += 160
    raw[2, 0, 0, 0] += 170
    off = rng.integers(-40, 41, size=(3, T, H, W // B)).repeat(B, axis=3)
    a = o.process(raw.astype(np.uint16), dark, gain, B, keep_corrected=True)
    b = o.process((raw + off).astype(np.uint16), dark, gain, B, keep_corrected=True)
    assert np.array_equal(a["corrected"].view(np.uint32), b["corrected"].view(np.uint32))
    assert _hits_tuple(a["hits"]) == _hits_tuple(b["hits"]) and a["total"] >= 3


def pin_translation(o):
    """Shifting an isolated pattern inside a tile shifts its hits."""
    dark, gain, B = _flat_setup(T=1, H=16, W=32, B=16)
    pat = np.array([[0, 20, 0], [30, 160, 12], [0, 25, 0]])
    res = []
    for (r0, c0) in ((3, 4), (9, 20)):
        raw = np.full((1, 1, 16, 32), 1000, np.int64)
        raw[0, 0, r0:r0 + 3, c0:c0 + 3] += pat
        h = o.process(raw.astype(np.uint16), dark, gain, B, sigma=3.0)["hits"]
        assert len(h) == 1
        res.append((int(h["pixel"][0]) - ((r0 + 1) * 32 + c0 + 1), float(h["charge"][0])))
    assert res[0] == res[1] == (0, float(F32(20 + 30 + 160 + 12 + 25)))


def pin_batch_independence(o):
    """A frame's result does not depend on the other frames of its batch."""
    rng = np.random.default_rng(19)
    T, H, W, B = 1, 12, 24, 12
    dark = rng.normal(1500, 50, size=(T, H, W)).astype(F32)
    gain = rng.uniform(0.95, 1.05, size=(T, H, W)).astype(F32)
    raw = np.clip(np.rint(dark[None] + rng.normal(0, 3, size=(3, T, H, W))), 0, 16383)
    raw[:, 0, 4, 4] += 200
    raw[1, 0, 8, 17] += 450
    raw = raw.astype(np.uint16)
    full = o.process(raw, dark, gain, B)
    for i in range(3):
        one = o.process(raw[i:i + 1], dark, gain, B)
        mine = full["hits"][full["hits"]["frame"] == i]
        assert _hits_tuple(one["hits"]) == _hits_tuple(mine)
        assert one["frame_photons"][0] == full["frame_photons"][i]


def pin_frames2_fp64_bound(o):
    """Frames2 against a float64 evaluation: v = (a - d)/g - m with m the float64
    value of the same ranked pixel; error within a few binary32 roundings."""
    rng = np.random.default_rng(20)
    T, H, W, B = 1, 6, 40, 20
    dark = rng.normal(1500, 50, size=(T, H, W)).astype(F32)
    gain = rng.uniform(0.9, 1.1, size=(T, H, W)).astype(F32)
    raw = np.clip(np.rint(dark[None] + rng.normal(0, 30, size=(1, T, H, W))), 0, 16383).astype(np.uint16)
    v = o.process(raw, dark, gain, B, keep_corrected=True)["corrected"][0].astype(np.float64)
    u64 = (raw[0].astype(np.float64) - dark) / gain.astype(np.float64)
    k = (B - 1) // 2
    eps = 2.0 ** -24
    for t in range(T):
        for r in range(H):
            for b in range(W // B):
                bank = u64[t, r, b * B:(b + 1) * B]
                m = np.sort(bank)[k]
                want = bank - m
                bound = 3.01 * eps * (np.abs(bank) + abs(m)) + eps * np.abs(want) + 1e-30
                assert np.all(np.abs(v[t, r, b * B:(b + 1) * B] - want) <= bound)


def pin_thresholds_from_params(o):
    """T_seed = n_seed * sigma, T_nb = n_nb * sigma: pixels exactly at a threshold
    are below it, pixels 1 ADU above it are above it."""
    dark, gain, B = _flat_setup(T=1, H=8, W=16, B=16)
    raw = np.full((1, 1, 8, 16), 1000, np.int64)
    # sigma = 2: T_seed = 8, T_nb = 4 (n_seed 4, n_nb 2)
    raw[0, 0, 2, 3] += 8       # == T_seed: not a seed
    raw[0, 0, 5, 3] += 9       # seed; neighbours 4 (== T_nb, zeroed) and 5 (kept)
    raw[0, 0, 5, 2] += 4
    raw[0, 0, 5, 4] += 5
    raw[0, 0, 2, 10] += 9      # seed whose neighbour sits just at 3 (< T_nb)
    raw[0, 0, 3, 10] += 3
    res = o.process(raw.astype(np.uint16), dark, gain, B, sigma=2.0, n_seed=4.0, n_nb=2.0,
                    photon_adu=3.0)
    assert _hits_tuple(res["hits"]) == [(2 * 16 + 10, 9.0, 3), (5 * 16 + 3, 14.0, 5)]


PINS = [pin_adc_mask, pin_dark_gain_exact, pin_dark_gain_bound, pin_median_handworked,
        pin_median_rank_bruteforce, pin_common_mode_invariants, pin_golden_charge_sum_order,
        pin_golden_mask_threshold, pin_golden_photon_rounding, pin_golden_plateau,
        pin_golden_tile_edge, pin_hits_bruteforce, pin_injected_photons,
        pin_dark_frames_no_hits, pin_cm_offset_removal, pin_translation,
        pin_batch_independence, pin_frames2_fp64_bound, pin_thresholds_from_params]
