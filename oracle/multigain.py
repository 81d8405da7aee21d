"""Oracle for auto-ranging (multi-gain) detectors (TEST INFRASTRUCTURE ONLY;
never imported by the product path, shares no code with the GPU library).

Dark and Gain section and Fig. b: detectors that switch gain range per pixel
need one dark and one gain plane per range; the corrected value of a pixel
uses the planes of the range its raw word reports.  Raw word: bits 14-15 the
gain code, bits 0-13 the ADC value.
  gain_mode 1 (ePix10k-like):  codes 0, 1, 2 -> ranges 0, 1, 2; code 3 invalid
  gain_mode 2 (Jungfrau-like): codes 0, 1, 3 -> ranges 0, 1, 2; code 2 invalid
  Frames1 u = fl(fl(adc - dark[r]) * fl(1 / gain[r])) for range r.
Readings fixed here:
* an invalid pixel has no Frames1 value: it takes no part in the common mode
  (the bank median is the element of rank (n - 1) / 2 of the bank's n valid
  values, 0 when n = 0; the thresholded mean does not count it as noise, while
  its guard still uses the region's size) and its Frames2 value is +0.0, so it
  never seeds and adds nothing to a charge; each frame reports how many
  invalid pixels it had;
* one pair of thresholds applies to all ranges (Frames1 is in the same units
  for every range).
"""
from __future__ import annotations

import numpy as np

F32 = np.float32
RANGE_OF_CODE = {1: np.array([0, 1, 2, -1]), 2: np.array([0, 1, -1, 2])}


def decode(raw, gain_mode):
    """(range int [..], adc uint16 [..]); range -1 marks an invalid code."""
    raw = np.asarray(raw, np.uint16)
    code = (raw >> 14).astype(np.int64)
    return RANGE_OF_CODE[gain_mode][code], raw & np.uint16(0x3FFF)


def frames1(raw, ped, gain, gain_mode):
    """raw uint16 [T, H, W]; ped, gain float32 [3, T, H, W] -> float32
    [T, H, W] with +inf at invalid pixels."""
    r, adc = decode(raw, gain_mode)
    ped = np.asarray(ped, F32)
    k = (F32(1.0) / np.asarray(gain, F32)).astype(F32)
    rr = np.where(r < 0, 0, r)
    p = np.take_along_axis(ped, rr[None], 0)[0]
    kk = np.take_along_axis(k, rr[None], 0)[0]
    u = ((adc.astype(F32) - p).astype(F32) * kk).astype(F32)
    return np.where(r < 0, F32(np.inf), u).astype(F32)


def median_cm(f1, bank_cols):
    """Frames2 by the lower median of each bank's valid values."""
    T, H, W = f1.shape
    x = f1.reshape(T, H, W // bank_cols, bank_cols)
    s = np.sort(x, axis=-1)
    nv = np.count_nonzero(np.isfinite(x), axis=-1)
    rank = np.maximum(nv - 1, 0) // 2
    m = np.take_along_axis(s, rank[..., None], -1)[..., 0]
    m = np.where(nv > 0, m, F32(0)).astype(F32)
    v = (x - m[..., None]).astype(F32)
    return np.where(np.isfinite(x), v, F32(0)).reshape(T, H, W).astype(F32), m


def process(raw, ped, gain, bank_cols, gain_mode, cm_mode=0, stages=1, sigma=3.0, n_seed=5.0, n_nb=3.0,
            n_cm=3.0, photon_adu=150.0, keep_corrected=False):
    """Whole path for a multi-gain detector: same dict layout as the C
    oracle's process, plus per-frame invalid counts."""
    from oracle import cm_mean as M
    from oracle import oracle as C

    o = C.load()
    raw = np.ascontiguousarray(raw, np.uint16)
    N = raw.shape[0]
    t_seed = F32(F32(n_seed) * F32(sigma))
    t_nb = F32(F32(n_nb) * F32(sigma))
    t_cm = F32(F32(n_cm) * F32(sigma))
    hits, corr = [], []
    fh, fp, inv = np.zeros(N, np.uint32), np.zeros(N, np.uint64), np.zeros(N, np.uint32)
    for f in range(N):
        f1 = frames1(raw[f], ped, gain, gain_mode)
        bad = ~np.isfinite(f1)
        inv[f] = np.count_nonzero(bad)
        if cm_mode == 0:
            f2, _ = median_cm(f1, bank_cols)
        else:
            f2, _ = M.common_mode(f1, cm_mode, bank_cols, stages, t_cm)
            f2 = np.where(bad, F32(0), f2).astype(F32)
        h, ph = o.find_hits(f2, float(t_seed), float(t_nb), float(photon_adu), frame=f)
        hits.append(h)
        fh[f] = len(h)
        fp[f] = ph
        if keep_corrected:
            corr.append(f2)
    out = dict(hits=np.concatenate(hits) if hits else np.zeros(0, C.HIT_DTYPE), frame_hits=fh,
               frame_photons=fp, total=int(fh.sum()), invalid=inv)
    if keep_corrected:
        out["corrected"] = np.stack(corr) if corr else np.zeros(raw.shape, F32)
    return out
