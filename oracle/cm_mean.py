"""Oracle for the thresholded-mean common mode (TEST INFRASTRUCTURE ONLY;
never imported by the product path, shares no code with the GPU library).

Common Mode section and Fig. c: the pixels without signal are segmented
(Noise? = Frames1 < T with T = n_cm * sigma, the figure's 3 sigma), counted
(N0) and summed (the sum of Frames1 * Noise?); the common mode is that sum
divided by N = max(N0, sqrt(HW)), the guard that keeps a few noise pixels at
high occupancy from setting the correction, and it is subtracted from every
pixel.  The figure reduces over the whole frame; the section allows rows,
columns or blocks instead.  Here the region is a bank (one row of bank_cols
pixels of a tile; the guard is then sqrt(bank_cols)) or a tile (the guard is
sqrt(rows * cols); a one-tile detector's tile is its frame).  The
performance-model section stacks three common-mode stages: stage s works on
the output of stage s - 1.

Readings fixed here (the paper leaves them open):
* binary32 throughout; Frames2 = fl(v - CM) at each stage;
* the sum has no order: it is the exact sum of the region's noise pixels
  (a rational number), rounded once to the nearest binary32, ties to even;
  a pixel that is not below T adds nothing;
* N0 is converted to binary32, the guard is fl(sqrt(fl(region size))), and
  CM = fl(sum / max(N0, guard)).

The exact sum is computed with integers: a binary32 x is M 2^(E - 150),
M its 24-bit significand and E its exponent field (E = 1 and M the fraction
for subnormals), so every value is an integer multiple of 2^-149; the
multiples M are summed per exponent in int64 and the per-exponent sums are
combined in Python's unbounded integers before the one rounding.
"""
from __future__ import annotations

import math

import numpy as np

F32 = np.float32

BANK = 1
TILE = 2


def round_to_f32(n):
    """The binary32 nearest to n * 2^-149 (n a Python int), ties to even."""
    if n == 0:
        return F32(0.0)
    neg = n < 0
    a = -n if neg else n
    if a < (1 << 24):  # subnormal or normal with the unit 2^-149: exact
        r = math.ldexp(a, -149)
    else:
        sh = a.bit_length() - 24
        q, rem = a >> sh, a & ((1 << sh) - 1)
        half = 1 << (sh - 1)
        if rem > half or (rem == half and q & 1):
            q += 1
        r = math.ldexp(q, sh - 149)  # q <= 2^24: exact in a double
    r = F32(r)
    assert np.isfinite(r), "sum beyond the binary32 range"
    return F32(-r) if neg else r


def exact_sums(vals):
    """vals float32 [R, n] -> float32 [R]: each row's exact sum rounded once
    to binary32 (ties to even)."""
    v = np.ascontiguousarray(vals, F32)
    R, n = v.shape
    b = v.view(np.uint32).astype(np.int64)
    e = (b >> 23) & 0xFF
    frac = b & 0x7FFFFF
    m = np.where(e > 0, frac | (1 << 23), frac)
    m = np.where(b >> 31 == 1, -m, m)
    e = np.maximum(e, 1)
    per = np.zeros((R, 256), np.int64)  # |sum| <= n 2^24 per exponent
    np.add.at(per, (np.repeat(np.arange(R), n), e.ravel()), m.ravel())
    out = np.zeros(R, F32)
    for r in range(R):
        nz = np.nonzero(per[r])[0]
        out[r] = round_to_f32(sum(int(per[r, k]) << int(k - 1) for k in nz))
    return out


def region_cm(x, t_cm):
    """x float32 [regions, n] (each region's pixels); returns (cm float32
    [regions], n0 int64 [regions])."""
    x = np.asarray(x, F32)
    R, n = x.shape
    mask = x < F32(t_cm)
    s = exact_sums(np.where(mask, x, F32(0)))
    n0 = np.count_nonzero(mask, axis=1)
    guard = F32(np.sqrt(F32(n)))
    N = np.maximum(n0.astype(F32), guard)
    return (s / N).astype(F32), n0


def _regions(v, region, bank_cols):
    T, H, W = v.shape
    if region == BANK:
        return v.reshape(T * H * (W // bank_cols), bank_cols)
    if region == TILE:
        return v.reshape(T, H * W)
    raise ValueError("region must be BANK or TILE")


def common_mode(frames1, region, bank_cols, stages, t_cm):
    """frames1 float32 [T, H, W] -> (Frames2 float32 [T, H, W], cm float32
    [regions, 3]) with the stage values in columns 0..stages-1, zeros after."""
    if not 1 <= stages <= 3:
        raise ValueError("1 to 3 stages")
    v = np.array(frames1, F32, copy=True)
    shape = v.shape
    x = _regions(v, region, bank_cols)
    cms = np.zeros((x.shape[0], 3), F32)
    for s in range(stages):
        c, _ = region_cm(x, t_cm)
        cms[:, s] = c
        x = (x - c[:, None]).astype(F32)
    return x.reshape(shape), cms


def process(raw, ped, gain, bank_cols, region, stages, sigma=3.0, n_seed=5.0, n_nb=3.0, n_cm=3.0,
            photon_adu=150.0, keep_corrected=False):
    """The whole path with the thresholded-mean common mode: dark and gain,
    the stacked stages, then hit finding and photon counting (the C oracle's
    stages for those).  Same dict layout as the C oracle's process."""
    from oracle import oracle as C

    o = C.load()
    raw = np.ascontiguousarray(raw, np.uint16)
    N = raw.shape[0]
    t_seed = F32(F32(n_seed) * F32(sigma))
    t_nb = F32(F32(n_nb) * F32(sigma))
    t_cm = F32(F32(n_cm) * F32(sigma))
    hits, fh, fp, corr = [], np.zeros(N, np.uint32), np.zeros(N, np.uint64), []
    for f in range(N):
        f1 = o.dark_gain(raw[f], ped, gain)
        f2, _ = common_mode(f1, region, bank_cols, stages, t_cm)
        h, ph = o.find_hits(f2, float(t_seed), float(t_nb), float(photon_adu), frame=f)
        hits.append(h)
        fh[f] = len(h)
        fp[f] = ph
        if keep_corrected:
            corr.append(f2)
    out = dict(hits=np.concatenate(hits) if hits else np.zeros(0, C.HIT_DTYPE), frame_hits=fh,
               frame_photons=fp, total=int(fh.sum()))
    if keep_corrected:
        out["corrected"] = np.stack(corr) if corr else np.zeros(raw.shape, F32)
    return out
