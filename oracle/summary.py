"""Oracle for the summaries (TEST INFRASTRUCTURE ONLY; never imported by the
product path, shares no code with the GPU library).

Summarization section: the processed data are reduced to photon-counting
maps, histograms (spectra) and sparse photon lists, accumulated over frames;
the Dark and Gain section and the Results section (noise thresholds in units
of the noise sigma): pedestal and noise come from dark frames.

* count_map: per pixel, the sum of the photon counts of the hits at it.
* histogram: bin 0 holds values below lo, bins 1..nbins the range, bin
  nbins + 1 the rest; for x >= lo the bin is 1 + floor(t) with
  t = fl(fl(x - lo) * s) in binary32 and s = fl(nbins / fl(hi - lo)), or
  nbins + 1 when t >= nbins (float32 takes the integer decision, as on the GPU).
* cloud_sizes / size_spectra: for each hit, the number of pixels of its
  in-tile 3x3 window whose Frames2 value is above t_nb (the charge-sharing
  components of Fig. g: charges summed over 1, 2, 3, ... pixels), and the
  charge spectrum of the hits of each size.
* dark_stats: exact integer sums S1 = sum(adc), S2 = sum(adc^2) over the dark
  frames (adc = raw & 0x3FFF); pedestal = float32(S1 / n) and
  noise = float32(sqrt((n S2 - S1^2) / (n (n - 1)))), the quotient and the
  root in IEEE double from the exact integer numerator.
"""
from __future__ import annotations

import math

import numpy as np

F32 = np.float32


def count_map(hits, n_pixels):
    """hits: records with fields pixel and nphot; returns uint32 [n_pixels]."""
    out = np.zeros(n_pixels, np.uint64)
    np.add.at(out, np.asarray(hits["pixel"], np.int64), np.asarray(hits["nphot"], np.uint64))
    return (out & 0xFFFFFFFF).astype(np.uint32)


def hist_scale(lo, hi, nbins):
    return F32(F32(nbins) / F32(F32(hi) - F32(lo)))


def histogram(values, lo, hi, nbins):
    """uint32 [nbins + 2]: below, nbins bins, at or above (see module doc)."""
    x = np.asarray(values, F32).ravel()
    lo = F32(lo)
    s = hist_scale(lo, hi, nbins)
    out = np.zeros(nbins + 2, np.uint64)
    below = ~(x >= lo)
    out[0] = np.count_nonzero(below)
    xi = x[~below]
    t = ((xi - lo).astype(F32) * s).astype(F32)
    inside = t < F32(nbins)
    b = 1 + np.floor(t[inside]).astype(np.int64)
    np.add.at(out, b, 1)
    out[nbins + 1] += np.count_nonzero(~inside)
    return out.astype(np.uint32)


def cloud_sizes(frames2, hits, t_nb):
    """frames2 float32 [N, T, H, W]; hits with fields frame and pixel; returns
    int64 [len(hits)], each in 1..9 for a hit above a threshold >= t_nb."""
    v = np.asarray(frames2, F32)
    N, T, H, W = v.shape
    t_nb = F32(t_nb)
    out = np.zeros(len(hits), np.int64)
    for i, (f, p) in enumerate(zip(np.asarray(hits["frame"]), np.asarray(hits["pixel"]))):
        t, rem = divmod(int(p), H * W)
        r, c = divmod(rem, W)
        win = v[int(f), t, max(r - 1, 0):r + 2, max(c - 1, 0):c + 2]
        out[i] = np.count_nonzero(win > t_nb)
    return out


def size_spectra(frames2, hits, t_nb, lo, hi, nbins):
    """uint32 [9, nbins + 2]: row s - 1 is the charge histogram of the hits of
    cloud size s."""
    sizes = cloud_sizes(frames2, hits, t_nb)
    q = np.asarray(hits["charge"], F32)
    return np.stack([histogram(q[sizes == s], lo, hi, nbins) for s in range(1, 10)])


def dark_stats(darks):
    """darks: uint16 [n, ...]; returns (pedestal float32, noise float32) of the
    trailing shape, n >= 2."""
    d = np.asarray(darks).astype(np.int64) & 0x3FFF
    n = d.shape[0]
    s1 = d.sum(axis=0)
    s2 = (d * d).sum(axis=0)
    ped = np.empty(s1.shape, F32)
    noise = np.empty(s1.shape, F32)
    fs1, fs2, fp, fn = s1.ravel(), s2.ravel(), ped.ravel(), noise.ravel()
    for i in range(fs1.size):
        a, b = int(fs1[i]), int(fs2[i])
        fp[i] = F32(a / n)                       # Python: correctly rounded double quotient
        num = n * b - a * a                      # exact integer, >= 0
        fn[i] = F32(math.sqrt(float(num) / (float(n) * float(n - 1))))
    return ped, noise
