"""Seeded synthetic detector frames.

This module only *generates inputs*: calibration planes (pedestal, gain) and raw
14-bit ADC frames with injected X-ray photons, common-mode offsets and noise.  It
contains none of the correction or photon-finding arithmetic; both the CPU
oracle and the GPU path consume what it produces.

The private 55Fe ePix100 data set the paper measures on (Methods section:
50,000 frames of 704x768 pixels, about 1 MB each) is not available, so these
generators stand in for it with the same frame shapes and with distributions
chosen to look like such data:

* pedestal  ~ N(1500, 50) ADU per pixel (float32)
* gain      ~ U(0.95, 1.05) per pixel (float32)
* per-frame, per-bank common-mode offset ~ N(0, 10) ADU
* electronic noise ~ N(0, 3) ADU per pixel
* photons: Poisson(occupancy) per pixel, each 150 ADU (at unit gain) spread as a
  2-D Gaussian cloud (sigma 0.2 px) integrated over the pixel areas of a 5x5
  window, charge outside the tile is lost (tiles are separate ASICs)
* raw = clip(rint(ped + gain * signal + cm + noise), 0, 16383) as uint16

Random streams: numpy PCG64 seeded by SeedSequence([1903, 6838, cfg, ...]) so
every frame is reproducible on its own (frame i does not depend on frames < i).
"""
from __future__ import annotations

import dataclasses

import numpy as np
from scipy.special import ndtr

ADC_MAX = 16383


@dataclasses.dataclass(frozen=True)
class Geometry:
    """Detector geometry: n_tiles tiles of rows x cols pixels.

    A common-mode bank is one row of bank_cols contiguous columns of a tile.
    Pixel index within a frame is (tile * rows + row) * cols + col.
    """
    n_tiles: int
    rows: int
    cols: int
    bank_cols: int

    @property
    def pixels(self) -> int:
        return self.n_tiles * self.rows * self.cols

    @property
    def shape(self) -> tuple:
        return (self.n_tiles, self.rows, self.cols)


# ePix100 camera module: one 704x768 sensor, 96-pixel row banks.
EPIX100 = Geometry(1, 704, 768, 96)
# CSPAD-like: 32 ASICs of 185x388, common mode per 194-pixel half-row.
CSPAD = Geometry(32, 185, 388, 194)


@dataclasses.dataclass(frozen=True)
class SimParams:
    ped_mean: float = 1500.0
    ped_sigma: float = 50.0
    gain_lo: float = 0.95
    gain_hi: float = 1.05
    noise_sigma: float = 3.0
    cm_sigma: float = 10.0
    photon_adu: float = 150.0
    cloud_sigma: float = 0.2


def _rng(*key: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([1903, 6838, *key])))


def make_calibration(geom: Geometry, cfg_id: int, sim: SimParams = SimParams()):
    """Per-pixel pedestal and gain planes, float32 [T, H, W]."""
    rng = _rng(cfg_id, 0)
    ped = rng.normal(sim.ped_mean, sim.ped_sigma, size=geom.shape).astype(np.float32)
    gain = rng.uniform(sim.gain_lo, sim.gain_hi, size=geom.shape).astype(np.float32)
    return ped, gain


def photon_signal(geom: Geometry, rng: np.random.Generator, occupancy: float,
                  sim: SimParams = SimParams()):
    """Deposited signal (ADU at unit gain, float64 [T,H,W]) and the photon list.

    The photon list is an array of (tile, y, x) float64 rows with y, x the
    continuous impact position inside the tile in pixel pitches.
    """
    T, H, W = geom.shape
    sig = np.zeros(T * H * W, dtype=np.float64)
    counts = rng.poisson(occupancy, size=(T, H, W))
    t, r, c = np.nonzero(counts)
    reps = counts[t, r, c]
    t = np.repeat(t, reps)
    r = np.repeat(r, reps)
    c = np.repeat(c, reps)
    n = t.size
    y = r + rng.uniform(0.0, 1.0, size=n)
    x = c + rng.uniform(0.0, 1.0, size=n)
    if n:
        s = sim.cloud_sigma
        offs = np.arange(-2, 3)
        # fraction of the cloud in each of the 5 rows / 5 columns around the impact pixel
        rr = r[:, None] + offs[None, :]
        cc = c[:, None] + offs[None, :]
        fy = ndtr((rr + 1 - y[:, None]) / s) - ndtr((rr - y[:, None]) / s)
        fx = ndtr((cc + 1 - x[:, None]) / s) - ndtr((cc - x[:, None]) / s)
        frac = fy[:, :, None] * fx[:, None, :]                      # [n,5,5]
        R = np.broadcast_to(rr[:, :, None], frac.shape)
        C = np.broadcast_to(cc[:, None, :], frac.shape)
        Tt = np.broadcast_to(t[:, None, None], frac.shape)
        ok = (R >= 0) & (R < H) & (C >= 0) & (C < W)
        idx = (Tt[ok] * H + R[ok]) * W + C[ok]
        sig += np.bincount(idx, weights=sim.photon_adu * frac[ok], minlength=sig.size)
    photons = np.stack([t.astype(np.float64), y, x], axis=1) if n else np.zeros((0, 3))
    return sig.reshape(T, H, W), photons


def make_frame(geom: Geometry, ped: np.ndarray, gain: np.ndarray, occupancy: float,
               cfg_id: int, occ_id: int, frame_id: int, sim: SimParams = SimParams(),
               return_truth: bool = False):
    """One raw frame, uint16 [T,H,W] (values in [0, 16383])."""
    rng = _rng(cfg_id, occ_id + 1, frame_id)
    T, H, W = geom.shape
    sig, photons = photon_signal(geom, rng, occupancy, sim)
    nb = W // geom.bank_cols
    cm = rng.normal(0.0, sim.cm_sigma, size=(T, H, nb))
    cm_px = np.repeat(cm, geom.bank_cols, axis=2)
    noise = rng.normal(0.0, sim.noise_sigma, size=(T, H, W))
    val = ped.astype(np.float64) + gain.astype(np.float64) * sig + cm_px + noise
    raw = np.clip(np.rint(val), 0, ADC_MAX).astype(np.uint16)
    if return_truth:
        return raw, photons
    return raw


def make_frames(geom: Geometry, ped: np.ndarray, gain: np.ndarray, n_frames: int,
                occupancy: float, cfg_id: int, occ_id: int = 0, first_frame: int = 0,
                sim: SimParams = SimParams()) -> np.ndarray:
    """n_frames raw frames, uint16 [N,T,H,W]."""
    out = np.empty((n_frames, *geom.shape), dtype=np.uint16)
    for i in range(n_frames):
        out[i] = make_frame(geom, ped, gain, occupancy, cfg_id, occ_id, first_frame + i, sim)
    return out


# Occupancy sweep of the CSPAD throughput workload (photons per pixel).
CSPAD_OCCUPANCIES = (0.001, 0.01, 0.05)

# Default thresholds: sigma = 3 ADU, seed at 5 sigma, neighbour mask at 3 sigma,
# 150 ADU per photon.
DEFAULT_PARAMS = dict(sigma=3.0, n_seed=5.0, n_nb=3.0, photon_adu=150.0)


# ---------------------------------------------------------------------------
# Charge-sharing patches for the subpixel stage
# ---------------------------------------------------------------------------
def make_patches(n: int, seed: int, sigma_lo: float = 0.1, sigma_hi: float = 0.4,
                 noise_sigma: float = 3.0, photon_adu: float = 150.0, size: int = 5):
    """Simulated corrected 5x5 patches around single-photon hits.

    Each photon lands at a uniform position inside the central pixel; its
    charge (photon_adu) spreads as a 2-D Gaussian cloud of width
    sigma ~ U(sigma_lo, sigma_hi) px, integrated over the pixel areas of the
    patch, plus N(0, noise_sigma) noise per pixel.

    Returns (patches float32 [n, size, size], truth float32 [n, 2]) where truth
    is (dy, dx) of the impact point relative to the central pixel's centre, in
    pixel pitches, each in [-0.5, 0.5).
    """
    rng = _rng(7, 1, seed)
    h = size // 2
    truth = rng.uniform(-0.5, 0.5, size=(n, 2))
    sig = rng.uniform(sigma_lo, sigma_hi, size=n)
    edges = np.arange(-h, h + 2, dtype=np.float64) - 0.5          # pixel edges around the centre pixel
    out = np.empty((n, size, size), dtype=np.float32)
    chunk = 1 << 18
    for a in range(0, n, chunk):
        b = min(n, a + chunk)
        s = sig[a:b, None]
        cy = ndtr((edges[None, :] - truth[a:b, 0:1]) / s)
        cx = ndtr((edges[None, :] - truth[a:b, 1:2]) / s)
        fy = np.diff(cy, axis=1)
        fx = np.diff(cx, axis=1)
        pat = photon_adu * fy[:, :, None] * fx[:, None, :]
        pat += rng.normal(0.0, noise_sigma, size=pat.shape)
        out[a:b] = pat.astype(np.float32)
    return out, truth.astype(np.float32)


# ---------------------------------------------------------------------------
# Auto-ranging (multi-gain) detectors
# ---------------------------------------------------------------------------
# Gain code of each range in the raw word's bits 14-15 and the invalid code.
GAIN_CODES = {1: ((0, 1, 2), 3),      # ePix10k-like
              2: ((0, 1, 3), 2)}      # Jungfrau-like
# Relative gains of the three ranges (high, medium, low).
RANGE_GAINS = (1.0, 1.0 / 3.0, 1.0 / 100.0)


def make_calibration_multigain(geom: Geometry, cfg_id: int, sim: SimParams = SimParams()):
    """Per-range pedestal and gain planes, float32 [3, T, H, W]."""
    rng = _rng(cfg_id, 50)
    ped = rng.normal(sim.ped_mean, sim.ped_sigma, size=(3, *geom.shape)).astype(np.float32)
    g = rng.uniform(sim.gain_lo, sim.gain_hi, size=(3, *geom.shape))
    gain = (g * np.asarray(RANGE_GAINS)[:, None, None, None]).astype(np.float32)
    return ped, gain


def make_frames_multigain(geom: Geometry, ped: np.ndarray, gain: np.ndarray, n_frames: int, occupancy: float,
                          cfg_id: int, gain_mode: int, range_frac=(0.80, 0.12, 0.06), invalid_frac: float = 0.02,
                          sim: SimParams = SimParams()) -> np.ndarray:
    """n_frames raw words uint16 [N, T, H, W]: every pixel is forced into a
    range drawn with probabilities range_frac (an invalid code with
    probability invalid_frac); its ADC value is that range's pedestal plus
    gain times the signal, bank common mode and noise, clipped to 14 bits."""
    codes, bad = GAIN_CODES[gain_mode]
    T, H, W = geom.shape
    nb = W // geom.bank_cols
    p = np.asarray(list(range_frac) + [invalid_frac], np.float64)
    p = p / p.sum()
    out = np.empty((n_frames, T, H, W), np.uint16)
    for f in range(n_frames):
        rng = _rng(cfg_id, 60 + gain_mode, f)
        sig, _ = photon_signal(geom, rng, occupancy, sim)
        pick = rng.choice(4, size=(T, H, W), p=p)
        r = np.minimum(pick, 2)
        pr = np.take_along_axis(ped.astype(np.float64), r[None], 0)[0]
        gr = np.take_along_axis(gain.astype(np.float64), r[None], 0)[0]
        cm = np.repeat(rng.normal(0.0, sim.cm_sigma, size=(T, H, nb)), geom.bank_cols, axis=2)
        noise = rng.normal(0.0, sim.noise_sigma, size=(T, H, W))
        adc = np.clip(np.rint(pr + gr * sig + cm + noise), 0, ADC_MAX).astype(np.uint16)
        code = np.where(pick == 3, bad, np.asarray(codes)[r]).astype(np.uint16)
        out[f] = adc | (code << np.uint16(14))
    return out
