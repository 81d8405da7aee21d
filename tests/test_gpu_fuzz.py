"""Seeded random cases through the C ABI against the oracles, bit for bit:
geometries (tiles, rows, bank widths from 2 to 512 pixels, one to four banks
per row, so both kernels and every compiled lane layout), thresholds, photon
size, occupancy, Frames2 kept or not, gain modes and common-mode settings.
The case list is fixed by its seed, so a failure names a reproducible case."""
import numpy as np
import pytest

from oracle import cm_mean as M
from oracle import multigain as G
from paper_1903_06838_amd import synth
from tests.helpers import assert_same, oracle_threads

pytestmark = pytest.mark.gpu

BANKS = [2, 6, 8, 30, 64, 94, 96, 100, 128, 130, 150, 194, 208, 210, 256, 300, 512]


def _cases(n=120):
    rng = np.random.default_rng(20261202)
    out = []
    for i in range(n):
        B = int(rng.choice(BANKS))
        nb = int(rng.integers(1, 5))
        while B * nb > 2048:
            nb -= 1
        # mostly short tiles; taller ones give several strips per tile and strips across tile edges
        H = int(rng.integers(1, 50)) if rng.random() < 0.7 else int(rng.integers(50, 130))
        out.append(dict(
            i=i, T=int(rng.integers(1, 4)), H=H, W=B * nb, B=B,
            N=int(rng.integers(1, 4)), occ=float(rng.choice([0.001, 0.02, 0.08])),
            sigma=float(rng.uniform(2.0, 4.0)), n_seed=float(rng.uniform(3.5, 6.0)),
            nb_frac=float(rng.uniform(0.0, 1.0)), E=float(rng.uniform(80.0, 250.0)),
            keep=bool(rng.integers(0, 2)), gm=int(rng.choice([0, 0, 1, 2])), cm=int(rng.choice([0, 0, 1, 2])),
            stages=int(rng.integers(1, 4))))
    return out


CASES = _cases()


@pytest.fixture(scope="module")
def ctx():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1903_06838_amd import pdc

    c = pdc.create(0)
    yield c
    pdc.destroy(c)


@pytest.mark.parametrize("case", CASES, ids=lambda c: "c%02d-T%dH%dW%dB%d-gm%d-cm%d" % (
    c["i"], c["T"], c["H"], c["W"], c["B"], c["gm"], c["cm"]))
def test_random_case_equals_oracle(ctx, case):
    import torch

    from paper_1903_06838_amd import pdc

    c = case
    geom = synth.Geometry(c["T"], c["H"], c["W"], c["B"])
    n_nb = c["n_seed"] * c["nb_frac"]
    seed = 700 + c["i"]
    sim = synth.SimParams(cm_sigma=1.0) if c["cm"] == 2 else synth.SimParams()
    if c["gm"]:
        ped, gain = synth.make_calibration_multigain(geom, seed)
        raw = synth.make_frames_multigain(geom, ped, gain, c["N"], c["occ"], seed, c["gm"], sim=sim)
        want = G.process(raw, ped, gain, c["B"], c["gm"], c["cm"], c["stages"], c["sigma"], c["n_seed"], n_nb,
                         3.0, c["E"], keep_corrected=c["keep"])
    else:
        ped, gain = synth.make_calibration(geom, seed)
        raw = synth.make_frames(geom, ped, gain, c["N"], c["occ"], seed, sim=sim)
        if c["cm"]:
            want = M.process(raw, ped, gain, c["B"], c["cm"], c["stages"], c["sigma"], c["n_seed"], n_nb, 3.0,
                             c["E"], keep_corrected=c["keep"])
        else:
            want = oracle_threads(raw, ped, gain, c["B"], sigma=c["sigma"], n_seed=c["n_seed"], n_nb=n_nb,
                                  photon_adu=c["E"], keep_corrected=c["keep"])
    prm = pdc.params(c["sigma"], c["n_seed"], n_nb, c["E"], pdc.KEEP_CORRECTED if c["keep"] else 0,
                     cm_mode=c["cm"], cm_stages=c["stages"])
    det = pdc.calibrate(ctx, pdc.geometry(*geom.shape, c["B"], c["gm"]), ped, gain, prm)
    try:
        b = pdc.process_frames(ctx, det, torch.from_numpy(raw).cuda(), c["N"], max(1024, raw.size // 8))
        hits, total, fh, fp, _ = pdc.get_hits(ctx, b, c["N"])
        got = dict(hits=hits, total=total, frame_hits=fh, frame_photons=fp)
        if c["keep"]:
            corr = np.empty(raw.shape, np.float32)
            pdc.get_corrected(ctx, b, corr)
            got["corrected"] = corr
        if c["gm"]:
            assert np.array_equal(pdc.get_invalid_counts(ctx, b, c["N"]), want["invalid"])
        pdc.release_batch(ctx, b)
    finally:
        pdc.release_detector(ctx, det)
    assert_same(got, want, corrected=c["keep"])
