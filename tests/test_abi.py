"""C ABI checks that need no GPU: the library loads and exports every function
include/pdc.h declares, host-side validation accepts exactly the documented
ranges, and error paths return the documented status without touching a
device."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "pdc.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pdc_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def pdc():
    from paper_1903_06838_amd import pdc as mod
    return mod


def test_exports_every_declared_symbol(pdc):
    names = _declared()
    assert len(names) >= 12
    lib = ctypes.CDLL(pdc.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(pdc.EXPORTED)


def test_strerror(pdc):
    for st in (pdc.OK, pdc.WARN_TRUNCATED, pdc.EINVAL, pdc.ENOMEM, pdc.EDEVICE, pdc.ESTATE):
        assert pdc.strerror(st)
    assert pdc.strerror(1234) == "unknown status"


def _valid(T=2, H=6, W=8, B=4):
    geom_args = (T, H, W, B)
    rng = np.random.default_rng(0)
    ped = rng.normal(1500, 50, size=(T, H, W)).astype(np.float32)
    gain = rng.uniform(0.95, 1.05, size=(T, H, W)).astype(np.float32)
    return geom_args, ped, gain


def test_check_calibration_accepts_valid(pdc):
    g, ped, gain = _valid()
    assert pdc.check_calibration(pdc.geometry(*g), ped, gain, pdc.params()) == pdc.OK
    assert pdc.check_calibration(pdc.geometry(*g), ped, gain, pdc.params(flags=pdc.KEEP_CORRECTED)) == pdc.OK
    assert pdc.check_calibration(pdc.geometry(*g), ped, gain, pdc.params(flags=pdc.KEEP_MEDIANS)) == pdc.OK
    assert pdc.check_calibration(pdc.geometry(*g), ped, gain,
                                 pdc.params(flags=pdc.KEEP_CORRECTED | pdc.KEEP_MEDIANS)) == pdc.OK
    # edges of the documented ranges
    ped2 = ped.copy()
    ped2[0, 0, 0] = 0.0
    ped2[0, 0, 1] = 2.0 ** 24
    ped2[0, 0, 2] = -(2.0 ** -64)
    gain2 = gain.copy()
    gain2[0, 0, 0] = 2.0 ** -24
    gain2[0, 0, 1] = 2.0 ** 24
    assert pdc.check_calibration(pdc.geometry(*g), ped2, gain2, pdc.params()) == pdc.OK
    assert pdc.check_calibration(pdc.geometry(1, 1, 1, 1), np.zeros(1, np.float32),
                                 np.ones(1, np.float32), pdc.params()) == pdc.OK
    assert pdc.check_calibration(pdc.geometry(1, 2, 2048, 1024), np.zeros(4096, np.float32),
                                 np.ones(4096, np.float32), pdc.params(n_seed=0.0, n_nb=0.0)) == pdc.OK


BAD_GEOM = [(0, 6, 8, 4), (2, 0, 8, 4), (2, 6, 0, 4), (2, 6, 8, 0), (2, 6, 8, 3), (2, 6, 8, 16),
            (1, 2, 4096, 128), (1, 2, 2048, 2048), (40000, 40000, 2, 2)]


@pytest.mark.parametrize("g", BAD_GEOM)
def test_check_calibration_rejects_geometry(pdc, g):
    n = max(1, min(g[0] * g[1] * g[2], 64))
    st = pdc.check_calibration(pdc.geometry(*g), np.zeros(n, np.float32), np.ones(n, np.float32), pdc.params())
    assert st == pdc.EINVAL
    assert pdc.last_error()


def test_check_calibration_rejects_gain_mode(pdc):
    g, ped, gain = _valid()
    assert pdc.check_calibration(pdc.geometry(*g, gain_mode=1), ped, gain, pdc.params()) == pdc.EINVAL


BAD_PARAMS = [dict(sigma=0.0), dict(sigma=-1.0), dict(sigma=math.nan), dict(sigma=math.inf),
              dict(n_seed=-1.0), dict(n_nb=math.nan), dict(n_seed=3.0, n_nb=5.0),
              dict(photon_adu=0.0), dict(photon_adu=2.0 ** 25), dict(photon_adu=math.nan),
              dict(flags=4), dict(flags=8), dict(sigma=3e38, n_seed=5.0)]


@pytest.mark.parametrize("kw", BAD_PARAMS, ids=lambda k: str(k))
def test_check_calibration_rejects_params(pdc, kw):
    g, ped, gain = _valid()
    assert pdc.check_calibration(pdc.geometry(*g), ped, gain, pdc.params(**kw)) == pdc.EINVAL


BAD_PLANES = [("ped", math.nan), ("ped", math.inf), ("ped", 2.0 ** 25), ("ped", 1e-30),
              ("ped", -1e-38), ("gain", 0.0), ("gain", -1.0), ("gain", math.nan), ("gain", math.inf),
              ("gain", 2.0 ** -25), ("gain", 2.0 ** 25)]


@pytest.mark.parametrize("which,val", BAD_PLANES, ids=lambda x: str(x))
def test_check_calibration_rejects_planes(pdc, which, val):
    g, ped, gain = _valid()
    (ped if which == "ped" else gain)[1, 2, 3] = val
    assert pdc.check_calibration(pdc.geometry(*g), ped, gain, pdc.params()) == pdc.EINVAL
    assert "[%d]" % ((1 * 6 + 2) * 8 + 3) in pdc.last_error()


def test_null_context_paths(pdc):
    lib = pdc._lib
    b = ctypes.c_uint64(0)
    assert lib.pdc_destroy(None) == pdc.OK
    assert lib.pdc_process_frames(None, 0, None, 0, 0, None, ctypes.byref(b)) == pdc.EINVAL
    assert lib.pdc_get_hits(None, 1, None, 0, 0, None, None, None) == pdc.EINVAL
    assert lib.pdc_get_corrected(None, 1, None, 0) == pdc.EINVAL
    assert lib.pdc_release_batch(None, 1) == pdc.EINVAL
    assert lib.pdc_release_detector(None, 0) == pdc.EINVAL
    assert lib.pdc_batch_timing(None, 1, None, None) == pdc.EINVAL
    assert lib.pdc_calibrate(None, None, None, None, None, None) == pdc.EINVAL
    assert lib.pdc_create(0, None) == pdc.EINVAL
    assert lib.pdc_accumulate_hits(None, 1, None, None, None, 0.0, 1.0, 1, None) == pdc.EINVAL
    assert lib.pdc_histogram_corrected(None, 1, None, 0.0, 1.0, 1, None) == pdc.EINVAL
    assert lib.pdc_dark_stats(None, None, None, 2, None, None, None) == pdc.EINVAL
    assert lib.pdc_calibrate_darks(None, None, None, 2, None, None, None, None) == pdc.EINVAL
    assert lib.pdc_graph_create(None, 0, None, 1, 0, None) == pdc.EINVAL
    assert lib.pdc_graph_launch(None, None, ctypes.byref(b)) == pdc.EINVAL
    assert lib.pdc_graph_destroy(None) == pdc.OK
    assert lib.pdc_graph_create_mixed(None, None, 1, None) == pdc.EINVAL
    assert lib.pdc_graph_items(None) == 0
    assert lib.pdc_stream_read(None, None, 16, None, None) == pdc.EINVAL
    assert lib.pdc_capture_inputs(None, 1, 150.0, None, 0, None) == pdc.EINVAL
    assert lib.pdc_capture_centroids(None, 1, 9.0, None, 0, None, 0, 0, None) == pdc.EINVAL
    assert lib.pdc_mlp_make_inputs(None, None, 0, 150.0, None, None) == pdc.EINVAL
    assert lib.pdc_mlp_infer_inputs(None, None, 0, None, None) == pdc.EINVAL
    assert lib.pdc_autotune_strips(None, 0, None, 1, 0, None, None, None, None, None) == pdc.EINVAL


def test_create_without_gpu_is_edevice(pdc):
    import torch

    if torch.cuda.device_count() > 0:
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    assert pdc._lib.pdc_create(0, ctypes.byref(h)) == pdc.EDEVICE
    assert h.value is None


@pytest.mark.parametrize("pending,max_batch,pool,want", [
    ([], 8, 4, 0),
    ([0, 1, 2], 8, 16, 3),
    ([0, 1, 2], 2, 16, 2),            # at most max_batch
    ([3, 5], 8, 3, 1),                # frame 4 was dropped: the gap ends the run
    ([2, 3, 6, 7], 8, 16, 2),
    ([3, 4, 5, 6], 8, 5, 2),          # pool frames 3, 4, then the pool wraps
    ([5, 6, 7], 8, 5, 3),             # frame 5 is pool frame 0
])
def test_serve_batch_is_a_run_of_consecutive_frames(pdc, pending, max_batch, pool, want):
    """The serving loop launches the consecutive frames at the front of its
    queue: a frame dropped on arrival (queue full) leaves a gap that must end
    the batch, or the dropped frame would be processed in place of the one
    after the gap."""
    assert pdc.debug_serve_batch_len(pending, max_batch, pool) == want


def test_serve_batch_len_rejects_unordered(pdc):
    with pytest.raises(pdc.PdcError):
        pdc.debug_serve_batch_len([3, 3], 8, 16)
    with pytest.raises(pdc.PdcError):
        pdc.debug_serve_batch_len([4, 2], 8, 16)
