"""Thin Python binding of libpdc (include/pdc.h): argument marshalling only.

Every function has the C name without the ``pdc_`` prefix and raises
``PdcError`` on a negative status.  Device memory and streams come from
PyTorch (``tensor.data_ptr()``, ``stream.cuda_stream``); all computation runs
in the library's HIP kernels.  There is no fallback: if libpdc.so is missing
or cannot be loaded, importing this module raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# PDC_LIB selects another build of the library (the tracing build, libpdc_phase.so)
LIB_PATH = os.environ.get("PDC_LIB") or os.path.join(_HERE, "libpdc.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("libpdc.so is not built (run `python -m paper_1903_06838_amd.build` or "
                      "__graft_entry__.build()); there is no non-HIP fallback")

_lib = ctypes.CDLL(LIB_PATH)

OK = 0
WARN_TRUNCATED = 1
EINVAL = -1
ENOMEM = -2
EDEVICE = -3
ESTATE = -4
KEEP_CORRECTED = 1
KEEP_MEDIANS = 2

HIT_DTYPE = np.dtype([("frame", "<u4"), ("pixel", "<u4"), ("charge", "<f4"), ("nphot", "<u4")])


class Geometry(ctypes.Structure):
    _fields_ = [("n_tiles", ctypes.c_int32), ("rows", ctypes.c_int32), ("cols", ctypes.c_int32),
                ("bank_cols", ctypes.c_int32), ("gain_mode", ctypes.c_int32)]


class Params(ctypes.Structure):
    _fields_ = [("sigma", ctypes.c_float), ("n_seed", ctypes.c_float), ("n_nb", ctypes.c_float),
                ("photon_adu", ctypes.c_float), ("flags", ctypes.c_uint32), ("cm_mode", ctypes.c_int32),
                ("cm_stages", ctypes.c_int32), ("n_cm", ctypes.c_float)]


CM_MEDIAN = 0
CM_BANK_MEAN = 1
CM_TILE_MEAN = 2


class PdcError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("pdc status %d (%s): %s" % (status, strerror(status), message))
        self.status = status


_P = ctypes.c_void_p
_st = ctypes.c_int32
_sig = {
    "pdc_strerror": (ctypes.c_char_p, [_st]),
    "pdc_last_error": (ctypes.c_char_p, [_P]),
    "pdc_create": (_st, [ctypes.c_int32, ctypes.POINTER(_P)]),
    "pdc_destroy": (_st, [_P]),
    "pdc_check_calibration": (_st, [ctypes.POINTER(Geometry), _P, _P, ctypes.POINTER(Params)]),
    "pdc_calibrate": (_st, [_P, ctypes.POINTER(Geometry), _P, _P, ctypes.POINTER(Params),
                            ctypes.POINTER(ctypes.c_int32)]),
    "pdc_release_detector": (_st, [_P, ctypes.c_int32]),
    "pdc_process_frames": (_st, [_P, ctypes.c_int32, _P, ctypes.c_uint64, ctypes.c_uint64, _P,
                                 ctypes.POINTER(ctypes.c_uint64)]),
    "pdc_get_hits": (_st, [_P, ctypes.c_uint64, _P, ctypes.c_uint64, ctypes.c_int32,
                           ctypes.POINTER(ctypes.c_uint64), _P, _P]),
    "pdc_get_corrected": (_st, [_P, ctypes.c_uint64, _P, ctypes.c_int32]),
    "pdc_release_batch": (_st, [_P, ctypes.c_uint64]),
    "pdc_batch_bytes": (_st, [_P, ctypes.c_int32, ctypes.c_uint64, ctypes.c_uint64, ctypes.POINTER(ctypes.c_uint64)]),
    "pdc_batch_timing": (_st, [_P, ctypes.c_uint64, ctypes.POINTER(ctypes.c_float),
                               ctypes.POINTER(ctypes.c_float)]),
    "pdc_capture_patches": (_st, [_P, ctypes.c_uint64, _P, ctypes.c_uint64, ctypes.POINTER(ctypes.c_uint64)]),
    "pdc_capture_inputs": (_st, [_P, ctypes.c_uint64, ctypes.c_float, _P, ctypes.c_uint64,
                                 ctypes.POINTER(ctypes.c_uint64)]),
    "pdc_mlp_make_inputs": (_st, [_P, _P, ctypes.c_uint64, ctypes.c_float, _P, _P]),
    "pdc_capture_centroids": (_st, [_P, ctypes.c_uint64, ctypes.c_float, _P, ctypes.c_int32, _P, ctypes.c_uint64,
                                    ctypes.c_int32, ctypes.POINTER(ctypes.c_uint64)]),
    "pdc_mlp_infer_inputs": (_st, [_P, _P, ctypes.c_uint64, _P, _P]),
    "pdc_centroid": (_st, [_P, _P, ctypes.c_uint64, ctypes.c_float, _P, ctypes.c_int32, _P, _P]),
    "pdc_eta_table": (_st, [_P, _P, ctypes.c_uint64, ctypes.c_float, ctypes.c_int32, _P, _P, _P]),
    "pdc_mlp_create": (_st, [_P, _P, ctypes.POINTER(_P)]),
    "pdc_mlp_destroy": (_st, [_P]),
    "pdc_mlp_set_params": (_st, [_P, _P]),
    "pdc_mlp_get_params": (_st, [_P, _P]),
    "pdc_mlp_infer": (_st, [_P, _P, ctypes.c_uint64, ctypes.c_float, _P, _P]),
    "pdc_mlp_gradient": (_st, [_P, _P, _P, ctypes.c_uint64, ctypes.c_float, _P,
                               ctypes.POINTER(ctypes.c_double), _P]),
    "pdc_mlp_train_step": (_st, [_P, _P, _P, ctypes.c_uint64, ctypes.c_float, ctypes.c_float, _P]),
    "pdc_mlp_last_loss": (_st, [_P, ctypes.POINTER(ctypes.c_double)]),
    "pdc_debug_mfma_probe": (_st, [_P, _P, _P, _P]),
    "pdc_serve_run": (_st, [_P, _P, ctypes.c_int32, _P, _P]),
    "pdc_accumulate_hits": (_st, [_P, ctypes.c_uint64, _P, _P, _P, ctypes.c_float, ctypes.c_float, ctypes.c_int32,
                                  _P]),
    "pdc_histogram_corrected": (_st, [_P, ctypes.c_uint64, _P, ctypes.c_float, ctypes.c_float, ctypes.c_int32, _P]),
    "pdc_get_invalid_counts": (_st, [_P, ctypes.c_uint64, _P]),
    "pdc_process_mixed": (_st, [_P, _P, ctypes.c_int32, _P, _P]),
    "pdc_autotune": (_st, [_P, ctypes.c_int32, _P, ctypes.c_uint64, ctypes.c_uint64, _P,
                           ctypes.POINTER(ctypes.c_int32), _P]),
    "pdc_autotune_strips": (_st, [_P, ctypes.c_int32, _P, ctypes.c_uint64, ctypes.c_uint64, _P,
                                  ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32), _P,
                                  ctypes.POINTER(ctypes.c_int32)]),
    "pdc_debug_batch_path": (_st, [_P, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int32)]),
    "pdc_dark_stats": (_st, [_P, ctypes.POINTER(Geometry), _P, ctypes.c_uint64, _P, _P, _P]),
    "pdc_calibrate_darks": (_st, [_P, ctypes.POINTER(Geometry), _P, ctypes.c_uint64, _P, ctypes.POINTER(Params), _P,
                                  ctypes.POINTER(ctypes.c_int32)]),
    "pdc_graph_create": (_st, [_P, ctypes.c_int32, _P, ctypes.c_uint64, ctypes.c_uint64, ctypes.POINTER(_P)]),
    "pdc_graph_launch": (_st, [_P, _P, ctypes.POINTER(ctypes.c_uint64)]),
    "pdc_graph_destroy": (_st, [_P]),
    "pdc_graph_create_mixed": (_st, [_P, _P, ctypes.c_int32, ctypes.POINTER(_P)]),
    "pdc_graph_items": (ctypes.c_int32, [_P]),
    "pdc_process_frames_static": (_st, [_P, ctypes.c_int32, _P, ctypes.c_uint64, _P, ctypes.c_uint64, _P, _P, _P,
                                        ctypes.POINTER(ctypes.c_uint64)]),
    "pdc_stream_read": (_st, [_P, _P, ctypes.c_uint64, _P, ctypes.POINTER(ctypes.c_float)]),
    "pdc_debug_serve_batch_len": (_st, [_P, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                                        ctypes.POINTER(ctypes.c_uint64)]),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTED = tuple(_sig)


def strerror(status: int) -> str:
    return _lib.pdc_strerror(status).decode()


def last_error(ctx=None) -> str:
    return (_lib.pdc_last_error(ctx) or b"").decode()


def _check(status, ctx=None):
    if status < 0:
        raise PdcError(status, last_error(ctx))
    return status


def _ptr(x):
    """Address of a numpy array, a torch tensor, or an int."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if isinstance(x, np.ndarray):
        return x.ctypes.data
    return x.data_ptr()


def geometry(n_tiles, rows, cols, bank_cols, gain_mode=0) -> Geometry:
    return Geometry(n_tiles, rows, cols, bank_cols, gain_mode)


def params(sigma=3.0, n_seed=5.0, n_nb=3.0, photon_adu=150.0, flags=0, cm_mode=CM_MEDIAN, cm_stages=1,
           n_cm=3.0) -> Params:
    return Params(sigma, n_seed, n_nb, photon_adu, flags, cm_mode, cm_stages, n_cm)


def create(device: int = 0):
    h = _P()
    _check(_lib.pdc_create(device, ctypes.byref(h)))
    return h.value


def destroy(ctx) -> None:
    _check(_lib.pdc_destroy(ctx))


def check_calibration(geom: Geometry, pedestal: np.ndarray, gain: np.ndarray, prm: Params) -> int:
    """Host-only validation; returns the status (0 = accepted) without raising."""
    ped = np.ascontiguousarray(pedestal, dtype=np.float32)
    g = np.ascontiguousarray(gain, dtype=np.float32)
    return _lib.pdc_check_calibration(ctypes.byref(geom), ped.ctypes.data, g.ctypes.data,
                                      ctypes.byref(prm))


GAIN_SINGLE = 0
GAIN_EPIX10K = 1
GAIN_JUNGFRAU = 2


def calibrate(ctx, geom: Geometry, pedestal: np.ndarray, gain: np.ndarray, prm: Params) -> int:
    """pedestal, gain: float32 [n_tiles, rows, cols], or [3, n_tiles, rows, cols]
    for an auto-ranging gain_mode."""
    ped = np.ascontiguousarray(pedestal, dtype=np.float32)
    g = np.ascontiguousarray(gain, dtype=np.float32)
    n = (3 if geom.gain_mode else 1) * geom.n_tiles * geom.rows * geom.cols
    if ped.size != n or g.size != n:
        raise ValueError("pedestal/gain must hold n_ranges*n_tiles*rows*cols values")
    det = ctypes.c_int32(-1)
    _check(_lib.pdc_calibrate(ctx, ctypes.byref(geom), ped.ctypes.data, g.ctypes.data,
                              ctypes.byref(prm), ctypes.byref(det)), ctx)
    return det.value


def release_detector(ctx, det: int) -> None:
    _check(_lib.pdc_release_detector(ctx, det), ctx)


def process_frames(ctx, det: int, frames_dev, n_frames: int, hit_capacity: int, stream=None) -> int:
    """frames_dev: device uint16 tensor (or address); stream: torch stream, raw handle or None."""
    if stream is not None and not isinstance(stream, int):
        stream = stream.cuda_stream
    b = ctypes.c_uint64(0)
    _check(_lib.pdc_process_frames(ctx, det, _ptr(frames_dev), n_frames, hit_capacity, stream,
                                   ctypes.byref(b)), ctx)
    return b.value


class MixedItem(ctypes.Structure):
    _fields_ = [("det", ctypes.c_int32), ("frames_dev", ctypes.c_void_p), ("n_frames", ctypes.c_uint64),
                ("hit_capacity", ctypes.c_uint64)]


def process_mixed(ctx, items, stream=None) -> list:
    """items: (det, frames_dev, n_frames, hit_capacity) tuples; returns batch ids."""
    arr = (MixedItem * len(items))(*[MixedItem(d, _ptr(f), n, c) for d, f, n, c in items])
    out = (ctypes.c_uint64 * len(items))()
    if stream is not None and not isinstance(stream, int):
        stream = stream.cuda_stream
    _check(_lib.pdc_process_mixed(ctx, arr, len(items), stream, out), ctx)
    return list(out)


def autotune(ctx, det: int, frames_dev, n_frames: int, hit_capacity: int, stream=None):
    """Returns (chosen frame-group multiplier, frame-kernel ms for x1, x2, x4)."""
    m = ctypes.c_int32(0)
    ms = np.zeros(3, np.float32)
    _check(_lib.pdc_autotune(ctx, det, _ptr(frames_dev), n_frames, hit_capacity, _stream(stream), ctypes.byref(m),
                             ms.ctypes.data), ctx)
    return m.value, ms


def autotune_strips(ctx, det: int, frames_dev, n_frames: int, hit_capacity: int, stream=None):
    """Returns (chosen own rows per strip, frame-group multiplier, frame-kernel ms [heights tried][3])."""
    rows, m, n = ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_int32(0)
    ms = np.zeros(9, np.float32)
    _check(_lib.pdc_autotune_strips(ctx, det, _ptr(frames_dev), n_frames, hit_capacity, _stream(stream),
                                    ctypes.byref(rows), ctypes.byref(m), ms.ctypes.data, ctypes.byref(n)), ctx)
    return rows.value, m.value, ms.reshape(3, 3)[:n.value]


def get_hits(ctx, batch: int, n_frames: int, capacity: int | None = None, dst_dev=None):
    """Returns (hits, total, per_frame_hits, per_frame_photons, status).

    Without dst_dev, hits is a host numpy array of HIT_DTYPE; with dst_dev (a
    device tensor of >= capacity*16 bytes) the records are written there and
    hits is None."""
    fh = np.zeros(n_frames, dtype=np.uint32)
    fp = np.zeros(n_frames, dtype=np.uint64)
    total = ctypes.c_uint64(0)
    if capacity is None:
        # first call: learn the total
        _check(_lib.pdc_get_hits(ctx, batch, None, 0, 0, ctypes.byref(total), fh.ctypes.data,
                                 fp.ctypes.data), ctx)
        capacity = total.value
    if dst_dev is not None:
        st = _check(_lib.pdc_get_hits(ctx, batch, _ptr(dst_dev), capacity, 1, ctypes.byref(total),
                                      fh.ctypes.data, fp.ctypes.data), ctx)
        return None, total.value, fh, fp, st
    hits = np.zeros(capacity, dtype=HIT_DTYPE)
    st = _check(_lib.pdc_get_hits(ctx, batch, hits.ctypes.data if capacity else None, capacity, 0,
                                  ctypes.byref(total), fh.ctypes.data, fp.ctypes.data), ctx)
    return hits[:min(capacity, total.value)], total.value, fh, fp, st


def get_corrected(ctx, batch: int, dst) -> None:
    """dst: host float32 numpy array or device float32 tensor of n_frames*T*H*W."""
    is_dev = 0 if isinstance(dst, np.ndarray) else 1
    _check(_lib.pdc_get_corrected(ctx, batch, _ptr(dst), is_dev), ctx)


def get_invalid_counts(ctx, batch: int, n_frames: int) -> np.ndarray:
    out = np.zeros(n_frames, np.uint32)
    _check(_lib.pdc_get_invalid_counts(ctx, batch, out.ctypes.data if n_frames else None), ctx)
    return out


def debug_batch_path(ctx, batch: int) -> int:
    """1: general kernel, 2: persistent kernel."""
    p = ctypes.c_int32(0)
    _check(_lib.pdc_debug_batch_path(ctx, batch, ctypes.byref(p)), ctx)
    return p.value


STATIC_SCRATCH_BYTES = 64 << 20


def process_frames_static(ctx, det: int, frames_dev, n_frames: int, hits_dev, hits_capacity: int,
                          frame_hits_dev, frame_photons_dev, stream=None):
    """pdc_process_frames_static: results in the caller's device tensors, no
    allocation; returns (status, total hits)."""
    total = ctypes.c_uint64(0)
    st = _check(_lib.pdc_process_frames_static(ctx, det, _ptr(frames_dev), n_frames, _ptr(hits_dev), hits_capacity,
                                               _ptr(frame_hits_dev), _ptr(frame_photons_dev), _stream(stream),
                                               ctypes.byref(total)), ctx)
    return st, total.value


def stream_read(ctx, src_dev, nbytes: int, stream=None) -> float:
    """Milliseconds of a plain streaming read of nbytes of device memory."""
    ms = ctypes.c_float(0)
    _check(_lib.pdc_stream_read(ctx, _ptr(src_dev), nbytes, _stream(stream), ctypes.byref(ms)), ctx)
    return ms.value


def debug_serve_batch_len(pending, max_batch: int, pool_frames: int) -> int:
    """Frames the serving loop would launch next for this queue (host only)."""
    a = np.ascontiguousarray(pending, dtype=np.uint64)
    n = ctypes.c_uint64(0)
    _check(_lib.pdc_debug_serve_batch_len(a.ctypes.data if a.size else None, a.size, max_batch, pool_frames,
                                          ctypes.byref(n)))
    return n.value


def release_batch(ctx, batch: int) -> None:
    _check(_lib.pdc_release_batch(ctx, batch), ctx)


def batch_bytes(ctx, det: int, n_frames: int, hit_capacity: int) -> int:
    """Device bytes of a batch of this shape on detector det."""
    b = ctypes.c_uint64(0)
    _check(_lib.pdc_batch_bytes(ctx, det, n_frames, hit_capacity, ctypes.byref(b)), ctx)
    return b.value


def graph_create(ctx, det: int, frames_dev, n_frames: int, hit_capacity: int):
    """Capture a batch of n_frames frames read from frames_dev (device tensor or
    address) into a HIP graph; returns the graph handle."""
    g = _P()
    _check(_lib.pdc_graph_create(ctx, det, _ptr(frames_dev), n_frames, hit_capacity, ctypes.byref(g)), ctx)
    return g.value


def graph_create_mixed(ctx, items):
    """One graph over several detectors' batches; items: (det, frames_dev,
    n_frames, hit_capacity) tuples as for process_mixed."""
    arr = (MixedItem * len(items))(*[MixedItem(d, _ptr(f), n, c) for d, f, n, c in items])
    g = _P()
    _check(_lib.pdc_graph_create_mixed(ctx, arr, len(items), ctypes.byref(g)), ctx)
    return g.value


def graph_launch(ctx, graph, stream=None):
    """Replay the graph on stream (torch stream, raw handle or None); returns a
    batch id, or the list of batch ids (item order) of a mixed graph."""
    n = _lib.pdc_graph_items(graph)
    out = (ctypes.c_uint64 * max(n, 1))()
    _check(_lib.pdc_graph_launch(graph, _stream(stream), out), ctx)
    return out[0] if n == 1 else list(out)


def graph_destroy(ctx, graph) -> None:
    _check(_lib.pdc_graph_destroy(graph), ctx)


def batch_timing(ctx, batch: int):
    a = ctypes.c_float(0)
    t = ctypes.c_float(0)
    _check(_lib.pdc_batch_timing(ctx, batch, ctypes.byref(a), ctypes.byref(t)), ctx)
    return a.value, t.value


# ---------------------------------------------------------------------------
# subpixel stage
# ---------------------------------------------------------------------------
MLP_PARAMS = 5954


def _stream(stream):
    if stream is not None and not isinstance(stream, int):
        return stream.cuda_stream
    return stream


def capture_patches(ctx, batch: int, patches_dev, capacity: int) -> int:
    """5x5 Frames2 patches of the batch's first min(total, capacity) hits; returns the count."""
    n = ctypes.c_uint64(0)
    _check(_lib.pdc_capture_patches(ctx, batch, _ptr(patches_dev), capacity, ctypes.byref(n)), ctx)
    return n.value


MLP_INPUT_WORDS = 32


def capture_inputs(ctx, batch: int, photon_adu: float, inputs_dev, capacity: int) -> int:
    """The network inputs (uint16 [capacity][MLP_INPUT_WORDS]) of the batch's first hits; returns the count."""
    n = ctypes.c_uint64(0)
    _check(_lib.pdc_capture_inputs(ctx, batch, photon_adu, _ptr(inputs_dev), capacity, ctypes.byref(n)), ctx)
    return n.value


def capture_centroids(ctx, batch: int, t_nb: float, positions_dev, capacity: int, eta_dev=None, nbins: int = 0,
                      only_implausible: bool = False) -> int:
    """Centroid (+ eta) positions of the batch's first hits, or the fallback for implausible ones; returns the count."""
    n = ctypes.c_uint64(0)
    _check(_lib.pdc_capture_centroids(ctx, batch, t_nb, _ptr(eta_dev), nbins, _ptr(positions_dev), capacity,
                                      1 if only_implausible else 0, ctypes.byref(n)), ctx)
    return n.value


def mlp_make_inputs(ctx, patches_dev, n: int, photon_adu: float, inputs_dev, stream=None) -> None:
    _check(_lib.pdc_mlp_make_inputs(ctx, _ptr(patches_dev), n, photon_adu, _ptr(inputs_dev), _stream(stream)), ctx)


def centroid(ctx, patches_dev, n: int, t_nb: float, out_dev, eta_dev=None, nbins: int = 0, stream=None) -> None:
    _check(_lib.pdc_centroid(ctx, _ptr(patches_dev), n, t_nb, _ptr(eta_dev), nbins, _ptr(out_dev),
                             _stream(stream)), ctx)


def eta_table(ctx, patches_dev, n: int, t_nb: float, nbins: int, workspace_dev, table_dev, stream=None) -> None:
    _check(_lib.pdc_eta_table(ctx, _ptr(patches_dev), n, t_nb, nbins, _ptr(workspace_dev), _ptr(table_dev),
                              _stream(stream)), ctx)


def mlp_create(ctx, theta: np.ndarray):
    t = np.ascontiguousarray(theta, dtype=np.float32)
    if t.size != MLP_PARAMS:
        raise ValueError("theta must hold %d values" % MLP_PARAMS)
    h = _P()
    _check(_lib.pdc_mlp_create(ctx, t.ctypes.data, ctypes.byref(h)), ctx)
    return h.value


def mlp_destroy(net) -> None:
    _check(_lib.pdc_mlp_destroy(net))


def mlp_set_params(net, theta: np.ndarray) -> None:
    t = np.ascontiguousarray(theta, dtype=np.float32)
    if t.size != MLP_PARAMS:
        raise ValueError("theta must hold %d values" % MLP_PARAMS)
    _check(_lib.pdc_mlp_set_params(net, t.ctypes.data))


def mlp_get_params(net) -> np.ndarray:
    t = np.zeros(MLP_PARAMS, np.float32)
    _check(_lib.pdc_mlp_get_params(net, t.ctypes.data))
    return t


def mlp_infer(net, patches_dev, n: int, photon_adu: float, out_dev, stream=None) -> None:
    _check(_lib.pdc_mlp_infer(net, _ptr(patches_dev), n, photon_adu, _ptr(out_dev), _stream(stream)))


def mlp_infer_inputs(net, inputs_dev, n: int, out_dev, stream=None) -> None:
    _check(_lib.pdc_mlp_infer_inputs(net, _ptr(inputs_dev), n, _ptr(out_dev), _stream(stream)))


def mlp_gradient(net, patches_dev, target_dev, n: int, photon_adu: float, stream=None):
    """Returns (grad float32 [MLP_PARAMS], loss)."""
    g = np.zeros(MLP_PARAMS, np.float32)
    loss = ctypes.c_double(0)
    _check(_lib.pdc_mlp_gradient(net, _ptr(patches_dev), _ptr(target_dev), n, photon_adu, g.ctypes.data,
                                 ctypes.byref(loss), _stream(stream)))
    return g, loss.value


def mlp_train_step(net, patches_dev, target_dev, n: int, photon_adu: float, lr: float, stream=None) -> None:
    _check(_lib.pdc_mlp_train_step(net, _ptr(patches_dev), _ptr(target_dev), n, photon_adu, lr, _stream(stream)))


def mlp_last_loss(net) -> float:
    loss = ctypes.c_double(0)
    _check(_lib.pdc_mlp_last_loss(net, ctypes.byref(loss)))
    return loss.value


def debug_mfma_probe(ctx, a_bits: np.ndarray, b_bits: np.ndarray) -> np.ndarray:
    """D = A B for bf16 bit patterns A uint16 [16][32], B uint16 [32][16]."""
    a = np.ascontiguousarray(a_bits, dtype=np.uint16)
    b = np.ascontiguousarray(b_bits, dtype=np.uint16)
    assert a.shape == (16, 32) and b.shape == (32, 16)
    d = np.zeros((16, 16), np.float32)
    _check(_lib.pdc_debug_mfma_probe(ctx, a.ctypes.data, b.ctypes.data, d.ctypes.data), ctx)
    return d


# ---------------------------------------------------------------------------
# serving loop
# ---------------------------------------------------------------------------
SERVE_PENDING, SERVE_DONE, SERVE_DROPPED = 0, 1, 2
SERVE_FRAME_DTYPE = np.dtype([("arrival_ns", "<u8"), ("launch_ns", "<u8"), ("done_ns", "<u8"), ("hits", "<u4"),
                              ("batch_frames", "<u4"), ("photons", "<u8"), ("status", "<i4"), ("reserved", "<i4")])


class ServeStream(ctypes.Structure):
    _fields_ = [("det", ctypes.c_int32), ("pool_frames", ctypes.c_uint32), ("pool_dev", _P),
                ("pixels_per_frame", ctypes.c_uint64), ("n_frames", ctypes.c_uint64), ("arrival_ns", _P),
                ("hit_fraction", ctypes.c_double), ("results", _P), ("hits", _P),
                ("hits_capacity", ctypes.c_uint64), ("hits_kept", ctypes.c_uint64), ("subpixel", ctypes.c_int32),
                ("photon_adu", ctypes.c_float), ("t_nb", ctypes.c_float), ("positions", _P)]


class ServeConfig(ctypes.Structure):
    _fields_ = [("max_batch", ctypes.c_uint32), ("max_inflight", ctypes.c_uint32), ("max_queue", ctypes.c_uint64),
                ("hbm_budget", ctypes.c_uint64), ("net", _P), ("eta_dev", _P), ("eta_bins", ctypes.c_int32)]


class ServeSummary(ctypes.Structure):
    _fields_ = [("frames_done", ctypes.c_uint64), ("frames_dropped", ctypes.c_uint64), ("batches", ctypes.c_uint64),
                ("peak_bytes", ctypes.c_uint64), ("wall_ns", ctypes.c_uint64)]


SERVE_SUBPIXEL_NONE, SERVE_SUBPIXEL_MLP, SERVE_SUBPIXEL_CENTROID, SERVE_SUBPIXEL_MLP_FALLBACK = 0, 1, 2, 3


def serve_run(ctx, streams, max_batch=64, max_inflight=2, max_queue=0, hbm_budget=0, net=None, eta_dev=None,
              eta_bins=0, return_positions=False):
    """streams: list of dicts with det, pool (device uint16 tensor [P, T, H, W]), arrival_ns (host
    uint64 array), hit_fraction, keep_hits (capacity or 0), and for a subpixel stage subpixel
    (SERVE_SUBPIXEL_*), photon_adu and t_nb.  Returns (results, hits, summary): per stream a
    SERVE_FRAME_DTYPE array and a HIT_DTYPE array (or None); with return_positions, a fourth
    item: per stream float32 [hits_kept, 2] positions of the kept hits (or None)."""
    descs = (ServeStream * len(streams))()
    keep = []
    for d, st in zip(descs, streams):
        arr = np.ascontiguousarray(st["arrival_ns"], dtype=np.uint64)
        res = np.zeros(len(arr), SERVE_FRAME_DTYPE)
        cap = int(st.get("keep_hits", 0))
        hits = np.zeros(cap, HIT_DTYPE) if cap else None
        pool = st["pool"]
        d.det = st["det"]
        d.pool_frames = pool.shape[0]
        d.pool_dev = _ptr(pool)
        d.pixels_per_frame = int(np.prod(pool.shape[1:]))
        d.n_frames = len(arr)
        d.arrival_ns = arr.ctypes.data
        d.hit_fraction = float(st.get("hit_fraction", 0.05))
        d.results = res.ctypes.data
        d.hits = hits.ctypes.data if cap else None
        d.hits_capacity = cap
        d.subpixel = int(st.get("subpixel", SERVE_SUBPIXEL_NONE))
        d.photon_adu = float(st.get("photon_adu", 150.0))
        d.t_nb = float(st.get("t_nb", 9.0))
        pos = np.zeros((cap, 2), np.float32) if (cap and d.subpixel) else None
        d.positions = pos.ctypes.data if pos is not None else None
        keep.append((arr, res, hits, pos))
    cfg = ServeConfig(max_batch, max_inflight, max_queue, hbm_budget, net, _ptr(eta_dev), eta_bins)
    summ = ServeSummary()
    _check(_lib.pdc_serve_run(ctx, descs, len(streams), ctypes.byref(cfg), ctypes.byref(summ)), ctx)
    out_hits = [h[:d.hits_kept] if h is not None else None for (_, _, h, _), d in zip(keep, descs)]
    summary = {f: getattr(summ, f) for f, _ in ServeSummary._fields_}
    if return_positions:
        out_pos = [p[:d.hits_kept] if p is not None else None for (_, _, _, p), d in zip(keep, descs)]
        return [r for _, r, _, _ in keep], out_hits, summary, out_pos
    return [r for _, r, _, _ in keep], out_hits, summary


# ---------------------------------------------------------------------------
# summaries
# ---------------------------------------------------------------------------
def accumulate_hits(ctx, batch: int, count_map_dev=None, spectrum_dev=None, size_spectra_dev=None,
                    lo: float = 0.0, hi: float = 1.0, nbins: int = 1, stream=None) -> None:
    """Add a batch's hits to device uint32 arrays: count map [pixels], charge
    spectrum [nbins + 2], spectra by cloud size [9][nbins + 2] (any may be None)."""
    _check(_lib.pdc_accumulate_hits(ctx, batch, _ptr(count_map_dev), _ptr(spectrum_dev), _ptr(size_spectra_dev),
                                    lo, hi, nbins, _stream(stream)), ctx)


def histogram_corrected(ctx, batch: int, hist_dev, lo: float, hi: float, nbins: int, stream=None) -> None:
    """Add the histogram of a kept batch's Frames2 values to device uint32 [nbins + 2]."""
    _check(_lib.pdc_histogram_corrected(ctx, batch, _ptr(hist_dev), lo, hi, nbins, _stream(stream)), ctx)


def dark_stats(ctx, geom: Geometry, darks_dev, n_frames: int, stream=None):
    """(pedestal, noise) float32 host arrays [n_tiles, rows, cols] from device dark frames."""
    shape = (geom.n_tiles, geom.rows, geom.cols)
    ped = np.zeros(shape, np.float32)
    noise = np.zeros(shape, np.float32)
    _check(_lib.pdc_dark_stats(ctx, ctypes.byref(geom), _ptr(darks_dev), n_frames, ped.ctypes.data,
                               noise.ctypes.data, _stream(stream)), ctx)
    return ped, noise


def calibrate_darks(ctx, geom: Geometry, darks_dev, n_frames: int, gain: np.ndarray, prm: Params):
    """Calibrate from dark frames; returns (detector id, noise float32 [n_tiles, rows, cols])."""
    g = np.ascontiguousarray(gain, dtype=np.float32)
    if g.size != geom.n_tiles * geom.rows * geom.cols:
        raise ValueError("gain must hold n_tiles*rows*cols values")
    noise = np.zeros((geom.n_tiles, geom.rows, geom.cols), np.float32)
    det = ctypes.c_int32(-1)
    _check(_lib.pdc_calibrate_darks(ctx, ctypes.byref(geom), _ptr(darks_dev), n_frames, g.ctypes.data,
                                    ctypes.byref(prm), noise.ctypes.data, ctypes.byref(det)), ctx)
    return det.value, noise
