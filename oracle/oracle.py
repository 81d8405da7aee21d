"""Python access to the plain C oracle (``pdc_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.  It shares no code
with the GPU library.

The shared object is built with gcc (``-O2 -ffp-contract=off``, no fast-math)
next to the source.  ``build()`` always recompiles; ``load()`` compiles only
if the library is missing or older than its source.  ``load(path=...)`` opens
another build of the same source (the mutation tests compile planted-mistake
copies and open them this way).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "pdc_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
          "-fexcess-precision=standard", "-Wall", "-Wextra"]

HIT_DTYPE = np.dtype([("frame", "<u4"), ("pixel", "<u4"), ("charge", "<f4"), ("nphot", "<u4")])


def compile_oracle(src: str = SRC, out: str = LIB) -> str:
    tmp = out + ".tmp%d" % os.getpid()
    subprocess.run(["gcc", *CFLAGS, "-o", tmp, src, "-lm"], check=True)
    os.replace(tmp, out)
    return out


def build() -> str:
    return compile_oracle()


_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_I32 = ctypes.c_int32
_F = ctypes.c_float


class Oracle:
    """ctypes view of one build of the oracle."""

    def __init__(self, path: str):
        self.path = path
        lib = ctypes.CDLL(path)
        lib.oracle_dark_gain.argtypes = [_P, _P, _P, _I64, _P]
        lib.oracle_dark_gain.restype = None
        lib.oracle_bank_medians.argtypes = [_P, _I32, _I32, _I32, _I32, _P]
        lib.oracle_bank_medians.restype = None
        lib.oracle_common_mode.argtypes = [_P, _I32, _I32, _I32, _I32, _P]
        lib.oracle_common_mode.restype = None
        lib.oracle_find_hits.argtypes = [_P, _I32, _I32, _I32, _F, _F, _F, ctypes.c_uint32,
                                         _P, _I64, _P, _P]
        lib.oracle_find_hits.restype = _I64
        lib.oracle_process.argtypes = [_P, _I64, _I32, _I32, _I32, _I32, _P, _P, _F, _F, _F, _F,
                                       _P, _I64, _P, _P, _P, _P]
        lib.oracle_process.restype = _I64
        self.lib = lib

    # -- single stages -------------------------------------------------------
    def dark_gain(self, raw, dark, gain):
        raw = np.ascontiguousarray(raw, dtype=np.uint16)
        dark = np.ascontiguousarray(dark, dtype=np.float32)
        gain = np.ascontiguousarray(gain, dtype=np.float32)
        assert raw.shape == dark.shape == gain.shape
        out = np.empty(raw.shape, dtype=np.float32)
        self.lib.oracle_dark_gain(raw.ctypes.data, dark.ctypes.data, gain.ctypes.data,
                                  raw.size, out.ctypes.data)
        return out

    def bank_medians(self, frames1, bank_cols):
        f1 = np.ascontiguousarray(frames1, dtype=np.float32)
        T, H, W = f1.shape
        assert W % bank_cols == 0
        out = np.empty((T, H, W // bank_cols), dtype=np.float32)
        self.lib.oracle_bank_medians(f1.ctypes.data, T, H, W, bank_cols, out.ctypes.data)
        return out

    def common_mode(self, frames1, bank_cols):
        f1 = np.ascontiguousarray(frames1, dtype=np.float32)
        T, H, W = f1.shape
        assert W % bank_cols == 0
        out = np.empty_like(f1)
        self.lib.oracle_common_mode(f1.ctypes.data, T, H, W, bank_cols, out.ctypes.data)
        return out

    def find_hits(self, frames2, t_seed, t_nb, photon_adu, frame=0):
        v = np.ascontiguousarray(frames2, dtype=np.float32)
        T, H, W = v.shape
        cap = max(1, ((H + 1) // 2) * ((W + 1) // 2) * T)
        hits = np.empty(cap, dtype=HIT_DTYPE)
        n = ctypes.c_int64(0)
        ph = ctypes.c_uint64(0)
        total = self.lib.oracle_find_hits(v.ctypes.data, T, H, W, t_seed, t_nb, photon_adu,
                                          frame, hits.ctypes.data, cap, ctypes.byref(n),
                                          ctypes.byref(ph))
        assert total == n.value
        return hits[:n.value].copy(), ph.value

    # -- whole batch ---------------------------------------------------------
    def process(self, raw, dark, gain, bank_cols, sigma=3.0, n_seed=5.0, n_nb=3.0,
                photon_adu=150.0, keep_corrected=False, hit_cap=None):
        """raw uint16 [N,T,H,W] -> dict(hits, frame_hits, frame_photons, total[, corrected])."""
        raw = np.ascontiguousarray(raw, dtype=np.uint16)
        N, T, H, W = raw.shape
        dark = np.ascontiguousarray(dark, dtype=np.float32)
        gain = np.ascontiguousarray(gain, dtype=np.float32)
        assert dark.shape == gain.shape == (T, H, W)
        auto_cap = hit_cap is None
        if auto_cap:
            hit_cap = max(1, N * T * ((H + 1) // 2) * ((W + 1) // 2) // 8 + 1024)
        while True:
            hits = np.empty(hit_cap, dtype=HIT_DTYPE)
            n = ctypes.c_int64(0)
            fh = np.empty(N, dtype=np.uint32)
            fp = np.empty(N, dtype=np.uint64)
            corr = np.empty(raw.shape, dtype=np.float32) if keep_corrected else None
            total = self.lib.oracle_process(
                raw.ctypes.data, N, T, H, W, bank_cols, dark.ctypes.data, gain.ctypes.data,
                sigma, n_seed, n_nb, photon_adu, hits.ctypes.data, hit_cap, ctypes.byref(n),
                fh.ctypes.data, fp.ctypes.data, corr.ctypes.data if corr is not None else None)
            if auto_cap and total > n.value:
                hit_cap = int(total)     # the first capacity was a guess: run again
                continue
            break
        out = dict(hits=hits[:n.value].copy(), frame_hits=fh, frame_photons=fp, total=int(total))
        if corr is not None:
            out["corrected"] = corr
        return out


_default = None


def load(path: str | None = None) -> Oracle:
    global _default
    if path is not None:
        return Oracle(path)
    if _default is None:
        if (not os.path.exists(LIB)) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            compile_oracle()
        _default = Oracle(LIB)
    return _default
