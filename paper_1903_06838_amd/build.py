"""Compile libpdc.so (HIP for gfx950 + host runtime) in-tree with hipcc.

    python -m paper_1903_06838_amd.build

Flags:
  --offload-arch=gfx950         MI355X only
  -ffp-contract=off             no FMA contraction: every binary32 operation
                                rounds on its own (bit-exact contract)
  -fhip-fp32-correctly-rounded-divide-sqrt
                                IEEE division for the photon count
  -Xclang -target-feature -Xclang -packed-fp32-ops
                                no packed FP32 instructions are generated
  -mllvm -amdgpu-mfma-vgpr-form MFMA results in ordinary VGPRs, so that the
                                network kernels feed one layer's results to
                                the next without copies out of AGPRs
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libpdc.so")
# PDC_PHASE_TIMERS=1: the tracing build, with per-phase cycle counters in the
# persistent kernel (same results), as libpdc_phase.so beside the product library
PHASE_LIB = os.path.join(PKG, "libpdc_phase.so")

SOURCES = ["pdc_kernels.hip", "pdc_frame_v2.hip", "pdc_subpixel.hip", "pdc_summary.hip", "pdc_cmmean.hip", "pdc_runtime.cpp", "pdc_serve.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off", "-fhip-fp32-correctly-rounded-divide-sqrt",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-mllvm", "-amdgpu-mfma-vgpr-form",
    "-Wall", "-Wno-unused-function",
    "-I", INCLUDE, "-I", CSRC,
]


def build(verbose: bool = False, phase_timers: bool = False) -> str:
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    out = PHASE_LIB if phase_timers else LIB
    tmp = out + ".tmp%d" % os.getpid()
    cmd = [HIPCC, *FLAGS, *(["-DPDC_PHASE_TIMERS"] if phase_timers else []), "-o", tmp, *srcs]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed building libpdc.so")
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True, phase_timers=os.environ.get("PDC_PHASE_TIMERS") == "1"))
