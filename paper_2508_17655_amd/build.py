"""Build libgsb.so (gfx950), and the measurement library libgsb_probe.so, in-tree with hipcc.

    python -m paper_2508_17655_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libgsb.so")
PROBE_LIB = os.path.join(HERE, "libgsb_probe.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

# Packed-FP32 instructions are disabled for all device code; contraction is off so the
# binary32 update is evaluated exactly as written.
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-ffp-contract=off"]


def build(verbose: bool = False) -> str:
    objs = []
    common = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Wall", "-Wno-unused-result"]
    for src, extra in (("gsb_kernels.hip", DEVICE_FLAGS), ("gsb_steps_rj.hip", DEVICE_FLAGS),
                       ("gsb_steps_ws.hip", DEVICE_FLAGS),
                       ("gsb_api.cpp", ["-ffp-contract=off"]), ("gsb_batch.cpp", ["-ffp-contract=off"])):
        obj = os.path.join(CSRC, src + ".o")
        cmd = [HIPCC, *common, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
        if src.endswith(".cpp"):
            cmd = [HIPCC, "-x", "hip", *common, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            sys.stderr.write(r.stdout + r.stderr)
            raise RuntimeError(f"hipcc failed on {src}")
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc link failed")
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    # the device-ceiling probes: a library of their own, not part of the product's
    obj = os.path.join(CSRC, "gsb_probe.hip.o")
    tmp = PROBE_LIB + ".tmp"
    for cmd in ([HIPCC, *common, *DEVICE_FLAGS, "-c", os.path.join(CSRC, "gsb_probe.hip"), "-o", obj],
                [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", obj, "-o", tmp]):
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            sys.stderr.write(r.stdout + r.stderr)
            raise RuntimeError("hipcc failed on gsb_probe.hip")
    os.replace(tmp, PROBE_LIB)
    os.remove(obj)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
