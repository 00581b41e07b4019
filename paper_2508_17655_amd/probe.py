"""ctypes binding of libgsb_probe.so (include/gsb_probe.h): this device's measured ceilings.
Marshalling only; the probes are kernels in csrc/gsb_probe.hip."""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgsb_probe.so")
SYMBOLS = ("gsb_probe_ceilings",)
CEILING_NAMES = ("mfma_fp8_flops", "mfma_fp4xfp8_flops", "mfma_int8_ops", "mfma_bf16_flops", "mfma_fp32_flops",
                 "read_l2_2MiB_Bps", "read_mall_64MiB_Bps", "read_hbm_2GiB_Bps", "write_hbm_2GiB_Bps", "shader_clock_hz",
                 "mfma_fp8_32x32_flops", "mfma_int8_32x32_ops", "mfma_bf16_32x32_flops",
                 "coissue_mfma_only_ms", "coissue_valu_only_ms", "coissue_both_ms")
_lib = None


def load_library(path: str = LIB_PATH):
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is missing: build it with python -m paper_2508_17655_amd.build")
        # PyTorch ships its own HIP runtime under the system runtime's soname: load it first
        # so that this library binds to the same runtime as libgsb and PyTorch (two runtimes
        # in one process do not share the device)
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        lib = ctypes.CDLL(path)
        lib.gsb_probe_ceilings.restype = ctypes.c_int32
        lib.gsb_probe_ceilings.argtypes = [ctypes.c_void_p, ctypes.c_int32]
        _lib = lib
    return _lib


def device_ceilings() -> dict:
    """This device's measured MFMA rates, bandwidths, clock and MFMA/VALU sharing."""
    out = np.zeros(len(CEILING_NAMES), dtype=np.float64)
    rc = load_library().gsb_probe_ceilings(out.ctypes.data_as(ctypes.c_void_p), out.size)
    if rc != 0:
        raise RuntimeError(f"gsb_probe_ceilings failed with HIP error {rc}")
    return dict(zip(CEILING_NAMES, (float(v) for v in out)))
