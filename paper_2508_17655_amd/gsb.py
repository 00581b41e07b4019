"""ctypes binding of libgsb (include/gsb.h) -- argument marshalling only.

Every function carries the name of the C entry point it calls.  All computation of the
method happens in the library's gfx950 kernels; this module never falls back to host
arithmetic and raises when the library is missing.

``GSB`` is a convenience wrapper that gives the library a PyTorch-owned device workspace
and PyTorch's current HIP stream (PyTorch is used for device memory and streams only).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libgsb.so")

# enums of gsb.h
GSB_OK, GSB_EINVAL, GSB_ENOTSYM, GSB_EDIAG, GSB_ENONFINITE = 0, -1, -2, -3, -4
GSB_ENOMEM, GSB_EDEVICE, GSB_ESTATE, GSB_EUNSUPPORTED = -5, -6, -7, -8
GSB_BSB, GSB_DSB, GSB_GBSB, GSB_GDSB = 0, 1, 2, 3
GSB_SCHED_LINEAR, GSB_SCHED_CONSTANT = 0, 1
GSB_PREC_FP32, GSB_PREC_BF16X2, GSB_PREC_FP8, GSB_PREC_FIX16 = 0, 1, 2, 3
GSB_INIT_X, GSB_INIT_XY, GSB_INIT_PM01, GSB_INIT_PAIRS = 0, 1, 2, 3
(GSB_OPT_C, GSB_OPT_PRECISION, GSB_OPT_INIT_MODE, GSB_OPT_LAMBDA_MAX, GSB_OPT_LAMBDA_MIN, GSB_OPT_N,
 GSB_OPT_STEP, GSB_OPT_REPLICAS, GSB_OPT_DT_STABLE, GSB_OPT_N_DYN, GSB_OPT_STEP_KERNEL,
 GSB_OPT_GRID_PAD, GSB_OPT_LLE_FROM) = range(13)

(GSB_BATCH_C, GSB_BATCH_DT, GSB_BATCH_LAMBDA_MAX, GSB_BATCH_LAMBDA_MIN, GSB_BATCH_TILE_ROWS, GSB_BATCH_STEP_US,
 GSB_BATCH_N, GSB_BATCH_GRAPH, GSB_BATCH_INIT_MODE, GSB_BATCH_COUNT, GSB_BATCH_REPLICAS, GSB_BATCH_GRID,
 GSB_BATCH_OCCUPANCY) = range(13)

VARIANTS = {"bsb": GSB_BSB, "dsb": GSB_DSB, "gbsb": GSB_GBSB, "gsb": GSB_GBSB, "gdsb": GSB_GDSB}
PRECISIONS = {"fp32": GSB_PREC_FP32, "bf16x2": GSB_PREC_BF16X2, "fp8": GSB_PREC_FP8, "fix16": GSB_PREC_FIX16}

STATUS_NAMES = {0: "GSB_OK", -1: "GSB_EINVAL", -2: "GSB_ENOTSYM", -3: "GSB_EDIAG", -4: "GSB_ENONFINITE",
                -5: "GSB_ENOMEM", -6: "GSB_EDEVICE", -7: "GSB_ESTATE", -8: "GSB_EUNSUPPORTED"}

# Every symbol include/gsb.h declares.
SYMBOLS = ("gsb_create", "gsb_destroy", "gsb_set", "gsb_get", "gsb_set_stream", "gsb_workspace_size",
           "gsb_bind_workspace", "gsb_init", "gsb_step", "gsb_run", "gsb_run_noalloc", "gsb_energy", "gsb_best", "gsb_spins",
           "gsb_state", "gsb_set_state", "gsb_state_device", "gsb_set_state_device", "gsb_delta",
           "gsb_lle_workspace_size", "gsb_lle", "gsb_vjp", "gsb_vjp_device", "gsb_last_step_ms",
           "gsb_batch_create", "gsb_batch_destroy", "gsb_batch_set_stream", "gsb_batch_workspace_size",
           "gsb_batch_bind_workspace", "gsb_batch_set_coupling", "gsb_batch_set", "gsb_batch_get", "gsb_batch_autotune",
           "gsb_batch_run", "gsb_batch_energy", "gsb_batch_best", "gsb_batch_state", "gsb_batch_last_ms",
           "gsb_batch_plan", "gsb_encode_operand", "gsb_last_error", "gsb_version")


class GsbError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libgsb.so and declare the signatures of every entry point."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"libgsb.so is not built ({path}); run `python -m paper_2508_17655_amd.build`")
    # PyTorch ships its own HIP runtime with the same soname as the system one.  Loading
    # PyTorch first makes libgsb bind to that runtime, so streams and device memory handed
    # over from PyTorch belong to the runtime the library calls.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    vp, i32, u64, dbl, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint64, ctypes.c_double, ctypes.c_size_t
    sig = {
        "gsb_create": (i32, [vp, vp, i32, ctypes.POINTER(vp)]),
        "gsb_destroy": (None, [vp]),
        "gsb_set": (i32, [vp, i32, dbl]),
        "gsb_get": (i32, [vp, i32, ctypes.POINTER(dbl)]),
        "gsb_set_stream": (i32, [vp, vp]),
        "gsb_workspace_size": (i32, [vp, i32, i32, ctypes.POINTER(sz)]),
        "gsb_bind_workspace": (i32, [vp, vp, sz]),
        "gsb_init": (i32, [vp, i32, i32, dbl, dbl, i32, i32, u64]),
        "gsb_step": (i32, [vp, i32]),
        "gsb_run": (i32, [vp, i32, i32, dbl, dbl, i32, i32, u64]),
        "gsb_run_noalloc": (i32, [vp, i32, i32, dbl, dbl, i32, i32, u64, vp, vp]),
        "gsb_energy": (i32, [vp, vp]),
        "gsb_best": (i32, [vp, vp, ctypes.POINTER(dbl), ctypes.POINTER(i32)]),
        "gsb_spins": (i32, [vp, vp]),
        "gsb_state": (i32, [vp, vp, vp, vp, ctypes.POINTER(i32)]),
        "gsb_set_state": (i32, [vp, vp, vp, vp, i32]),
        "gsb_state_device": (i32, [vp, vp, vp, vp, ctypes.POINTER(i32)]),
        "gsb_set_state_device": (i32, [vp, vp, vp, vp, i32]),
        "gsb_delta": (i32, [vp, vp]),
        "gsb_lle_workspace_size": (i32, [vp, i32, i32, ctypes.POINTER(sz)]),
        "gsb_lle": (i32, [vp, i32, i32, dbl, vp, dbl, i32, i32, u64, u64, i32, vp, vp]),
        "gsb_vjp": (i32, [vp, i32, vp, vp, vp]),
        "gsb_vjp_device": (i32, [vp, i32, vp, vp, vp]),
        "gsb_last_step_ms": (i32, [vp, ctypes.POINTER(dbl)]),
        "gsb_batch_create": (i32, [i32, vp, i32, ctypes.POINTER(vp)]),
        "gsb_batch_destroy": (None, [vp]),
        "gsb_batch_set_stream": (i32, [vp, vp]),
        "gsb_batch_workspace_size": (i32, [vp, ctypes.POINTER(sz)]),
        "gsb_batch_bind_workspace": (i32, [vp, vp, sz]),
        "gsb_batch_set_coupling": (i32, [vp, i32, vp, dbl, dbl]),
        "gsb_batch_set": (i32, [vp, i32, i32, dbl]),
        "gsb_batch_get": (i32, [vp, i32, i32, ctypes.POINTER(dbl)]),
        "gsb_batch_autotune": (i32, [vp, i32, dbl, i32, u64]),
        "gsb_batch_run": (i32, [vp, i32, dbl, i32, u64]),
        "gsb_batch_energy": (i32, [vp, i32, vp]),
        "gsb_batch_best": (i32, [vp, vp, vp]),
        "gsb_batch_state": (i32, [vp, i32, vp, vp, vp]),
        "gsb_batch_last_ms": (i32, [vp, ctypes.POINTER(dbl)]),
        "gsb_batch_plan": (i32, [i32, vp, vp, vp, i32, i32, vp, vp]),
        "gsb_encode_operand": (i32, [i32, i32, vp, ctypes.c_int64, vp, vp]),
        "gsb_last_error": (ctypes.c_char_p, []),
        "gsb_version": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _check(status: int, where: str):
    if status != GSB_OK:
        raise GsbError(status, where, gsb_last_error())


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def gsb_last_error() -> str:
    return load_library().gsb_last_error().decode()


def gsb_version() -> str:
    return load_library().gsb_version().decode()


def gsb_create(J: np.ndarray, h: np.ndarray | None = None):
    J = np.ascontiguousarray(J, dtype=np.float32)
    if J.ndim != 2 or J.shape[0] != J.shape[1]:
        raise ValueError("J must be a square matrix")
    hh = None if h is None else np.ascontiguousarray(h, dtype=np.float32)
    out = ctypes.c_void_p()
    _check(load_library().gsb_create(_ptr(J), None if hh is None else _ptr(hh), J.shape[0], ctypes.byref(out)),
           "gsb_create")
    return out


def gsb_destroy(ctx) -> None:
    load_library().gsb_destroy(ctx)


def gsb_set(ctx, option: int, value: float) -> None:
    _check(load_library().gsb_set(ctx, option, float(value)), "gsb_set")


def gsb_get(ctx, option: int) -> float:
    v = ctypes.c_double()
    _check(load_library().gsb_get(ctx, option, ctypes.byref(v)), "gsb_get")
    return v.value


def gsb_set_stream(ctx, stream: int | None) -> None:
    _check(load_library().gsb_set_stream(ctx, ctypes.c_void_p(stream or 0)), "gsb_set_stream")


def gsb_workspace_size(ctx, replicas: int, steps: int) -> int:
    v = ctypes.c_size_t()
    _check(load_library().gsb_workspace_size(ctx, replicas, steps, ctypes.byref(v)), "gsb_workspace_size")
    return v.value


def gsb_bind_workspace(ctx, device_ptr: int | None, nbytes: int) -> None:
    _check(load_library().gsb_bind_workspace(ctx, ctypes.c_void_p(device_ptr or 0), nbytes), "gsb_bind_workspace")


def gsb_init(ctx, variant: int, schedule: int, control_strength: float, dt: float, replicas: int, steps: int,
             seed: int) -> None:
    _check(load_library().gsb_init(ctx, variant, schedule, control_strength, dt, replicas, steps,
                                   seed & (2**64 - 1)), "gsb_init")


def gsb_step(ctx, count: int) -> None:
    _check(load_library().gsb_step(ctx, count), "gsb_step")


def gsb_run(ctx, variant: int, schedule: int, control_strength: float, dt: float, replicas: int, steps: int,
            seed: int) -> None:
    _check(load_library().gsb_run(ctx, variant, schedule, control_strength, dt, replicas, steps,
                                  seed & (2**64 - 1)), "gsb_run")


def gsb_run_noalloc(ctx, variant: int, schedule: int, control_strength: float, dt: float, replicas: int,
                    steps: int, seed: int, x_ptr: int, energies_ptr: int) -> None:
    """x_ptr, energies_ptr: device addresses (replicas * n_dyn binary32, replicas doubles)."""
    _check(load_library().gsb_run_noalloc(ctx, variant, schedule, control_strength, dt, replicas, steps,
                                          seed & (2**64 - 1), x_ptr, energies_ptr), "gsb_run_noalloc")


def gsb_energy(ctx) -> np.ndarray:
    R = int(gsb_get(ctx, GSB_OPT_REPLICAS))
    E = np.empty(R, dtype=np.float64)
    _check(load_library().gsb_energy(ctx, _ptr(E)), "gsb_energy")
    return E


def gsb_best(ctx):
    n = int(gsb_get(ctx, GSB_OPT_N))
    s = np.empty(n, dtype=np.int8)
    e = ctypes.c_double()
    r = ctypes.c_int32()
    _check(load_library().gsb_best(ctx, _ptr(s), ctypes.byref(e), ctypes.byref(r)), "gsb_best")
    return s, e.value, r.value


def gsb_spins(ctx) -> np.ndarray:
    R = int(gsb_get(ctx, GSB_OPT_REPLICAS))
    n = int(gsb_get(ctx, GSB_OPT_N))
    s = np.empty((R, n), dtype=np.int8)
    _check(load_library().gsb_spins(ctx, _ptr(s)), "gsb_spins")
    return s


def gsb_state(ctx):
    R = int(gsb_get(ctx, GSB_OPT_REPLICAS))
    n = int(gsb_get(ctx, GSB_OPT_N_DYN))
    x = np.empty((R, n), dtype=np.float32)
    y = np.empty((R, n), dtype=np.float32)
    p = np.empty((R, n), dtype=np.float32)
    m = ctypes.c_int32()
    _check(load_library().gsb_state(ctx, _ptr(x), _ptr(y), _ptr(p), ctypes.byref(m)), "gsb_state")
    return x, y, p, m.value


def gsb_set_state(ctx, x: np.ndarray, y: np.ndarray, p: np.ndarray, m: int) -> None:
    x = np.ascontiguousarray(x, dtype=np.float32)
    y = np.ascontiguousarray(y, dtype=np.float32)
    p = np.ascontiguousarray(p, dtype=np.float32)
    _check(load_library().gsb_set_state(ctx, _ptr(x), _ptr(y), _ptr(p), m), "gsb_set_state")


def _device_arrays(ctx, *ts):
    """Device pointers of float32 tensors [replicas, n_dyn], contiguous, on a GPU."""
    R = int(gsb_get(ctx, GSB_OPT_REPLICAS))
    n = int(gsb_get(ctx, GSB_OPT_N_DYN))
    out = []
    for t in ts:
        if not t.is_cuda or t.dtype.itemsize != 4 or not t.dtype.is_floating_point:
            raise ValueError("device state arrays must be float32 tensors on the GPU")
        if tuple(t.shape) != (R, n) or not t.is_contiguous():
            raise ValueError(f"device state arrays must be contiguous [{R}, {n}]")
        out.append(ctypes.c_void_p(t.data_ptr()))
    return out


def gsb_state_device(ctx, x, y, p) -> int:
    """The current state into float32 tensors x, y, p [replicas, n_dyn] on the device; returns m."""
    m = ctypes.c_int32()
    _check(load_library().gsb_state_device(ctx, *_device_arrays(ctx, x, y, p), ctypes.byref(m)), "gsb_state_device")
    return m.value


def gsb_set_state_device(ctx, x, y, p, m: int) -> None:
    _check(load_library().gsb_set_state_device(ctx, *_device_arrays(ctx, x, y, p), m), "gsb_set_state_device")


def gsb_vjp_device(ctx, count: int, xb, yb, pb) -> None:
    """gsb_vjp on float32 tensors [replicas, n_dyn] on the device, overwritten in place."""
    _check(load_library().gsb_vjp_device(ctx, count, *_device_arrays(ctx, xb, yb, pb)), "gsb_vjp_device")


def gsb_delta(ctx) -> np.ndarray:
    R = int(gsb_get(ctx, GSB_OPT_REPLICAS))
    out = np.empty(max(R // 2, 1), dtype=np.float64)
    _check(load_library().gsb_delta(ctx, _ptr(out)), "gsb_delta")
    return out[: R // 2]


def gsb_lle_workspace_size(ctx, replicas: int, steps: int) -> int:
    v = ctypes.c_size_t()
    _check(load_library().gsb_lle_workspace_size(ctx, replicas, steps, ctypes.byref(v)), "gsb_lle_workspace_size")
    return v.value


def gsb_lle(ctx, variant: int, schedule: int, control_strength: float, A_per_replica, dt: float, replicas: int,
            steps: int, seed: int, tangent_seed: int, renorm_every: int, want_state: bool = False):
    """Returns lle[replicas] and, with want_state, the (6, replicas, n_dyn) float32 final state
    (x, y, p, dx, dy, dp)."""
    lle = np.empty(replicas, dtype=np.float64)
    Ar = None if A_per_replica is None else np.ascontiguousarray(A_per_replica, dtype=np.float64)
    if Ar is not None and Ar.shape != (replicas,):
        raise ValueError("A_per_replica must have one entry per replica")
    st = None
    if want_state:
        st = np.empty((6, replicas, int(gsb_get(ctx, GSB_OPT_N_DYN))), dtype=np.float32)
    _check(load_library().gsb_lle(ctx, variant, schedule, control_strength, None if Ar is None else _ptr(Ar), dt,
                                  replicas, steps, seed & (2**64 - 1), tangent_seed & (2**64 - 1), renorm_every,
                                  _ptr(lle), None if st is None else _ptr(st)), "gsb_lle")
    return (lle, st) if want_state else lle


def gsb_vjp(ctx, count: int, xb: np.ndarray, yb: np.ndarray, pb: np.ndarray):
    """Cotangents at the current step from those `count` steps later (new arrays)."""
    xb, yb, pb = (np.array(v, dtype=np.float32, order="C", copy=True) for v in (xb, yb, pb))
    _check(load_library().gsb_vjp(ctx, count, _ptr(xb), _ptr(yb), _ptr(pb)), "gsb_vjp")
    return xb, yb, pb


def gsb_last_step_ms(ctx) -> float:
    v = ctypes.c_double()
    _check(load_library().gsb_last_step_ms(ctx, ctypes.byref(v)), "gsb_last_step_ms")
    return v.value


def gsb_batch_create(n, replicas: int):
    nn = np.ascontiguousarray(n, dtype=np.int32)
    out = ctypes.c_void_p()
    _check(load_library().gsb_batch_create(int(nn.size), _ptr(nn), replicas, ctypes.byref(out)), "gsb_batch_create")
    return out


def gsb_batch_destroy(batch) -> None:
    load_library().gsb_batch_destroy(batch)


def gsb_batch_set_stream(batch, stream: int | None) -> None:
    _check(load_library().gsb_batch_set_stream(batch, ctypes.c_void_p(stream or 0)), "gsb_batch_set_stream")


def gsb_batch_workspace_size(batch) -> int:
    v = ctypes.c_size_t()
    _check(load_library().gsb_batch_workspace_size(batch, ctypes.byref(v)), "gsb_batch_workspace_size")
    return v.value


def gsb_batch_bind_workspace(batch, device_ptr: int, nbytes: int) -> None:
    _check(load_library().gsb_batch_bind_workspace(batch, ctypes.c_void_p(device_ptr), nbytes),
           "gsb_batch_bind_workspace")


def gsb_batch_set_coupling(batch, k: int, J: np.ndarray, c: float = 0.0, dt: float = 0.0) -> None:
    J = np.ascontiguousarray(J, dtype=np.float32)
    if J.ndim != 2 or J.shape[0] != J.shape[1]:
        raise ValueError("J must be a square matrix")
    _check(load_library().gsb_batch_set_coupling(batch, k, _ptr(J), float(c), float(dt)), "gsb_batch_set_coupling")


def gsb_batch_set(batch, k: int, option: int, value: float) -> None:
    _check(load_library().gsb_batch_set(batch, k, option, float(value)), "gsb_batch_set")


def gsb_batch_get(batch, k: int, option: int) -> float:
    v = ctypes.c_double()
    _check(load_library().gsb_batch_get(batch, k, option, ctypes.byref(v)), "gsb_batch_get")
    return v.value


def gsb_batch_autotune(batch, variant: int, control_strength: float, trial_steps: int, seed: int) -> None:
    _check(load_library().gsb_batch_autotune(batch, variant, control_strength, trial_steps, seed & (2**64 - 1)),
           "gsb_batch_autotune")


def gsb_batch_run(batch, variant: int, control_strength: float, steps: int, seed: int) -> None:
    _check(load_library().gsb_batch_run(batch, variant, control_strength, steps, seed & (2**64 - 1)), "gsb_batch_run")


def gsb_batch_energy(batch, k: int) -> np.ndarray:
    E = np.empty(int(gsb_batch_get(batch, -1, GSB_BATCH_REPLICAS)), dtype=np.float64)
    _check(load_library().gsb_batch_energy(batch, k, _ptr(E)), "gsb_batch_energy")
    return E


def gsb_batch_best(batch):
    count = int(gsb_batch_get(batch, -1, GSB_BATCH_COUNT))
    e = np.empty(count, dtype=np.float64)
    r = np.empty(count, dtype=np.int32)
    _check(load_library().gsb_batch_best(batch, _ptr(e), _ptr(r)), "gsb_batch_best")
    return e, r


def gsb_batch_state(batch, k: int):
    R = int(gsb_batch_get(batch, -1, GSB_BATCH_REPLICAS))
    n = int(gsb_batch_get(batch, k, GSB_BATCH_N))
    x, y, p = (np.empty((R, n), dtype=np.float32) for _ in range(3))
    _check(load_library().gsb_batch_state(batch, k, _ptr(x), _ptr(y), _ptr(p)), "gsb_batch_state")
    return x, y, p


def gsb_batch_last_ms(batch) -> float:
    v = ctypes.c_double()
    _check(load_library().gsb_batch_last_ms(batch, ctypes.byref(v)), "gsb_batch_last_ms")
    return v.value


def gsb_batch_plan(width, gangs, cost, queues: int, workers: int):
    """Queue and rank of every unit in the plan gsb_batch_run uses."""
    w = np.ascontiguousarray(width, dtype=np.int32)
    g = np.ascontiguousarray(gangs, dtype=np.int32)
    c = np.ascontiguousarray(cost, dtype=np.float64)
    q = np.empty(w.size, dtype=np.int32)
    r = np.empty(w.size, dtype=np.int32)
    _check(load_library().gsb_batch_plan(int(w.size), _ptr(w), _ptr(g), _ptr(c), queues, workers, _ptr(q), _ptr(r)),
           "gsb_batch_plan")
    return q, r



def gsb_encode_operand(precision: int, discrete: int, x_ptr: int | None, count: int, out_ptr: int | None,
                       stream: int | None) -> None:
    _check(load_library().gsb_encode_operand(precision, discrete, ctypes.c_void_p(x_ptr or 0), count,
                                             ctypes.c_void_p(out_ptr or 0), ctypes.c_void_p(stream or 0)),
           "gsb_encode_operand")


def encode_operand(x, precision: int, discrete: bool = False):
    """The operand of the coupling product for the binary32 device tensor x (1-D), as the
    step kernels encode it: FP8 -> uint8 E4M3 codes; BF16X2 -> (hi, lo) bfloat16;
    FIX16 -> (hi, lo) int8 with rint(x 2^14) = 256 hi + lo; FP32 -> float32.  Runs on
    PyTorch's current stream."""
    import torch
    if x.dtype != torch.float32 or x.dim() != 1 or not x.is_cuda:
        raise ValueError("x must be a 1-D float32 device tensor")
    x = x.contiguous()
    n = x.numel()
    if precision == GSB_PREC_FP8:
        out = torch.empty(n, dtype=torch.uint8, device=x.device)
    elif precision == GSB_PREC_BF16X2:
        out = torch.empty((2, n), dtype=torch.int16, device=x.device)
    elif precision == GSB_PREC_FIX16:
        out = torch.empty((2, n), dtype=torch.int8, device=x.device)
    else:
        out = torch.empty(n, dtype=torch.float32, device=x.device)
    gsb_encode_operand(precision, int(discrete), x.data_ptr(), n, out.data_ptr(),
                       torch.cuda.current_stream().cuda_stream)
    if precision == GSB_PREC_BF16X2:
        return out[0].view(torch.bfloat16), out[1].view(torch.bfloat16)
    if precision == GSB_PREC_FIX16:
        return out[0], out[1]
    return out


class Batch:
    """Many instances of different sizes, all replicas in one persistent launch (FP8 product).

    >>> b = Batch([n0, n1, ...], replicas=128)
    >>> b.set_couplings(lambda k: J_k)           # c = 1/lambda_max, dt from eq. (13)
    >>> b.autotune("gbsb", A=0.2, trial_steps=50, seed=1)
    >>> b.run("gbsb", A=0.2, steps=1000, seed=1)
    >>> energies, replicas = b.best()
    """

    def __init__(self, sizes, replicas: int):
        import torch  # device memory and streams only

        if not torch.cuda.is_available():
            raise RuntimeError("Batch needs a HIP device")
        self._torch = torch
        self.sizes = [int(v) for v in sizes]
        self.replicas = int(replicas)
        self.b = gsb_batch_create(self.sizes, self.replicas)
        need = gsb_batch_workspace_size(self.b)
        self._ws = torch.empty(need + 256, dtype=torch.uint8, device="cuda")
        base = self._ws.data_ptr()
        aligned = (base + 255) // 256 * 256
        gsb_batch_bind_workspace(self.b, aligned, need + 256 - (aligned - base))
        gsb_batch_set_stream(self.b, torch.cuda.current_stream().cuda_stream)

    def close(self):
        if self.b is not None:
            gsb_batch_destroy(self.b)
            self.b = None
            self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_coupling(self, k: int, J, c: float = 0.0, dt: float = 0.0):
        gsb_batch_set_coupling(self.b, k, J, c, dt)

    def set_couplings(self, make, threads: int = 8):
        """make(k) -> J or (J, c, dt); the instances are generated and uploaded by a pool of
        host threads (the library call releases the interpreter lock)."""
        from concurrent.futures import ThreadPoolExecutor

        def one(k):
            v = make(k)
            J, c, dt = (v if isinstance(v, tuple) else (v, 0.0, 0.0))
            gsb_batch_set_coupling(self.b, k, J, c, dt)

        with ThreadPoolExecutor(max_workers=max(1, threads)) as ex:
            list(ex.map(one, range(len(self.sizes))))

    def set(self, k: int, option: int, value: float):
        gsb_batch_set(self.b, k, option, value)

    def get(self, k: int, option: int) -> float:
        return gsb_batch_get(self.b, k, option)

    def autotune(self, variant, *, A: float = 0.0, trial_steps: int = 50, seed: int = 1):
        v = VARIANTS[variant] if isinstance(variant, str) else int(variant)
        gsb_batch_autotune(self.b, v, A, trial_steps, seed)

    def run(self, variant, *, A: float = 0.0, steps: int, seed: int):
        v = VARIANTS[variant] if isinstance(variant, str) else int(variant)
        gsb_batch_set_stream(self.b, self._torch.cuda.current_stream().cuda_stream)
        gsb_batch_run(self.b, v, A, steps, seed)

    def energy(self, k: int) -> np.ndarray:
        return gsb_batch_energy(self.b, k)

    def best(self):
        return gsb_batch_best(self.b)

    def state(self, k: int):
        return gsb_batch_state(self.b, k)

    def last_ms(self) -> float:
        return gsb_batch_last_ms(self.b)

    def params(self, k: int):
        return gsb_batch_get(self.b, k, GSB_BATCH_C), gsb_batch_get(self.b, k, GSB_BATCH_DT)


class GSB:
    """One Ising instance on the current HIP device, with a PyTorch-owned workspace.

    >>> g = GSB(J, precision="fp8", c=1 / (2 * np.sqrt(n)))
    >>> g.run("gbsb", A=0.2, dt=1.25, replicas=1024, steps=2000, seed=1)
    >>> spins, energy, replica = g.best()
    """

    def __init__(self, J: np.ndarray, h: np.ndarray | None = None, *, precision: str | None = None,
                 c: float | None = None, init_mode: int | None = None, step_kernel: int | None = None,
                 grid_pad: bool | None = None):
        import torch  # device memory and streams only

        if not torch.cuda.is_available():
            raise RuntimeError("GSB needs a HIP device")
        self._torch = torch
        self.ctx = gsb_create(J, h)
        self._ws = None
        if precision is not None:
            gsb_set(self.ctx, GSB_OPT_PRECISION, PRECISIONS[precision])
        if c is not None:
            gsb_set(self.ctx, GSB_OPT_C, c)
        if init_mode is not None:
            gsb_set(self.ctx, GSB_OPT_INIT_MODE, init_mode)
        if step_kernel is not None:
            gsb_set(self.ctx, GSB_OPT_STEP_KERNEL, step_kernel)
        if grid_pad is not None:
            gsb_set(self.ctx, GSB_OPT_GRID_PAD, 1 if grid_pad else 0)

    def close(self):
        if self.ctx is not None:
            gsb_destroy(self.ctx)
            self.ctx = None
            self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _prepare(self, replicas: int, steps: int, lle: bool = False):
        torch = self._torch
        need = (gsb_lle_workspace_size if lle else gsb_workspace_size)(self.ctx, replicas, steps)
        if self._ws is None or self._ws.numel() < need + 256:
            self._ws = torch.empty(need + 256, dtype=torch.uint8, device="cuda")
            base = self._ws.data_ptr()
            aligned = (base + 255) // 256 * 256
            gsb_bind_workspace(self.ctx, aligned, need + 256 - (aligned - base))
        gsb_set_stream(self.ctx, torch.cuda.current_stream().cuda_stream)

    def init(self, variant, *, A: float = 0.0, dt: float, replicas: int, steps: int, seed: int,
             schedule: int = GSB_SCHED_LINEAR):
        v = VARIANTS[variant] if isinstance(variant, str) else int(variant)
        self._prepare(replicas, steps)
        gsb_init(self.ctx, v, schedule, A, dt, replicas, steps, seed)

    def step(self, count: int):
        gsb_set_stream(self.ctx, self._torch.cuda.current_stream().cuda_stream)
        gsb_step(self.ctx, count)

    def run(self, variant, *, A: float = 0.0, dt: float, replicas: int, steps: int, seed: int,
            schedule: int = GSB_SCHED_LINEAR):
        v = VARIANTS[variant] if isinstance(variant, str) else int(variant)
        self._prepare(replicas, steps)
        gsb_run(self.ctx, v, schedule, A, dt, replicas, steps, seed)

    def energy(self) -> np.ndarray:
        return gsb_energy(self.ctx)

    def best(self):
        return gsb_best(self.ctx)

    def spins(self) -> np.ndarray:
        return gsb_spins(self.ctx)

    def state(self):
        return gsb_state(self.ctx)

    def set_state(self, x, y, p, m):
        gsb_set_state(self.ctx, x, y, p, m)

    def delta(self) -> np.ndarray:
        return gsb_delta(self.ctx)

    def lle(self, variant, *, A=0.0, dt: float, replicas: int, steps: int, seed: int, tangent_seed: int,
            renorm_every: int = 10, schedule: int = GSB_SCHED_LINEAR, want_state: bool = False,
            window_from: int = 0):
        """Largest-Lyapunov-exponent estimates; A is one value or one per replica.  The
        growth is counted from step `window_from` on (GSB_OPT_LLE_FROM)."""
        v = VARIANTS[variant] if isinstance(variant, str) else int(variant)
        per = None if np.isscalar(A) else np.asarray(A, dtype=np.float64)
        gsb_set(self.ctx, GSB_OPT_LLE_FROM, window_from)
        self._prepare(replicas, steps, lle=True)
        return gsb_lle(self.ctx, v, schedule, float(A) if per is None else 0.0, per, dt, replicas, steps, seed,
                       tangent_seed, renorm_every, want_state)

    def vjp(self, count: int, xb, yb, pb):
        gsb_set_stream(self.ctx, self._torch.cuda.current_stream().cuda_stream)
        return gsb_vjp(self.ctx, count, xb, yb, pb)

    # the device-memory forms (torch tensors on the GPU, on torch's current stream)
    def state_device(self, x, y, p) -> int:
        gsb_set_stream(self.ctx, self._torch.cuda.current_stream().cuda_stream)
        return gsb_state_device(self.ctx, x, y, p)

    def set_state_device(self, x, y, p, m: int) -> None:
        gsb_set_stream(self.ctx, self._torch.cuda.current_stream().cuda_stream)
        gsb_set_state_device(self.ctx, x, y, p, m)

    def vjp_device(self, count: int, xb, yb, pb) -> None:
        gsb_set_stream(self.ctx, self._torch.cuda.current_stream().cuda_stream)
        gsb_vjp_device(self.ctx, count, xb, yb, pb)

    def last_step_ms(self) -> float:
        return gsb_last_step_ms(self.ctx)

    def get(self, option: int) -> float:
        return gsb_get(self.ctx, option)

    def set(self, option: int, value: float) -> None:
        gsb_set(self.ctx, option, value)
