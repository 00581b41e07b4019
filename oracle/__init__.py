"""CPU oracle for simulated bifurcation (bSB / dSB / GbSB / GdSB) -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py``
may import this package.  It wraps ``gsb_oracle.c`` (plain C, built with gcc) through
ctypes.  It shares no code with the GPU library and never imports it.

Every function cites the passage of Goto, Hidaka & Tatsumura (arXiv 2508.17655) it
follows; see the header of ``gsb_oracle.c`` for the readings taken where the paper is
silent.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gsb_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

BSB, DSB, GBSB, GDSB = 0, 1, 2, 3
VARIANTS = {"bsb": BSB, "dsb": DSB, "gbsb": GBSB, "gdsb": GDSB}
SCHED_LINEAR, SCHED_CONSTANT = 0, 1
FORM_EXACT, FORM_E4M3, FORM_BF16X2, FORM_FIX16 = 0, 1, 2, 3
INIT_X, INIT_XY, INIT_PM01 = 0, 1, 2

_lib = None


def build(force: bool = True) -> str:
    """Compile gsb_oracle.c with gcc into liboracle.so (no contraction, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
               "-fno-fast-math", "-fexcess-precision=standard", "-D_GNU_SOURCE", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build(force=True)
    lib = ctypes.CDLL(_LIB)
    u64, i32, i64, dbl = ctypes.c_uint64, ctypes.c_int, ctypes.c_int64, ctypes.c_double
    vp = ctypes.c_void_p
    lib.orc_splitmix64_mix.restype = u64
    lib.orc_splitmix64_mix.argtypes = [u64]
    lib.orc_splitmix64_at.restype = u64
    lib.orc_splitmix64_at.argtypes = [u64, u64]
    lib.orc_init_state.restype = None
    lib.orc_init_state.argtypes = [i32, i32, u64, i32, vp, vp]
    lib.orc_e4m3_round.restype = dbl
    lib.orc_e4m3_round.argtypes = [dbl]
    lib.orc_e4m3_encode.restype = ctypes.c_uint8
    lib.orc_e4m3_encode.argtypes = [dbl]
    lib.orc_e4m3_decode.restype = dbl
    lib.orc_e4m3_decode.argtypes = [ctypes.c_uint8]
    lib.orc_bf16_round.restype = ctypes.c_float
    lib.orc_bf16_round.argtypes = [ctypes.c_float]
    lib.orc_fix16_round.restype = dbl
    lib.orc_fix16_round.argtypes = [dbl]
    lib.orc_e4m3_round_array.restype = None
    lib.orc_e4m3_round_array.argtypes = [vp, vp, i64]
    lib.orc_e4m3_encode_array.restype = None
    lib.orc_e4m3_encode_array.argtypes = [vp, vp, i64]
    lib.orc_bf16_round_array.restype = None
    lib.orc_bf16_round_array.argtypes = [vp, vp, i64]
    lib.orc_operand_array.restype = None
    lib.orc_operand_array.argtypes = [vp, vp, i64, i32, i32]
    for name in ("orc_run_f64", "orc_run_f32"):
        f = getattr(lib, name)
        f.restype = i32
        f.argtypes = [vp, i32, i32, i32, i32, dbl, dbl, dbl, i32, i32, i32, i32, vp, vp, vp, vp]
    lib.orc_spins_f32.restype = None
    lib.orc_spins_f32.argtypes = [vp, i64, vp]
    lib.orc_spins_f64.restype = None
    lib.orc_spins_f64.argtypes = [vp, i64, vp]
    lib.orc_energy.restype = None
    lib.orc_energy.argtypes = [vp, i32, vp, i32, vp]
    lib.orc_cut_direct.restype = dbl
    lib.orc_cut_direct.argtypes = [vp, i32, vp]
    lib.orc_best.restype = i32
    lib.orc_best.argtypes = [vp, i32]
    lib.orc_ground_state.restype = dbl
    lib.orc_ground_state.argtypes = [vp, i32, vp]
    lib.orc_delta.restype = dbl
    lib.orc_delta.argtypes = [vp, vp, i32]
    lib.orc_num_threads.restype = i32
    lib.orc_num_threads.argtypes = []
    lib.orc_set_num_threads.restype = None
    lib.orc_set_num_threads.argtypes = [i32]
    lib.orc_init_pairs.restype = None
    lib.orc_init_pairs.argtypes = [i32, i32, u64, vp, vp]
    lib.orc_tangent_run_f64.restype = i32
    lib.orc_tangent_run_f64.argtypes = [vp, i32, i32, i32, dbl, dbl, dbl, i32, i32, i32, i32, i32,
                                        vp, vp, vp, vp, vp, vp, vp]
    lib.orc_adjoint_step_f64.restype = i32
    lib.orc_adjoint_step_f64.argtypes = [vp, i32, i32, dbl, dbl, dbl, dbl, vp, vp, vp, vp, vp, vp]
    _lib = lib
    return lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def num_threads() -> int:
    return int(_load().orc_num_threads())


def set_num_threads(t: int) -> None:
    """Threads of the loops over replicas (timing only; results do not depend on it)."""
    _load().orc_set_num_threads(int(t))


# ---- generator (SplitMix64, counter form) -----------------------------------------------
def splitmix64_at(seed: int, k: int) -> int:
    """k-th output (k >= 1) of SplitMix64 seeded with `seed`."""
    return int(_load().orc_splitmix64_at(seed & (2**64 - 1), k & (2**64 - 1)))


def init_state(n: int, replicas: int, seed: int, mode: int = INIT_X):
    """Initial x, y (float32, [replicas, n]); App. A (x ~ U(-0.1, 0.1), y = 0),
    mode XY draws y the same way, mode PM01 is the chaos start x = +-0.1 (Sec. IV)."""
    x = np.zeros((replicas, n), dtype=np.float32)
    y = np.zeros((replicas, n), dtype=np.float32)
    _load().orc_init_state(n, replicas, seed & (2**64 - 1), mode, _p(x), _p(y))
    return x, y


# ---- number formats ----------------------------------------------------------------------
def e4m3_round(v: np.ndarray) -> np.ndarray:
    v = np.ascontiguousarray(v, dtype=np.float64)
    out = np.empty_like(v)
    _load().orc_e4m3_round_array(_p(v), _p(out), v.size)
    return out


def e4m3_encode(v: np.ndarray) -> np.ndarray:
    v = np.ascontiguousarray(v, dtype=np.float32)
    out = np.empty(v.shape, dtype=np.uint8)
    _load().orc_e4m3_encode_array(_p(v), _p(out), v.size)
    return out


def e4m3_decode(b: int) -> float:
    return float(_load().orc_e4m3_decode(b))


def bf16_round(v: np.ndarray) -> np.ndarray:
    v = np.ascontiguousarray(v, dtype=np.float32)
    out = np.empty_like(v)
    _load().orc_bf16_round_array(_p(v), _p(out), v.size)
    return out


def fix16_round(v: float) -> float:
    return float(_load().orc_fix16_round(v))


def operand(v: np.ndarray, form: int, discrete: bool = False) -> np.ndarray:
    """Value the coupling product of eq. (3) uses for each binary32 x (float64 out): the
    rounding of `form`, or the sign s(x) (+1 for x >= 0) of the dSB/GdSB product."""
    v = np.ascontiguousarray(v, dtype=np.float32)
    out = np.empty(v.shape, dtype=np.float64)
    _load().orc_operand_array(_p(v), _p(out), v.size, int(discrete), form)
    return out


# ---- dynamics ----------------------------------------------------------------------------
def run(J: np.ndarray, variant: int, *, A: float = 0.0, dt: float, c: float, steps: int,
        x: np.ndarray, y: np.ndarray, p: np.ndarray | None = None, m_begin: int = 0,
        m_end: int | None = None, schedule: int = SCHED_LINEAR, form: int = FORM_EXACT,
        mode: str = "fp64", record: bool = False):
    """Advance replicas (rows of x, y, p) through steps m_begin .. m_end-1 of an
    M = `steps` schedule: eqs. (3)-(5) with eq. (7) control (A = 0 for bSB/dSB).

    mode "fp64": binary64 state; mode "fp32": binary32 state, one rounding per
    operation (Fig. 2(a): the PXY part is 32-bit floating point).
    Returns (x, y, p[, traj]) as new arrays; traj[r, k] is x after step m_begin + k.
    """
    J = np.ascontiguousarray(J, dtype=np.float64)
    n = J.shape[0]
    if m_end is None:
        m_end = steps
    dt_ = np.float64 if mode == "fp64" else np.float32
    x = np.array(x, dtype=dt_, order="C", copy=True).reshape(-1, n)
    y = np.array(y, dtype=dt_, order="C", copy=True).reshape(-1, n)
    R = x.shape[0]
    p = np.ones((R, n), dtype=dt_) if p is None else np.array(p, dtype=dt_, order="C", copy=True).reshape(R, n)
    traj = np.zeros((R, m_end - m_begin, n), dtype=dt_) if record else None
    f = _load().orc_run_f64 if mode == "fp64" else _load().orc_run_f32
    rc = f(_p(J), n, variant, schedule, form, float(A), float(dt), float(c), int(steps), int(m_begin),
           int(m_end), R, _p(x), _p(y), _p(p), _p(traj) if record else None)
    if rc != 0:
        raise ValueError("oracle run: bad arguments")
    return (x, y, p, traj) if record else (x, y, p)


# ---- readout, energy, cut ------------------------------------------------------------------
def spins(x: np.ndarray) -> np.ndarray:
    """s_i = sgn(x_i) with sgn(0) = +1 (Sec. II)."""
    x = np.ascontiguousarray(x)
    s = np.empty(x.shape, dtype=np.int8)
    if x.dtype == np.float32:
        _load().orc_spins_f32(_p(x), x.size, _p(s))
    else:
        x = np.ascontiguousarray(x, dtype=np.float64)
        _load().orc_spins_f64(_p(x), x.size, _p(s))
    return s


def energy(J: np.ndarray, s: np.ndarray) -> np.ndarray:
    """Ising energy, eq. (1), of each row of s."""
    J = np.ascontiguousarray(J, dtype=np.float64)
    n = J.shape[0]
    s = np.ascontiguousarray(s, dtype=np.int8).reshape(-1, n)
    E = np.empty(s.shape[0], dtype=np.float64)
    _load().orc_energy(_p(J), n, _p(s), s.shape[0], _p(E))
    return E


def cut_direct(J: np.ndarray, s: np.ndarray) -> float:
    """MAX-CUT value with weights -J (Sec. III), by counting cut edges."""
    J = np.ascontiguousarray(J, dtype=np.float64)
    s = np.ascontiguousarray(s, dtype=np.int8)
    return float(_load().orc_cut_direct(_p(J), J.shape[0], _p(s)))


def best(E: np.ndarray) -> int:
    E = np.ascontiguousarray(E, dtype=np.float64)
    return int(_load().orc_best(_p(E), E.size))


def ground_state(J: np.ndarray):
    """Exhaustive minimum of eq. (1) for n <= 24: (E0, one minimiser)."""
    J = np.ascontiguousarray(J, dtype=np.float64)
    n = J.shape[0]
    s = np.empty(n, dtype=np.int8)
    E0 = float(_load().orc_ground_state(_p(J), n, _p(s)))
    return E0, s


def delta(x1: np.ndarray, x2: np.ndarray) -> float:
    """Normalised distance between two trajectories, eq. (8)."""
    x1 = np.ascontiguousarray(x1, dtype=np.float64)
    x2 = np.ascontiguousarray(x2, dtype=np.float64)
    return float(_load().orc_delta(_p(x1), _p(x2), x1.size))


def init_pairs(n: int, pairs: int, seed: int):
    """Trajectory pairs of Sec. IV (replicas 2k, 2k+1): x1 = +-0.1, x2 = x1 +- 2e-6, y = 0.
    Returns float32 (x, y) of shape (2 pairs, n)."""
    x = np.empty((2 * pairs, n), dtype=np.float32)
    y = np.empty((2 * pairs, n), dtype=np.float32)
    _load().orc_init_pairs(n, pairs, seed, _p(x), _p(y))
    return x, y


def tangent_run(J: np.ndarray, variant: int, *, A: float = 0.0, dt: float, c: float, steps: int,
                x: np.ndarray, y: np.ndarray, p: np.ndarray | None = None, dx: np.ndarray, dy=None, dp=None,
                m_begin: int = 0, m_end: int | None = None, schedule: int = SCHED_LINEAR, renorm: int = 1):
    """Primal and tangent of the continuous-product dynamics in binary64 (bSB, GbSB).
    Returns (x, y, p, dx, dy, dp, log_growth[replicas]); the tangent comes back with unit norm
    and log_growth = ln(|v(t_end)| / |v(t_begin)|)."""
    J = np.ascontiguousarray(J, dtype=np.float64)
    n = J.shape[0]
    x = np.array(x, dtype=np.float64, order="C", ndmin=2)
    R = x.shape[0]
    y = np.array(y, dtype=np.float64, order="C", ndmin=2)
    p = np.ones_like(x) if p is None else np.array(p, dtype=np.float64, order="C", ndmin=2)
    dx = np.array(dx, dtype=np.float64, order="C", ndmin=2)
    dy = np.zeros_like(x) if dy is None else np.array(dy, dtype=np.float64, order="C", ndmin=2)
    dp = np.zeros_like(x) if dp is None else np.array(dp, dtype=np.float64, order="C", ndmin=2)
    lg = np.zeros(R, dtype=np.float64)
    me = steps if m_end is None else m_end
    rc = _load().orc_tangent_run_f64(_p(J), n, variant, schedule, A, dt, c, steps, m_begin, me, renorm, R,
                                     _p(x), _p(y), _p(p), _p(dx), _p(dy), _p(dp), _p(lg))
    if rc != 0:
        raise ValueError("oracle tangent run rejected its arguments")
    return x, y, p, dx, dy, dp, lg


def adjoint_step(J: np.ndarray, variant: int, *, A: float, dt: float, c: float, rm: float,
                 x: np.ndarray, y: np.ndarray, p: np.ndarray, xb: np.ndarray, yb: np.ndarray, pb: np.ndarray):
    """Cotangents of one step's inputs from those of its outputs, at input state (x, y, p)."""
    J = np.ascontiguousarray(J, dtype=np.float64)
    n = J.shape[0]
    x, y, p = (np.ascontiguousarray(v, dtype=np.float64) for v in (x, y, p))
    xb, yb, pb = (np.array(v, dtype=np.float64, order="C") for v in (xb, yb, pb))
    rc = _load().orc_adjoint_step_f64(_p(J), n, variant, A, dt, c, rm, _p(x), _p(y), _p(p), _p(xb), _p(yb), _p(pb))
    if rc != 0:
        raise ValueError("oracle adjoint step rejected its arguments")
    return xb, yb, pb
