"""Success statistics of a run of R replicas (Sec. VI): success probability, its
statistical error, the time to solution at 99% and the error of that time.

Definitions (Sec. VI):
  P_S      : fraction of runs that reach the target energy.
  dP_S     : sqrt((P_S - P_S^2) / N_rep), N_rep the number of repetitions.
  TTS      : T_com ln(1 - 0.99) / ln(1 - P_S), or T_com when P_S > 0.99.
  dTTS     : TTS dP_S / ((1 - P_S) |ln(1 - P_S)|) (the absolute value of the logarithm; one
             table caption prints it without).

Batch semantics (Sec. VI, batch processing: several runs side by side in one machine, the
better result kept): one launch of R replicas is one run of duration T_com, and it succeeds
when any replica does, so P_run = 1 - (1 - p)^R for the per-replica probability p, which
the R replicas of a launch estimate as p_hat = hits / R.  Then ln(1 - P_run) = R ln(1 - p),
so TTS = T_com ln 0.01 / (R ln(1 - p_hat)), and propagating dp_hat = sqrt((p_hat -
p_hat^2) / R) through it gives dTTS = TTS dp_hat / ((1 - p_hat) |ln(1 - p_hat)|): the
paper's expression with the per-replica quantities.  When P_run > 0.99 the TTS is the
constant T_com and its error is 0.
"""
from __future__ import annotations

import math

TARGET = 0.99


def p_hat(hits: int, replicas: int) -> float:
    """Per-replica success probability estimated from one launch."""
    if replicas <= 0 or hits < 0 or hits > replicas:
        raise ValueError("need 0 <= hits <= replicas, replicas > 0")
    return hits / replicas


def dp_s(p: float, n_rep: int) -> float:
    """Statistical error of a success probability estimated from n_rep repetitions."""
    if n_rep <= 0:
        raise ValueError("n_rep must be positive")
    return math.sqrt(max(p - p * p, 0.0) / n_rep)


def p_run(p: float, replicas: int) -> float:
    """Success probability of one launch of `replicas` replicas (any replica succeeds)."""
    return 1.0 - (1.0 - p) ** replicas


def tts99(t_com: float, p_s: float) -> float:
    """Time to solution at 99%; +inf when p_s = 0."""
    if p_s > TARGET:
        return t_com
    if p_s <= 0.0:
        return math.inf
    return t_com * math.log(1.0 - TARGET) / math.log(1.0 - p_s)


def dtts(tts: float, p_s: float, dp: float) -> float:
    """Statistical error of a TTS (Sec. VI), with |ln(1 - P_S)|; 0 when the TTS is T_com
    (P_S > 0.99) and +inf when P_S is 0."""
    if p_s > TARGET:
        return 0.0
    if p_s <= 0.0:
        return math.inf
    return tts * dp / ((1.0 - p_s) * abs(math.log(1.0 - p_s)))


def batch_tts(t_com: float, hits: int, replicas: int) -> dict:
    """p_hat, dP_S, P_run, TTS99 and dTTS of one launch of `replicas` replicas of duration
    t_com with `hits` replicas at the target (batch semantics, see the module docstring)."""
    p = p_hat(hits, replicas)
    dp = dp_s(p, replicas)
    pr = p_run(p, replicas)
    t = tts99(t_com, pr)
    if pr > TARGET:
        dt = 0.0
    elif p <= 0.0:
        dt = math.inf
    else:
        dt = dtts(t, p, dp)
    return {"p_hat": p, "dp_hat": dp, "p_run": pr, "tts99_s": t, "dtts99_s": dt}


def finite_or_none(v: float):
    return v if math.isfinite(v) else None
