"""Seeded synthetic Ising instances (inputs only; none of the method's arithmetic).

Stand-ins for the paper's workloads, which are not available here (Sec. III: K2000 is a
fully connected N = 2000 instance with J_ij in {+-1}; the 700-spin set is fully
connected with J_ij in {+-1}; G-set instances are sparse with J_ij in {0, -1} or
{0, +-1}).  Every generator is a pure function of (n, seed, ...), built on counter-based
SplitMix64 (Steele, Lea, Flood 2014): draw k (k >= 1) of stream `seed` is
mix(seed + k * 0x9E3779B97F4A7C15).  Draws run over the upper triangle i < j in
row-major order, then J is mirrored; the diagonal is zero.

This module is shared by the tests and the benchmark as the one source of inputs; it
imports nothing from the GPU binding or from the oracle.
"""
from __future__ import annotations

import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, k: np.ndarray) -> np.ndarray:
    """Draws number k (uint64 array, k >= 1) of SplitMix64 seeded with `seed`."""
    with np.errstate(over="ignore"):
        z = np.uint64(seed & (2**64 - 1)) + k.astype(np.uint64) * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def _upper(n: int, draws: np.ndarray) -> np.ndarray:
    J = np.zeros((n, n), dtype=np.float32)
    o = 0
    for i in range(n - 1):  # row-major upper triangle, row by row
        J[i, i + 1:] = draws[o:o + n - 1 - i]
        o += n - 1 - i
    return J + J.T


def dense_pm1(n: int, seed: int) -> np.ndarray:
    """Fully connected, J_ij iid uniform on {-1, +1} (bit 63 of each draw gives the sign)."""
    t = n * (n - 1) // 2
    z = splitmix64(seed, np.arange(1, t + 1, dtype=np.uint64))
    v = np.where((z >> np.uint64(63)) != 0, -1.0, 1.0).astype(np.float32)
    return _upper(n, v)


def dense_gaussian(n: int, seed: int) -> np.ndarray:
    """Fully connected, J_ij iid N(0, 1)/sqrt(n) (Box-Muller on two draws per coupling),
    rounded to binary32."""
    t = n * (n - 1) // 2
    k = np.arange(1, 2 * t + 1, dtype=np.uint64)
    z = splitmix64(seed, k)
    u = ((z >> np.uint64(11)).astype(np.float64) + 1.0) * 2.0**-53  # (0, 1]
    u1, u2 = u[0::2], u[1::2]
    g = np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)
    return _upper(n, (g / np.sqrt(n)).astype(np.float32))


def erdos_renyi_pm1(n: int, prob: float, seed: int) -> np.ndarray:
    """Sparse G(n, prob) graph with J_ij in {+-1} on its edges (G-set-like)."""
    t = n * (n - 1) // 2
    k = np.arange(1, 2 * t + 1, dtype=np.uint64)
    z = splitmix64(seed, k)
    u = (z[0::2] >> np.uint64(11)).astype(np.float64) * 2.0**-53
    sign = np.where((z[1::2] >> np.uint64(63)) != 0, -1.0, 1.0)
    return _upper(n, np.where(u < prob, sign, 0.0).astype(np.float32))


def paper_c(n: int) -> float:
    """c = 1/(2 sqrt(N) sigma) with sigma = 1 for J_ij in {+-1} (App. A)."""
    return 1.0 / (2.0 * np.sqrt(n))


def batch_workload(count: int, seed: int, n_min: int = 64, n_max: int = 4096):
    """Specs of a batch of uneven instances: n iid uniform integer in [n_min, n_max]; even
    indices dense +-1, odd indices Erdos-Renyi with edge probability p iid U[0.01, 0.06]
    and +-1 weights.  Spec k uses draws 3k+1 (n), 3k+2 (p) and 3k+3 (the instance's own
    generator seed) of stream `seed`.  Returns a list of (kind, n, p, instance_seed)."""
    z = splitmix64(seed, np.arange(1, 3 * count + 1, dtype=np.uint64))
    specs = []
    for k in range(count):
        n = n_min + int(z[3 * k] % np.uint64(n_max - n_min + 1))
        u = float(z[3 * k + 1] >> np.uint64(11)) * 2.0**-53
        iseed = int(z[3 * k + 2] >> np.uint64(1))
        if k % 2 == 0:
            specs.append(("dense", n, 1.0, iseed))
        else:
            specs.append(("sparse", n, 0.01 + 0.05 * u, iseed))
    return specs


def make_instance(spec) -> np.ndarray:
    kind, n, p, iseed = spec
    return dense_pm1(n, iseed) if kind == "dense" else erdos_renyi_pm1(n, p, iseed)
