"""Checks against the values the paper prints (tests/golden/paper_values.json, each entry
with its citation).  CPU only: the oracle, the library's host-side eigenvalue code and the
host statistics module."""
import json
import math
import os

import numpy as np
import pytest

import oracle
from paper_2508_17655_amd import gsb, instances

HERE = os.path.dirname(os.path.abspath(__file__))
with open(os.path.join(HERE, "golden", "paper_values.json")) as f:
    PAPER = json.load(f)


def test_fixture_values_match_their_expressions():
    assert PAPER["delta_chaos"]["value"] == pytest.approx(1 / math.sqrt(2), rel=1e-15)
    assert PAPER["dt_bound_random_matrix"]["value"] == pytest.approx(math.sqrt(2), rel=1e-15)


def test_delta_levels():
    # eq. (8): half of the +-1 entries disagreeing is the typical state of two independent
    # random configurations and gives exactly the printed chaos level
    n = 4096
    rng = np.random.default_rng(3)
    a = rng.choice([-1.0, 1.0], n)
    b = a.copy()
    b[rng.permutation(n)[: n // 2]] *= -1
    assert abs(oracle.delta(a, b) - PAPER["delta_chaos"]["value"]) < 1e-15
    # the Sec. IV start: x^(2) = x^(1) shifted by 2 delta_0 in every coordinate
    x1 = rng.choice([-0.1, 0.1], n)
    x2 = x1 + rng.choice([-2.0, 2.0], n) * PAPER["delta_start"]["value"]
    assert abs(oracle.delta(x1, x2) - PAPER["delta_start"]["value"]) < 1e-15


def test_initial_state_range():
    h = PAPER["x0_halfwidth"]["value"]
    x, y = oracle.init_state(3000, 4, 11, oracle.INIT_X)
    assert np.all(np.abs(x) < h) and np.all(y == 0)
    assert np.abs(x).max() > 0.99 * h  # fills the interval rather than a narrower one


def test_random_pm1_matrix_step_size():
    # App. A: for a random +-1 matrix lambda_max ~ 2 sqrt(N) = -lambda_min, so c approaches
    # 1/(2 sqrt(N)), the eq. (12) bound approaches sqrt(2), and the library's eq. (13) step
    # with D_t = 1.25 approaches the fixed dt = 1.25 the paper uses for K2000.
    # Finite-N edge fluctuations are O(N^(-2/3)) relative; 4% covers N = 2000.
    n = 2000
    ctx = gsb.gsb_create(instances.dense_pm1(n, 2))
    try:
        lmax = gsb.gsb_get(ctx, gsb.GSB_OPT_LAMBDA_MAX)
        lmin = gsb.gsb_get(ctx, gsb.GSB_OPT_LAMBDA_MIN)
        c = gsb.gsb_get(ctx, gsb.GSB_OPT_C)
        dt = gsb.gsb_get(ctx, gsb.GSB_OPT_DT_STABLE)
    finally:
        gsb.gsb_destroy(ctx)
    assert abs(lmax / (2 * math.sqrt(n)) - 1) < 0.04 and abs(-lmin / (2 * math.sqrt(n)) - 1) < 0.04
    assert abs(c * 2 * math.sqrt(n) - 1) < 0.04
    bound = 2 / math.sqrt(1 - lmin / lmax)
    assert abs(bound / PAPER["dt_bound_random_matrix"]["value"] - 1) < 0.04
    assert abs(dt / PAPER["dt_K2000"]["value"] - 1) < 0.04
    assert PAPER["D_t"]["value"] == PAPER["dt_K2000"]["value"]
    assert PAPER["dt_K2000"]["value"] < bound  # inside the stability region


def test_tts_definition():
    from paper_2508_17655_amd import stats
    p99 = PAPER["tts_target"]["value"]
    assert stats.tts99(3.0, 0.995) == 3.0          # P_S above the target: one run
    assert stats.tts99(3.0, 1.0) == 3.0
    assert stats.tts99(3.0, 0.0) == math.inf
    # P_S = 0.5: ln(0.01)/ln(0.5) = 6.644 runs
    assert stats.tts99(1.0, 0.5) == pytest.approx(6.6439, abs=1e-4)
    # P_S = 1 - (1 - 0.99)^(1/k) needs exactly k runs: 1 - (1 - P_S)^k = 0.99
    for k in (2, 5, 40):
        ps = 1 - (1 - p99) ** (1 / k)
        assert stats.tts99(1.0, ps) == pytest.approx(k, rel=1e-12)
