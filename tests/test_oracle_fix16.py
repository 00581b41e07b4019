"""Pins of the oracle's 16-bit fixed-point operand form (FORM_FIX16; App. C runs the JX
product in 16-bit fixed point, the scale 2^-14 is this library's choice), independent of
its own formula:

- the quantiser equals numpy's round-half-to-even on the 2^-14 grid, including ties;
- operands already on the grid reach the product unchanged: a FIX16 run equals the
  exact-operand run bit for bit;
- sign products (dSB, GdSB) ignore the operand form;
- one step off the grid differs from the exact operand by no more than the quantisation
  bound c dt sum_j |J_ij| 2^-15 (a wrong scale, e.g. 2^-13, breaks it)."""
import numpy as np
import pytest

import oracle
from paper_2508_17655_amd import instances


def test_quantiser_is_round_half_even_on_the_grid():
    rng = np.random.default_rng(1)
    v = np.concatenate([rng.uniform(-1, 1, 2000), (np.arange(-40, 41) + 0.5) / 16384.0,  # exact ties
                        np.array([0.0, -0.0, 1.0, -1.0, 2.0 ** -15, 3 * 2.0 ** -15])])
    got = np.array([oracle.fix16_round(float(t)) for t in v])
    ref = np.rint(v * 16384.0) / 16384.0
    np.testing.assert_array_equal(got, ref)
    # ties go to the even multiple: 0.5 ulp -> 0, 1.5 ulp -> 2 ulp
    assert oracle.fix16_round(2.0 ** -15) == 0.0
    assert oracle.fix16_round(3 * 2.0 ** -15) == 2 * 2.0 ** -14


@pytest.mark.parametrize("mode", ["fp32", "fp64"])
def test_grid_operands_equal_the_exact_product(mode):
    n, R, M = 60, 3, 40
    J = instances.dense_pm1(n, 4).astype(np.float64)
    rng = np.random.default_rng(2)
    x = (rng.integers(-1600, 1601, size=(R, n)) / 16384.0).astype(np.float32)  # on the 2^-14 grid
    y = np.zeros((R, n), np.float32)
    kw = dict(A=0.2, dt=0.5, c=0.1, steps=M, x=x, y=y, m_end=1, mode=mode)
    a = oracle.run(J, oracle.GBSB, form=oracle.FORM_FIX16, **kw)
    b = oracle.run(J, oracle.GBSB, form=oracle.FORM_EXACT, **kw)
    for u, v in zip(a, b):
        np.testing.assert_array_equal(u, v)


def test_sign_products_ignore_the_form():
    n, R, M = 50, 4, 80
    J = instances.erdos_renyi_pm1(n, 0.2, 5).astype(np.float64)
    x0, y0 = oracle.init_state(n, R, 6)
    kw = dict(A=0.3, dt=0.7, c=0.15, steps=M, x=x0, y=y0, mode="fp32")
    a = oracle.run(J, oracle.GDSB, form=oracle.FORM_FIX16, **kw)
    b = oracle.run(J, oracle.GDSB, form=oracle.FORM_EXACT, **kw)
    for u, v in zip(a, b):
        np.testing.assert_array_equal(u, v)


def test_one_step_within_the_quantisation_bound():
    n, R, M, dt, c = 200, 4, 100, 0.8, 0.05
    J = instances.dense_pm1(n, 7).astype(np.float64)
    rng = np.random.default_rng(8)
    x = rng.uniform(-0.9, 0.9, size=(R, n))
    y = rng.uniform(-0.1, 0.1, size=(R, n))
    kw = dict(A=0.0, dt=dt, c=c, steps=M, x=x, y=y, m_end=1, mode="fp64")
    yf = oracle.run(J, oracle.BSB, form=oracle.FORM_FIX16, **kw)[1]
    ye = oracle.run(J, oracle.BSB, form=oracle.FORM_EXACT, **kw)[1]
    bound = c * dt * np.abs(J).sum(axis=1) * 2.0 ** -15
    diff = np.abs(yf - ye)
    assert np.all(diff <= bound[None, :] * (1 + 1e-12))
    # the bound is not vacuous: the rounding moves y by a sizeable part of it somewhere
    assert diff.max() > 0.05 * bound.max()
