"""Pins of the oracle's chaos diagnostics and step derivatives (CPU only).

- Trajectory pairs of Sec. IV: delta(0) = 1e-6 (eq. (8)), x1 is the +-0.1 start.
- Tangent of the step vs central finite differences of the binary64 dynamics (T = 20
  steps, eps = 1e-6, no wall contact in the window).
- Adjoint vs tangent: <T u, w> = <u, T^T w> for one and several steps, with and without
  wall contacts.
- Largest-Lyapunov-exponent estimate in the linear regime: bSB with constant p = 1 from
  the fixed point x = y = 0 has the tangent dynamics of eq. (10) mode by mode, so its
  log growth equals the one obtained from the eigenmodes of J (numpy eigh) and 2 x 2
  mode matrices, and tends to ln r_max / dt with r^2 - (2 - k dt^2) r + 1 = 0,
  k = p - c lambda_max.
- The window estimate (growth counted from a step m_w on) against the same eigenmode
  propagation with its log sums started at m_w, and the growths of two intervals adding
  up to that of their union.
"""
import numpy as np
import pytest

import oracle
from paper_2508_17655_amd import instances


def _sym_pm1(n, seed):
    return instances.dense_pm1(n, seed).astype(np.float64)


def test_pairs_start():
    n, pairs, seed = 500, 3, 11
    x, y = oracle.init_pairs(n, pairs, seed)
    xs, ys = oracle.init_state(n, pairs, seed, oracle.INIT_PM01)
    for k in range(pairs):
        np.testing.assert_array_equal(x[2 * k], xs[k])
        assert np.all(y[2 * k] == 0) and np.all(y[2 * k + 1] == 0)
        d = x[2 * k + 1].astype(np.float64) - x[2 * k].astype(np.float64)
        assert np.all(np.abs(np.abs(d) - 2e-6) < 1e-8)
        # delta(0) = 1e-6 (eq. (8) with |x1 - x2| = 2e-6), up to the binary32 rounding of x2
        assert abs(oracle.delta(x[2 * k], x[2 * k + 1]) - 1e-6) < 5e-3 * 1e-6
    # the perturbation signs are random and independent of the base signs
    d = (x[1] - x[0]) > 0
    assert 0.3 < d.mean() < 0.7


def _primal(J, variant, A, dt, c, M, m0, m1, x, y, p):
    r = oracle.run(J, variant, A=A, dt=dt, c=c, steps=M, x=x, y=y, p=p, m_begin=m0, m_end=m1, mode="fp64")
    return r[0], r[1], r[2]


@pytest.mark.parametrize("variant,A", [(oracle.BSB, 0.0), (oracle.GBSB, 0.3)])
def test_tangent_matches_finite_differences(variant, A):
    n, M, T, dt = 40, 200, 20, 0.5
    J = _sym_pm1(n, 3)
    c = 0.5 / np.max(np.abs(np.linalg.eigvalsh(J)))
    rng = np.random.default_rng(4)
    x0 = rng.uniform(-0.05, 0.05, size=(1, n))
    y0 = rng.uniform(-0.05, 0.05, size=(1, n))
    p0 = np.ones((1, n))
    u = rng.standard_normal((3, n))
    u /= np.linalg.norm(u)
    xt, yt, pt, dx, dy, dp, lg = oracle.tangent_run(J, variant, A=A, dt=dt, c=c, steps=M, x=x0, y=y0, p=p0,
                                                   dx=u[0:1], dy=u[1:2], dp=u[2:3], m_end=T, renorm=0)
    assert np.max(np.abs(xt)) < 0.9, "the window must not touch a wall"
    scale = np.exp(lg[0])
    eps = 1e-6
    plus = _primal(J, variant, A, dt, c, M, 0, T, x0 + eps * u[0], y0 + eps * u[1], p0 + eps * u[2])
    minus = _primal(J, variant, A, dt, c, M, 0, T, x0 - eps * u[0], y0 - eps * u[1], p0 - eps * u[2])
    for k, tang in enumerate((dx, dy, dp)):
        fd = (plus[k] - minus[k]) / (2 * eps)
        ref = np.max(np.abs(fd)) + 1e-300
        assert np.max(np.abs(fd - scale * tang)) < 1e-6 * ref, k


def _tangent_map(J, variant, A, dt, c, M, m, x, y, p, u):
    """T u for one step at state (x, y, p) and step index m (u stacked as (dx, dy, dp))."""
    *_, dx, dy, dp, lg = oracle.tangent_run(J, variant, A=A, dt=dt, c=c, steps=M, x=x, y=y, p=p, dx=u[0:1],
                                            dy=u[1:2], dp=u[2:3], m_begin=m, m_end=m + 1, renorm=0)
    return np.concatenate([dx, dy, dp]) * np.exp(lg[0]) * np.linalg.norm(u)


@pytest.mark.parametrize("near_wall", [False, True])
def test_adjoint_is_the_transpose_of_the_tangent(near_wall):
    n, M, dt, A = 30, 50, 0.7, 0.4
    J = _sym_pm1(n, 8)
    c = 1.5 / np.max(np.abs(np.linalg.eigvalsh(J)))
    rng = np.random.default_rng(9)
    amp = 0.98 if near_wall else 0.1
    x = rng.uniform(-amp, amp, size=(1, n))
    y = rng.uniform(-0.5, 0.5, size=(1, n)) if near_wall else rng.uniform(-0.05, 0.05, size=(1, n))
    p = rng.uniform(0.2, 1.0, size=(1, n))
    m = 7
    rm = 1.0 / (M - m)
    # does this step touch a wall?
    x1 = _primal(J, oracle.GBSB, A, dt, c, M, m, m + 1, x, y, p)[0]
    hits = int(np.sum(np.abs(x1) == 1.0))
    assert (hits > 0) == near_wall
    for trial in range(3):
        u = rng.standard_normal((3, n))
        w = rng.standard_normal((3, n))
        tu = _tangent_map(J, oracle.GBSB, A, dt, c, M, m, x, y, p, u)
        xb, yb, pb = oracle.adjoint_step(J, oracle.GBSB, A=A, dt=dt, c=c, rm=rm, x=x[0], y=y[0], p=p[0],
                                         xb=w[0], yb=w[1], pb=w[2])
        lhs = float(np.sum(tu * w))
        rhs = float(np.sum(u[0] * xb) + np.sum(u[1] * yb) + np.sum(u[2] * pb))
        assert abs(lhs - rhs) < 1e-12 * (abs(lhs) + np.linalg.norm(tu) * np.linalg.norm(w))


def test_adjoint_over_several_steps():
    n, M, dt, A, K = 24, 40, 0.6, 0.25, 6
    J = _sym_pm1(n, 12)
    c = 0.8 / np.max(np.abs(np.linalg.eigvalsh(J)))
    rng = np.random.default_rng(13)
    x = rng.uniform(-0.3, 0.3, size=(1, n))
    y = rng.uniform(-0.1, 0.1, size=(1, n))
    p = np.ones((1, n))
    states = []
    for m in range(K):  # checkpoints of every step's input
        states.append((x.copy(), y.copy(), p.copy()))
        x, y, p = _primal(J, oracle.GBSB, A, dt, c, M, m, m + 1, x, y, p)
    u = rng.standard_normal((3, n))
    w = rng.standard_normal((3, n))
    v = u.copy()
    for m in range(K):
        v = _tangent_map(J, oracle.GBSB, A, dt, c, M, m, *states[m], v)
    b = w.copy()
    for m in reversed(range(K)):
        xs, ys, ps = states[m]
        b = np.stack(oracle.adjoint_step(J, oracle.GBSB, A=A, dt=dt, c=c, rm=1.0 / (M - m), x=xs[0], y=ys[0],
                                         p=ps[0], xb=b[0], yb=b[1], pb=b[2]))
    lhs = float(np.sum(v * w))
    rhs = float(np.sum(u * b))
    assert abs(lhs - rhs) < 1e-11 * (abs(lhs) + np.linalg.norm(v) * np.linalg.norm(w))


def test_lle_linear_regime_closed_form():
    """bSB, constant p = 1, primal at the fixed point x = y = 0: every eigenmode k of J
    evolves as [a; b] <- [[1 - k dt^2, dt], [-k dt, 1]] [a; b] with k = p - c lambda."""
    n, T, dt = 32, 300, 0.5
    J = _sym_pm1(n, 21)
    lam, V = np.linalg.eigh(J)
    c = 2.0 / lam[-1]
    rng = np.random.default_rng(22)
    u = rng.standard_normal(n)
    u /= np.linalg.norm(u)
    z = np.zeros((1, n))
    *_, dx, dy, dp, lg = oracle.tangent_run(J, oracle.BSB, dt=dt, c=c, steps=T, x=z, y=z, p=np.ones((1, n)),
                                            dx=u[None, :], schedule=oracle.SCHED_CONSTANT, renorm=10)
    # mode propagation with numpy
    a = V.T @ u
    b = np.zeros(n)
    logs = 0.0
    for t in range(T):
        k = 1.0 - c * lam
        a, b = (1.0 - k * dt * dt) * a + dt * b, -k * dt * a + b
        if (t + 1) % 10 == 0:
            s = np.sqrt(np.sum(a * a) + np.sum(b * b))
            logs += np.log(s)
            a /= s
            b /= s
    assert abs(lg[0] - logs) < 1e-9 * abs(logs)
    assert np.all(dp == 0.0)
    # and the exponent approaches ln r_max / dt of the top mode (k = 1 - 2 = -1)
    kk = -1.0
    q = 2.0 - kk * dt * dt
    r_max = (q + np.sqrt(q * q - 4.0)) / 2.0
    lle = lg[0] / (T * dt)
    assert abs(lle - np.log(r_max) / dt) < 0.02 * np.log(r_max) / dt


def test_lle_window_is_the_growth_after_its_start():
    """The post-bifurcation window estimate: the tangent run over [0, m_w), then over
    [m_w, T) from the state reached, counts only the second interval's growth.  In the
    linear regime of the test above that is the eigenmode propagation with the log sums
    started at m_w; and the two intervals' growths add up to the one-interval growth."""
    n, T, m_w, dt = 32, 300, 120, 0.5
    J = _sym_pm1(n, 23)
    lam, V = np.linalg.eigh(J)
    c = 1.5 / lam[-1]
    rng = np.random.default_rng(24)
    u = rng.standard_normal(n)
    z = np.zeros((1, n))
    one = np.ones((1, n))
    kw = dict(dt=dt, c=c, steps=T, schedule=oracle.SCHED_CONSTANT, renorm=10)
    *_, lg_all = oracle.tangent_run(J, oracle.BSB, x=z, y=z, p=one, dx=u[None, :], **kw)
    x1, y1, p1, dx1, dy1, dp1, lg_a = oracle.tangent_run(J, oracle.BSB, x=z, y=z, p=one, dx=u[None, :], m_end=m_w,
                                                         **kw)
    *_, lg_b = oracle.tangent_run(J, oracle.BSB, x=x1, y=y1, p=p1, dx=dx1, dy=dy1, dp=dp1, m_begin=m_w, **kw)
    assert abs((lg_a[0] + lg_b[0]) - lg_all[0]) < 1e-11 * abs(lg_all[0])
    a = V.T @ (u / np.linalg.norm(u))
    b = np.zeros(n)
    logs = 0.0
    k = 1.0 - c * lam
    for t in range(T):
        a, b = (1.0 - k * dt * dt) * a + dt * b, -k * dt * a + b
        if t + 1 == m_w:  # the window starts: unit norm, log sums from 0
            s = np.sqrt(np.sum(a * a) + np.sum(b * b))
            a /= s
            b /= s
        elif t + 1 > m_w and ((t + 1 - m_w) % 10 == 0 or t + 1 == T):
            s = np.sqrt(np.sum(a * a) + np.sum(b * b))
            logs += np.log(s)
            a /= s
            b /= s
    assert abs(lg_b[0] - logs) < 1e-9 * abs(logs)


def test_gbsb_at_zero_control_is_bsb():
    n, M, dt = 20, 60, 0.5
    J = _sym_pm1(n, 30)
    c = 0.7 / np.max(np.abs(np.linalg.eigvalsh(J)))
    rng = np.random.default_rng(31)
    x = rng.uniform(-0.1, 0.1, size=(2, n))
    u = rng.standard_normal((2, n))
    r1 = oracle.tangent_run(J, oracle.BSB, dt=dt, c=c, steps=M, x=x, y=np.zeros_like(x), dx=u, renorm=5)
    r2 = oracle.tangent_run(J, oracle.GBSB, A=0.0, dt=dt, c=c, steps=M, x=x, y=np.zeros_like(x), dx=u, renorm=5)
    for a, b in zip(r1, r2):
        np.testing.assert_array_equal(a, b)


def test_tangent_rejects_sign_products():
    J = _sym_pm1(8, 1)
    with pytest.raises(ValueError):
        oracle.tangent_run(J, oracle.DSB, dt=0.5, c=0.1, steps=4, x=np.zeros((1, 8)), y=np.zeros((1, 8)),
                           dx=np.ones((1, 8)))
