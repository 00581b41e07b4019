"""GPU parity of the chaos diagnostics (through the C ABI): eq. (8) on the Sec. IV
trajectory pairs, and the tangent / largest-Lyapunov-exponent run."""
import numpy as np
import pytest

import oracle
from paper_2508_17655_amd import instances

pytestmark = pytest.mark.gpu


def _gsb():
    from paper_2508_17655_amd import gsb
    return gsb


def test_pairs_start_and_delta_zero():
    gsb = _gsb()
    n, R, seed = 333, 20, 41
    J = instances.dense_pm1(n, 5)
    g = gsb.GSB(J, precision="fp8", c=instances.paper_c(n), init_mode=gsb.GSB_INIT_PAIRS)
    g.init("gbsb", A=0.2, dt=1.25, replicas=R, steps=50, seed=seed)
    x, y, p, m = g.state()
    xo, yo = oracle.init_pairs(n, R // 2, seed)
    np.testing.assert_array_equal(x, xo)
    np.testing.assert_array_equal(y, yo)
    d = g.delta()
    ref = np.array([oracle.delta(xo[2 * k], xo[2 * k + 1]) for k in range(R // 2)])
    np.testing.assert_allclose(d, ref, rtol=1e-13, atol=0)
    assert np.all(np.abs(d - 1e-6) < 5e-9)
    g.close()


@pytest.mark.parametrize("variant", ["gbsb", "gdsb"])
def test_delta_after_run_matches_oracle(variant):
    gsb = _gsb()
    n, R, M, seed = 333, 24, 300, 42
    J = instances.dense_pm1(n, 6)
    c = instances.paper_c(n)
    g = gsb.GSB(J, precision="fp8", c=c, init_mode=gsb.GSB_INIT_PAIRS)
    g.run(variant, A=0.3, dt=1.25, replicas=R, steps=M, seed=seed)
    d = g.delta()
    xg = g.state()[0]
    x0, y0 = oracle.init_pairs(n, R // 2, seed)
    xo, yo, po = oracle.run(J.astype(np.float64), oracle.VARIANTS[variant], A=0.3, dt=1.25, c=c, steps=M, x=x0, y=y0,
                            form=oracle.FORM_E4M3, mode="fp32")[:3]
    np.testing.assert_array_equal(xg, xo)  # the E4M3 / sign forms are bit-exact
    ref = np.array([oracle.delta(xo[2 * k], xo[2 * k + 1]) for k in range(R // 2)])
    np.testing.assert_allclose(d, ref, rtol=1e-13, atol=0)
    assert np.all(d <= 1.0)
    g.close()


def _tangent_start(n, R, tseed):
    s = np.array([[oracle.splitmix64_at(tseed, r * n + i + 1) >> 63 for i in range(n)] for r in range(R)])
    return np.where(s == 1, -1.0, 1.0)


@pytest.mark.parametrize("variant,schedule", [("bsb", 1), ("gbsb", 0)])
def test_tangent_matches_oracle_short_horizon(variant, schedule):
    """Binary32 GPU vs binary64 oracle over 25 steps without wall contacts."""
    gsb = _gsb()
    n, R, T, dt, seed, tseed = 250, 40, 25, 0.5, 7, 99
    J = instances.dense_pm1(n, 8)
    lam = np.linalg.eigvalsh(J.astype(np.float64))
    c = 0.5 / lam[-1]
    A = np.linspace(0.0, 0.6, R)
    g = gsb.GSB(J, c=c)
    lle, st = g.lle(variant, A=A, dt=dt, replicas=R, steps=T, seed=seed, tangent_seed=tseed, renorm_every=7,
                    schedule=schedule, want_state=True)
    x0, y0 = oracle.init_state(n, R, seed, oracle.INIT_X)
    dx0 = _tangent_start(n, R, tseed)
    ref_x = np.empty((6, R, n))
    ref_lg = np.empty(R)
    for r in range(R):
        out = oracle.tangent_run(J.astype(np.float64), oracle.VARIANTS[variant], A=float(A[r]), dt=dt, c=c, steps=T,
                                 x=x0[r:r + 1], y=y0[r:r + 1], dx=dx0[r:r + 1], schedule=schedule, renorm=7)
        for k in range(6):
            ref_x[k, r] = out[k][0]
        ref_lg[r] = out[6][0]
    assert np.max(np.abs(ref_x[0])) < 0.95, "the window must stay away from the walls"
    for k in range(6):
        scale = np.max(np.abs(ref_x[k])) + 1e-30
        assert np.max(np.abs(st[k] - ref_x[k])) < 2e-5 * scale, k
    np.testing.assert_allclose(lle * T * dt, ref_lg, atol=2e-5, rtol=0)
    g.close()


def test_lle_window_matches_oracle():
    """GSB_OPT_LLE_FROM: growth counted from step m_w, against the oracle's tangent run over
    [0, m_w) followed by one over [m_w, T) from the state reached (binary32 vs binary64,
    no wall contacts in the window)."""
    gsb = _gsb()
    n, R, T, m_w, dt, seed, tseed = 250, 40, 25, 11, 0.5, 7, 99
    J = instances.dense_pm1(n, 8)
    lam = np.linalg.eigvalsh(J.astype(np.float64))
    c = 0.5 / lam[-1]
    A = np.linspace(0.0, 0.6, R)
    g = gsb.GSB(J, c=c)
    lle, st = g.lle("gbsb", A=A, dt=dt, replicas=R, steps=T, seed=seed, tangent_seed=tseed, renorm_every=7,
                    want_state=True, window_from=m_w)
    assert g.get(gsb.GSB_OPT_LLE_FROM) == m_w
    x0, y0 = oracle.init_state(n, R, seed, oracle.INIT_X)
    dx0 = _tangent_start(n, R, tseed)
    ref_lg = np.empty(R)
    for r in range(R):
        kw = dict(A=float(A[r]), dt=dt, c=c, steps=T, renorm=7)
        x1, y1, p1, dx1, dy1, dp1, _ = oracle.tangent_run(J.astype(np.float64), oracle.GBSB, x=x0[r:r + 1],
                                                          y=y0[r:r + 1], dx=dx0[r:r + 1], m_end=m_w, **kw)
        out = oracle.tangent_run(J.astype(np.float64), oracle.GBSB, x=x1, y=y1, p=p1, dx=dx1, dy=dy1, dp=dp1,
                                 m_begin=m_w, **kw)
        assert np.max(np.abs(out[0])) < 0.95, "the window must stay away from the walls"
        ref_lg[r] = out[6][0]
    np.testing.assert_allclose(lle * (T - m_w) * dt, ref_lg, atol=2e-5, rtol=0)
    # the whole-run estimate is back once the option is 0; a window start at or past the end
    # is rejected
    whole = g.lle("gbsb", A=A, dt=dt, replicas=R, steps=T, seed=seed, tangent_seed=tseed, renorm_every=7)
    assert not np.allclose(whole, lle)
    with pytest.raises(gsb.GsbError):
        g.lle("gbsb", A=A, dt=dt, replicas=R, steps=T, seed=seed, tangent_seed=tseed, window_from=T)
    with pytest.raises(gsb.GsbError):
        g.set(gsb.GSB_OPT_LLE_FROM, -1)
    g.close()


def test_lle_sweep_full_size_invariants():
    """N = 2000 dense +-1 (the benchmark instance), 8 control strengths x 8 replicas."""
    gsb = _gsb()
    n, T = 2000, 200
    J = instances.dense_pm1(n, 2)
    A = np.repeat(np.linspace(0.0, 0.7, 8), 8)
    g = gsb.GSB(J, c=instances.paper_c(n))
    lle, st = g.lle("gbsb", A=A, dt=1.25, replicas=A.size, steps=T, seed=3, tangent_seed=4, renorm_every=10,
                    want_state=True)
    assert np.all(np.isfinite(lle) | (lle == -np.inf))
    assert np.all(np.abs(st[0]) <= 1.0)
    tn = np.sqrt(np.sum(st[3].astype(np.float64) ** 2 + st[4] ** 2 + st[5] ** 2, axis=1))
    np.testing.assert_allclose(tn[np.isfinite(lle)], 1.0, rtol=1e-5)
    # a clamped component carries no tangent
    clamped = np.abs(st[0]) == 1.0
    assert np.all(st[3][clamped] == 0.0) and np.all(st[4][clamped] == 0.0)
    assert g.last_step_ms() > 0
    g.close()


def test_lle_rejects_sign_products_and_leaves_no_run():
    gsb = _gsb()
    J = instances.dense_pm1(64, 1)
    g = gsb.GSB(J)
    with pytest.raises(gsb.GsbError):
        g.lle("dsb", dt=0.5, replicas=4, steps=5, seed=1, tangent_seed=2)
    g.lle("bsb", dt=0.5, replicas=4, steps=5, seed=1, tangent_seed=2)
    with pytest.raises(gsb.GsbError):
        g.energy()  # no current run after an LLE run
    g.close()
