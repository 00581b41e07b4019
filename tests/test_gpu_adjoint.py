"""GPU reverse pass (gsb_vjp) and its torch.autograd wrapper, against the oracle's
adjoint composed over a binary64 trajectory, and against finite differences."""
import numpy as np
import pytest

import oracle
from paper_2508_17655_amd import instances

pytestmark = pytest.mark.gpu


def _gsb():
    from paper_2508_17655_amd import gsb
    return gsb


def _oracle_vjp(J, variant, A, dt, c, M, x0, y0, p0, xb, yb, pb):
    """Compose the oracle's one-step adjoint over the binary64 trajectory from (x0, y0, p0)."""
    states = []
    x, y, p = x0.astype(np.float64), y0.astype(np.float64), p0.astype(np.float64)
    for m in range(M):
        states.append((x.copy(), y.copy(), p.copy()))
        x, y, p = oracle.run(J, variant, A=A, dt=dt, c=c, steps=M, x=x, y=y, p=p, m_begin=m, m_end=m + 1,
                             mode="fp64")
    xb, yb, pb = (v.astype(np.float64) for v in (xb, yb, pb))
    out_x, out_y, out_p = np.empty_like(xb), np.empty_like(yb), np.empty_like(pb)
    for r in range(x0.shape[0]):
        b = (xb[r], yb[r], pb[r])
        for m in reversed(range(M)):
            xs, ys, ps = states[m]
            b = oracle.adjoint_step(J, variant, A=A, dt=dt, c=c, rm=1.0 / (M - m), x=xs[r], y=ys[r], p=ps[r],
                                    xb=b[0], yb=b[1], pb=b[2])
        out_x[r], out_y[r], out_p[r] = b
    return out_x, out_y, out_p, states, (x, y, p)


@pytest.mark.parametrize("variant", ["bsb", "gbsb"])
def test_vjp_matches_oracle_without_walls(variant):
    gsb = _gsb()
    n, R, M, dt, seed = 250, 16, 15, 0.5, 5
    J = instances.dense_pm1(n, 8).astype(np.float64)
    c = 0.5 / np.linalg.eigvalsh(J)[-1]
    g = gsb.GSB(J, precision="fp32", c=c)
    g.init(variant, A=0.4, dt=dt, replicas=R, steps=M, seed=seed)
    x0, y0, p0, _ = g.state()
    rng = np.random.default_rng(6)
    xb, yb, pb = (rng.standard_normal((R, n)).astype(np.float32) for _ in range(3))
    gx, gy, gp = g.vjp(M, xb, yb, pb)
    ox, oy, op, _, (xT, _, _) = _oracle_vjp(J, gsb.VARIANTS[variant], 0.4 if variant == "gbsb" else 0.0, dt, c, M,
                                            x0, y0, p0, xb, yb, pb)
    assert np.max(np.abs(xT)) < 0.95
    for a, b in ((gx, ox), (gy, oy), (gp, op)):
        assert np.max(np.abs(a - b)) < 1e-4 * np.max(np.abs(b))
    # the run did not advance
    assert g.state()[3] == 0
    g.close()


def test_vjp_matches_oracle_with_walls():
    gsb = _gsb()
    n, R, M, dt, seed, A = 96, 8, 12, 0.9, 9, 0.3
    J = instances.dense_pm1(n, 10).astype(np.float64)
    c = 1.2 / np.linalg.eigvalsh(J)[-1]
    g = gsb.GSB(J, precision="fp32", c=c, init_mode=gsb.GSB_INIT_XY)
    g.init("gbsb", A=A, dt=dt, replicas=R, steps=M, seed=seed)
    x0, y0, p0, _ = g.state()
    rng = np.random.default_rng(10)
    xb, yb, pb = (rng.standard_normal((R, n)).astype(np.float32) for _ in range(3))
    gx, gy, gp = g.vjp(M, xb, yb, pb)
    ox, oy, op, states, _ = _oracle_vjp(J, oracle.GBSB, A, dt, c, M, x0, y0, p0, xb, yb, pb)
    # the GPU trajectory meets the walls exactly where the binary64 one does
    walls = 0
    for m in range(1, M):
        g.step(1)
        xg = g.state()[0]
        np.testing.assert_array_equal(np.abs(xg) == 1.0, np.abs(states[m][0]) == 1.0)
        walls += int(np.sum(np.abs(xg) == 1.0))
    assert walls > 0, "this case must exercise the wall"
    for a, b in ((gx, ox), (gy, oy), (gp, op)):
        assert np.max(np.abs(a - b)) < 2e-4 * np.max(np.abs(b))
    g.close()


def _checkpointed_grads(device):
    """Gradients of a weighted sum of x(T), y(T) through autograd segments of 5 steps, the
    one-pass reverse reference (host gsb_vjp over all M steps), and a central difference."""
    import torch

    from paper_2508_17655_amd import autograd as sbad

    n, R, M, dt = 200, 8, 15, 0.5
    J = instances.dense_pm1(n, 11).astype(np.float64)
    c = 0.5 / np.linalg.eigvalsh(J)[-1]
    g, x0, y0, p0 = sbad.start(J, "gbsb", A=0.3, dt=dt, replicas=R, steps=M, seed=12, c=c, device=device)
    assert x0.device.type == torch.device(device).type
    rng = np.random.default_rng(13)
    wgt = torch.from_numpy(rng.standard_normal((R, n)).astype(np.float32)).to(device)

    def loss(x, y, p, every):
        xT, yT, pT = sbad.trajectory(g, x, y, p, M, every=every)
        assert xT.device == x0.device
        return (wgt * xT).sum() + 0.5 * (wgt * yT).sum()

    xs = x0.clone().requires_grad_(True)
    ys = y0.clone().requires_grad_(True)
    L = loss(xs, ys, p0, every=5)
    L.backward()
    assert xs.grad.device == x0.device
    # one reverse pass over all M steps
    g.set_state(x0.cpu().numpy(), y0.cpu().numpy(), p0.cpu().numpy(), 0)
    wn = wgt.cpu().numpy()
    gx, gy, _ = g.vjp(M, wn, 0.5 * wn, np.zeros((R, n), np.float32))
    u = torch.from_numpy(rng.standard_normal((R, n)).astype(np.float32)).to(device)
    u /= u.norm()
    eps = 1e-3
    with torch.no_grad():
        lp = float(loss(x0 + eps * u, y0, p0, every=M))
        lm = float(loss(x0 - eps * u, y0, p0, every=M))
    fd = (lp - lm) / (2 * eps)
    an = float((xs.grad * u).sum())
    g.close()
    return xs.grad.cpu().numpy(), ys.grad.cpu().numpy(), gx, gy, fd, an


def test_checkpointed_segments_equal_one_pass_and_finite_differences():
    """Host tensors and CUDA tensors (the device-resident path: no host copies of the state
    or the cotangents) give the same gradients, bit for bit, equal to the one-pass reverse
    pass and to central differences."""
    res = {}
    for device in ("cpu", "cuda"):
        gxs, gys, gx, gy, fd, an = _checkpointed_grads(device)
        np.testing.assert_allclose(gxs, gx, rtol=1e-5, atol=1e-6 * np.max(np.abs(gx)))
        np.testing.assert_allclose(gys, gy, rtol=1e-5, atol=1e-6 * np.max(np.abs(gy)))
        assert abs(fd - an) < 1e-2 * abs(an) + 1e-3
        res[device] = (gxs, gys)
    np.testing.assert_array_equal(res["cpu"][0], res["cuda"][0])
    np.testing.assert_array_equal(res["cpu"][1], res["cuda"][1])


def test_device_state_round_trip_and_checks():
    import torch

    gsb = _gsb()
    n, R = 150, 6
    J = instances.dense_pm1(n, 3)
    g = gsb.GSB(J, precision="fp32")
    g.init("gbsb", A=0.2, dt=0.5, replicas=R, steps=20, seed=4)
    g.step(7)
    xh, yh, ph, m = g.state()
    x, y, p = (torch.empty((R, n), dtype=torch.float32, device="cuda") for _ in range(3))
    assert g.state_device(x, y, p) == 7
    for a, b in ((x, xh), (y, yh), (p, ph)):
        np.testing.assert_array_equal(a.cpu().numpy(), b)
    # a state set from the device continues as the host one does
    g.set_state_device(x, y, p, 7)
    g.step(5)
    x1 = g.state()[0]
    g.set_state(xh, yh, ph, 7)
    g.step(5)
    np.testing.assert_array_equal(g.state()[0], x1)
    # the device-side checks: non-finite entries, |x| > 1, shapes; the state is left alone
    before = g.state()
    bad = y.clone()
    bad[2, 5] = float("nan")
    with pytest.raises(gsb.GsbError, match="ENONFINITE"):
        g.set_state_device(x, bad, p, 3)
    big = x.clone()
    big[R - 1, n - 1] = 1.5
    with pytest.raises(gsb.GsbError, match="EINVAL"):
        g.set_state_device(big, y, p, 3)
    with pytest.raises(ValueError):
        g.set_state_device(x[:, :-1].contiguous(), y, p, 3)
    after = g.state()
    for a, b in zip(before, after):
        np.testing.assert_array_equal(np.asarray(a), np.asarray(b))
    g.close()


def test_vjp_rejects_other_forms():
    gsb = _gsb()
    J = instances.dense_pm1(64, 1)
    g = gsb.GSB(J, precision="fp8")
    g.init("gbsb", A=0.2, dt=0.5, replicas=4, steps=5, seed=1)
    with pytest.raises(gsb.GsbError):
        g.vjp(2, *(np.zeros((4, 64), np.float32) for _ in range(3)))
    g.close()
