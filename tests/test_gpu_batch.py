"""GPU parity of batched uneven instances in one persistent launch (gsb_batch_*), through
the C ABI: every instance bit for bit against the oracle's E4M3 / sign forms and against
the single-instance FP8 path, for every tile shape, through a replayed HIP graph, after
autotuning, and on the full 256-instance workload (sampled)."""
import sys

import numpy as np
import pytest

import oracle
from paper_2508_17655_amd import instances

pytestmark = pytest.mark.gpu

# ragged; padded to 256 spins: 256 .. 2816, i.e. 2 to 22 k-steps, several of them not a
# multiple of the one-workgroup-per-CU variant's 4-k-step rounds (its unpipelined remainder)
SIZES = [64, 200, 333, 700, 1500, 2600]
R = 128


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _gsb():
    from paper_2508_17655_amd import gsb
    return gsb


def _instances(sizes, base_seed=100):
    """Even k dense +-1 with the semicircle c and dt = 1.25 (App. A); odd k sparse with c
    and dt left to the library (Lanczos, App. A and eq. (13))."""
    out = []
    for k, n in enumerate(sizes):
        if k % 2 == 0:
            out.append((instances.dense_pm1(n, base_seed + k), instances.paper_c(n), 1.25))
        else:
            out.append((instances.erdos_renyi_pm1(n, 0.05, base_seed + k), 0.0, 0.0))
    return out


def _batch(insts, replicas=R):
    gsb = _gsb()
    b = gsb.Batch([J.shape[0] for J, _, _ in insts], replicas)
    for k, (J, c, dt) in enumerate(insts):
        b.set_coupling(k, J, c, dt)
    return b


def _check_exact(a, b, what):
    a = np.asarray(a)
    b = np.asarray(b).astype(a.dtype)
    bad = np.flatnonzero(a.ravel() != b.ravel())
    assert bad.size == 0, f"{what}: {bad.size} mismatches, first at {bad[0]}: {a.ravel()[bad[0]]} vs {b.ravel()[bad[0]]}"


def _rows(n, R_):
    return np.arange(R_) if n <= 333 else np.array([0, R_ // 2 + 1, R_ - 1])


def _compare_with_oracle(b, insts, variant, A, M, seed, replicas=R):
    form = oracle.FORM_E4M3 if variant in ("gbsb", "bsb") else oracle.FORM_EXACT
    for k, (J, _, _) in enumerate(insts):
        n = J.shape[0]
        c, dt = b.params(k)
        rows = _rows(n, replicas)
        x0, y0 = oracle.init_state(n, replicas, seed + k)
        xo, yo, po = oracle.run(J.astype(np.float64), oracle.VARIANTS[variant], A=A, dt=dt, c=c, steps=M,
                                x=x0[rows], y=y0[rows], form=form, mode="fp32")
        x, y, p = b.state(k)
        _check_exact(x[rows], xo, f"instance {k} x")
        _check_exact(y[rows], yo, f"instance {k} y")
        _check_exact(p[rows], po, f"instance {k} p")
        E = b.energy(k)
        _check_exact(E[rows], oracle.energy(J.astype(np.float64), oracle.spins(xo)), f"instance {k} energies")
    e, r = b.best()
    for k in range(len(insts)):
        E = b.energy(k)
        assert e[k] == E.min() and r[k] == int(np.argmin(E))


@pytest.mark.parametrize("variant", ["gbsb", "gdsb"])
def test_batch_matches_oracle(variant):
    n_seed, M, A = 11, 60, 0.25
    say(f"case batch oracle variant={variant} sizes={SIZES} R={R} M={M}")
    insts = _instances(SIZES)
    b = _batch(insts)
    b.run(variant, A=A, steps=M, seed=n_seed)
    _compare_with_oracle(b, insts, variant, A, M, n_seed)
    # the library's c and dt for the sparse instances follow App. A and eq. (13)
    gsb = _gsb()
    for k in (1, 3):
        lmax = b.get(k, gsb.GSB_BATCH_LAMBDA_MAX)
        lmin = b.get(k, gsb.GSB_BATCH_LAMBDA_MIN)
        c, dt = b.params(k)
        assert c == 1.0 / lmax
        assert abs(dt - 1.25 * np.sqrt(2.0 / (1.0 - lmin / lmax))) < 1e-12
    b.close()


def test_every_tile_shape_gives_the_same_bits():
    gsb = _gsb()
    M, A, seed = 40, 0.2, 3
    say(f"case batch tiles sizes={SIZES} M={M}")
    insts = _instances(SIZES)
    b = _batch(insts)
    cap = int(b.get(-1, gsb.GSB_BATCH_GRID)) // 8  # workgroups of one XCD
    ref = None
    for rows in (64, 128, 256):
        for k, n in enumerate(SIZES):
            np_ = (n + 255) // 256 * 256
            b.set(k, gsb.GSB_BATCH_TILE_ROWS, rows if np_ // rows <= cap else 0)
        b.run("gbsb", A=A, steps=M, seed=seed)
        got = [b.state(k) for k in range(len(SIZES))]
        if ref is None:
            ref = got
            _compare_with_oracle(b, insts, "gbsb", A, M, seed)
        else:
            for k in range(len(SIZES)):
                for a, c_, what in zip(got[k], ref[k], "xyp"):
                    _check_exact(a, c_, f"tile {rows} instance {k} {what}")
    b.close()


def test_two_workgroups_per_cu_give_the_same_bits():
    gsb = _gsb()
    M, A, seed = 40, 0.2, 13
    say("case batch occupancy 1 vs 2")
    insts = _instances(SIZES)
    b = _batch(insts)
    b.set(-1, gsb.GSB_BATCH_OCCUPANCY, 1)
    b.run("gbsb", A=A, steps=M, seed=seed)
    ref = [b.state(k) for k in range(len(SIZES))]
    b.set(-1, gsb.GSB_BATCH_OCCUPANCY, 2)
    assert b.get(-1, gsb.GSB_BATCH_GRID) == 2 * b.get(-1, gsb.GSB_BATCH_GRID) // 2
    for rows in (64, 128, 256):  # the wider XCD queues also admit 64-row tiles of larger instances
        for k in range(len(SIZES)):
            b.set(k, gsb.GSB_BATCH_TILE_ROWS, rows)
        b.run("gbsb", A=A, steps=M, seed=seed)
        for k in range(len(SIZES)):
            for a_, c_, what in zip(b.state(k), ref[k], "xyp"):
                _check_exact(a_, c_, f"occupancy 2 tile {rows} instance {k} {what}")
    _compare_with_oracle(b, insts, "gbsb", A, M, seed)
    b.close()


def test_batch_equals_single_instance_path():
    gsb = _gsb()
    M, A, seed = 50, 0.3, 21
    say("case batch vs single-instance FP8")
    insts = _instances(SIZES[:4])
    b = _batch(insts)
    b.run("gbsb", A=A, steps=M, seed=seed)
    for k, (J, _, _) in enumerate(insts):
        c, dt = b.params(k)
        g = gsb.GSB(J, precision="fp8", c=c)
        g.run("gbsb", A=A, dt=dt, replicas=R, steps=M, seed=seed + k)
        xs, ys, ps, _ = g.state()
        Es = g.energy()
        g.close()
        x, y, p = b.state(k)
        for a, c_, what in ((x, xs, "x"), (y, ys, "y"), (p, ps, "p"), (b.energy(k), Es, "E")):
            _check_exact(a, c_, f"instance {k} {what}")
    b.close()


def test_graph_replays_equal_the_eager_run():
    import torch

    gsb = _gsb()
    M, A = 40, 0.2
    say("case batch graph replay")
    insts = _instances(SIZES)
    b = _batch(insts)
    b.run("gbsb", A=A, steps=M, seed=5)
    eager = [(b.state(k), b.energy(k)) for k in range(len(SIZES))]
    eager_best = b.best()
    b.set(-1, gsb.GSB_BATCH_GRAPH, 1)
    for rep in range(3):
        b.run("gbsb", A=A, steps=M, seed=5)  # first: capture and launch; then replays
        for k in range(len(SIZES)):
            (x, y, p), E = b.state(k), b.energy(k)
            for a, c_, what in zip((x, y, p, E), (*eager[k][0], eager[k][1]), ("x", "y", "p", "E")):
                _check_exact(a, c_, f"replay {rep} instance {k} {what}")
        e, r = b.best()
        _check_exact(e, eager_best[0], "best energies")
        _check_exact(r, eager_best[1], "best replicas")
        assert b.last_ms() > 0
        # the program's own eager work between replays
        t = torch.arange(1 << 20, device="cuda", dtype=torch.float32)
        assert float((t * 2).sum()) > 0
        torch.cuda.synchronize()
    # another seed is a new capture and still equals the oracle
    b.run("gbsb", A=A, steps=M, seed=9)
    _compare_with_oracle(b, insts, "gbsb", A, M, 9)
    b.close()


def test_autotune_measures_every_instance_and_keeps_results_exact():
    gsb = _gsb()
    M, A, seed = 40, 0.2, 7
    say("case batch autotune")
    insts = _instances(SIZES)
    b = _batch(insts)
    b.autotune("gbsb", A=A, trial_steps=20, seed=1)
    for k in range(len(SIZES)):
        rows = b.get(k, gsb.GSB_BATCH_TILE_ROWS)
        assert rows in (64, 128, 256)
        assert b.get(k, gsb.GSB_BATCH_STEP_US) > 0
    b.run("gbsb", A=A, steps=M, seed=seed)
    _compare_with_oracle(b, insts, "gbsb", A, M, seed)
    b.close()


def test_edge_sizes_and_few_replicas():
    """n = 1 (no coupling at all), n = 8192 (the largest), 5 replicas (padded to 128)."""
    gsb = _gsb()
    M, A, seed, reps = 12, 0.2, 4, 5
    say("case batch edges n=[1, 8192, 130] R=5")
    insts = [(np.zeros((1, 1), np.float32), 0.5, 1.25), (instances.dense_pm1(8192, 3), instances.paper_c(8192), 1.25),
             (instances.dense_pm1(130, 4), instances.paper_c(130), 1.25)]
    b = _batch(insts, replicas=reps)
    assert b.get(1, gsb.GSB_BATCH_TILE_ROWS) in (128, 256)
    b.run("gbsb", A=A, steps=M, seed=seed)
    for k, (J, c, dt) in enumerate(insts):
        n = J.shape[0]
        rows = np.arange(reps) if n < 8192 else np.array([0, reps - 1])
        x0, y0 = oracle.init_state(n, reps, seed + k)
        xo, yo, po = oracle.run(J.astype(np.float64), oracle.GBSB, A=A, dt=dt, c=c, steps=M, x=x0[rows], y=y0[rows],
                                form=oracle.FORM_E4M3, mode="fp32")
        x, y, p = b.state(k)
        assert x.shape == (reps, n)
        _check_exact(x[rows], xo, f"edge instance {k} x")
        _check_exact(y[rows], yo, f"edge instance {k} y")
        _check_exact(p[rows], po, f"edge instance {k} p")
    assert np.all(b.energy(0) == 0.0)
    b.close()


def test_full_workload_sampled():
    """256 instances, n iid U{64..4096}, half dense, half sparse, 128 replicas, 1000 steps
    (the launch the benchmark times): the smallest instance in full and one replica of a
    mid-sized sparse instance against the oracle; invariants on all."""
    gsb = _gsb()
    M, A, seed = 1000, 0.2, 1
    specs = instances.batch_workload(256, 1)
    say("case batch full workload: 256 instances, R=128, M=1000")
    b = gsb.Batch([s[1] for s in specs], R)

    def make(k):
        J = instances.make_instance(specs[k])
        if specs[k][0] == "dense":
            return J, instances.paper_c(specs[k][1]), 1.25
        return J, 0.0, 0.0

    b.set_couplings(make, threads=16)
    b.run("gbsb", A=A, steps=M, seed=seed)
    assert b.last_ms() > 0
    e, r = b.best()
    assert np.all(e < 0) and np.all((r >= 0) & (r < R))
    ns = np.array([s[1] for s in specs])
    small = int(np.argmin(ns))
    mid = [int(k) for k in np.argsort(ns) if specs[k][0] == "sparse"][128 // 2]
    for k, rows in ((small, np.arange(R)), (mid, np.array([R - 1]))):
        J = instances.make_instance(specs[k])
        n = J.shape[0]
        c, dt = b.params(k)
        say(f"  oracle instance {k} n={n} rows={rows.size}")
        x0, y0 = oracle.init_state(n, R, seed + k)
        xo, yo, po = oracle.run(J.astype(np.float64), oracle.GBSB, A=A, dt=dt, c=c, steps=M, x=x0[rows], y=y0[rows],
                                form=oracle.FORM_E4M3, mode="fp32")
        x, y, p = b.state(k)
        _check_exact(x[rows], xo, f"instance {k} x")
        _check_exact(y[rows], yo, f"instance {k} y")
        _check_exact(p[rows], po, f"instance {k} p")
        assert np.all(np.abs(x) <= 1.0)
    b.close()


def test_many_ragged_replicas():
    """1000 replicas per instance (padded to 1024: 8 to 32 replica groups per instance,
    depending on the tile), sign and E4M3 products, sampled replicas against the oracle."""
    gsb = _gsb()
    M, A, seed, reps = 30, 0.3, 17, 1000
    say("case batch R=1000 sizes=[150, 1100]")
    insts = [(instances.dense_pm1(150, 21), instances.paper_c(150), 1.25),
             (instances.erdos_renyi_pm1(1100, 0.03, 22), 0.0, 0.0)]
    b = _batch(insts, replicas=reps)
    for variant, form in (("gdsb", oracle.FORM_EXACT), ("gbsb", oracle.FORM_E4M3)):
        b.run(variant, A=A, steps=M, seed=seed)
        for k, (J, _, _) in enumerate(insts):
            n = J.shape[0]
            c, dt = b.params(k)
            rows = np.array([0, 511, 512, 999])
            x0, y0 = oracle.init_state(n, reps, seed + k)
            xo, yo, po = oracle.run(J.astype(np.float64), oracle.VARIANTS[variant], A=A, dt=dt, c=c, steps=M,
                                    x=x0[rows], y=y0[rows], form=form, mode="fp32")
            x, y, p = b.state(k)
            assert x.shape == (reps, n)
            _check_exact(x[rows], xo, f"{variant} instance {k} x")
            _check_exact(y[rows], yo, f"{variant} instance {k} y")
            E = b.energy(k)
            assert E.shape == (reps,)
            _check_exact(E[rows], oracle.energy(J.astype(np.float64), oracle.spins(xo)), f"{variant} instance {k} E")
        e, r = b.best()
        assert np.all((r >= 0) & (r < reps))
    b.close()
