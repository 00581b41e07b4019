"""Host logic of the batched path (no GPU): the queue plan, argument checking, and the
sparse form of the eigenvalue estimate that sets c and dt (App. A, eq. (13))."""
import numpy as np
import pytest

from paper_2508_17655_amd import gsb, instances


def _plan_case(units, queues, workers, seed):
    rng = np.random.default_rng(seed)
    width = rng.integers(1, workers + 1, size=units)
    gangs = rng.integers(1, 5, size=units)
    cost = rng.uniform(0.5, 10.0, size=units)
    q, r = gsb.gsb_batch_plan(width, gangs, cost, queues, workers)
    return width, gangs, cost, q, r


@pytest.mark.parametrize("units,queues,workers,seed", [(1, 8, 32, 0), (7, 8, 32, 1), (256, 8, 64, 2), (300, 3, 5, 3)])
def test_plan_is_a_valid_lpt_schedule(units, queues, workers, seed):
    width, gangs, cost, q, r = _plan_case(units, queues, workers, seed)
    assert np.all((q >= 0) & (q < queues))
    work = gangs * width * cost
    load = np.zeros(queues)
    for qq in range(queues):
        mine = np.flatnonzero(q == qq)
        # ranks are 0..len-1 within a queue, in decreasing cost
        assert sorted(r[mine].tolist()) == list(range(mine.size))
        order = mine[np.argsort(r[mine])]
        assert np.all(np.diff(cost[order]) <= 0)
        load[qq] = work[mine].sum()
    # list scheduling bound: no queue exceeds the mean by more than the largest unit
    assert load.max() <= work.sum() / queues + work.max() + 1e-9


def test_plan_lpt_order_matches_greedy_by_hand():
    # units of work 8, 7, 6, 5, 4 on 2 queues: 8 -> q0, 7 -> q1, 6 -> q1 (7 < 8), 5 -> q0, 4 -> q1 (13 = 13 -> q0)
    width = [1, 1, 1, 1, 1]
    gangs = [1, 1, 1, 1, 1]
    cost = [8.0, 7.0, 6.0, 5.0, 4.0]
    q, r = gsb.gsb_batch_plan(width, gangs, cost, 2, 4)
    assert q.tolist() == [0, 1, 1, 0, 0]
    assert r.tolist() == [0, 0, 1, 1, 2]


def test_plan_rejects_a_gang_wider_than_a_queue():
    with pytest.raises(gsb.GsbError) as e:
        gsb.gsb_batch_plan([33], [1], [1.0], 8, 32)
    assert e.value.status == gsb.GSB_EUNSUPPORTED
    with pytest.raises(gsb.GsbError):
        gsb.gsb_batch_plan([1], [0], [1.0], 8, 32)


def test_batch_arguments_are_checked_before_any_device_work():
    with pytest.raises(gsb.GsbError):
        gsb.gsb_batch_create([10, 0], 16)
    with pytest.raises(gsb.GsbError):
        gsb.gsb_batch_create([10, 9000], 16)
    with pytest.raises(gsb.GsbError):
        gsb.gsb_batch_create([10], 0)
    b = gsb.gsb_batch_create([12, 30], 16)
    try:
        assert gsb.gsb_batch_get(b, 1, gsb.GSB_BATCH_N) == 30
        assert gsb.gsb_batch_get(b, -1, gsb.GSB_BATCH_COUNT) == 2
        assert gsb.gsb_batch_get(b, -1, gsb.GSB_BATCH_REPLICAS) == 16
        assert gsb.gsb_batch_workspace_size(b) > 0
        with pytest.raises(gsb.GsbError) as e:
            gsb.gsb_batch_get(b, 0, gsb.GSB_BATCH_C)
        assert e.value.status == gsb.GSB_ESTATE
        J = instances.dense_pm1(12, 1)
        bad = J.copy()
        bad[0, 1] = -bad[0, 1]
        for M, status in ((bad, gsb.GSB_ENOTSYM), (J + np.eye(12, dtype=np.float32), gsb.GSB_EDIAG),
                          (0.5 * J, gsb.GSB_EUNSUPPORTED)):
            with pytest.raises(gsb.GsbError) as e:
                gsb.gsb_batch_set_coupling(b, 0, M)
            assert e.value.status == status
        with pytest.raises(ValueError):
            gsb.gsb_batch_set_coupling(b, 0, J[:, :5])
        with pytest.raises(gsb.GsbError):
            gsb.gsb_batch_set_coupling(b, 2, J)
        with pytest.raises(gsb.GsbError):
            gsb.gsb_batch_set(b, 0, gsb.GSB_BATCH_TILE_ROWS, 96)
        gsb.gsb_batch_set(b, 0, gsb.GSB_BATCH_TILE_ROWS, 128)
        for bad in (float("nan"), float("inf"), -float("inf"), 1e300, 64.5):
            with pytest.raises(gsb.GsbError):
                gsb.gsb_batch_set(b, 0, gsb.GSB_BATCH_TILE_ROWS, bad)
            with pytest.raises(gsb.GsbError):
                gsb.gsb_batch_set(b, -1, gsb.GSB_BATCH_GRAPH, bad)
            with pytest.raises(gsb.GsbError):
                gsb.gsb_batch_set(b, -1, gsb.GSB_BATCH_INIT_MODE, bad)
        with pytest.raises(gsb.GsbError):
            gsb.gsb_batch_set(b, 0, gsb.GSB_BATCH_GRAPH, 1)  # batch-wide: k must be -1
        gsb.gsb_batch_set(b, -1, gsb.GSB_BATCH_GRAPH, 1)
        assert gsb.gsb_batch_get(b, -1, gsb.GSB_BATCH_GRAPH) == 1
        with pytest.raises(gsb.GsbError) as e:
            gsb.gsb_batch_run(b, gsb.GSB_GBSB, 0.2, 10, 1)
        assert e.value.status in (gsb.GSB_ESTATE, gsb.GSB_EDEVICE)
    finally:
        gsb.gsb_batch_destroy(b)


@pytest.mark.parametrize("n,p", [(300, 0.03), (500, 0.01)])
def test_sparse_eigenvalue_estimate(n, p):
    """The compressed-row Lanczos path (a quarter or fewer nonzeros) against numpy."""
    J = instances.erdos_renyi_pm1(n, p, 5)
    ctx = gsb.gsb_create(J)
    try:
        lam = np.linalg.eigvalsh(J.astype(np.float64))
        assert abs(gsb.gsb_get(ctx, gsb.GSB_OPT_LAMBDA_MAX) - lam[-1]) < 1e-8 * abs(lam[-1])
        assert abs(gsb.gsb_get(ctx, gsb.GSB_OPT_LAMBDA_MIN) - lam[0]) < 1e-8 * abs(lam[0])
        dt = 1.25 * np.sqrt(2.0 / (1.0 - lam[0] / lam[-1]))
        assert abs(gsb.gsb_get(ctx, gsb.GSB_OPT_DT_STABLE) - dt) < 1e-8
    finally:
        gsb.gsb_destroy(ctx)


def test_batch_workload_recipe():
    specs = instances.batch_workload(256, 7)
    assert len(specs) == 256
    ns = np.array([s[1] for s in specs])
    assert ns.min() >= 64 and ns.max() <= 4096
    assert 1800 < ns.mean() < 2350  # uniform on [64, 4096]: mean 2080
    kinds = [s[0] for s in specs]
    assert kinds.count("dense") == 128
    ps = np.array([s[2] for s in specs if s[0] == "sparse"])
    assert ps.min() >= 0.01 and ps.max() <= 0.06
    assert instances.batch_workload(256, 7) == specs
    J = instances.make_instance(("sparse", 200, 0.05, 3))
    assert np.array_equal(J, instances.erdos_renyi_pm1(200, 0.05, 3))
