"""GPU path (libgsb through its C ABI) against the CPU oracle, element by element.

Bars (derived in the design notes):
  - sign products (dSB, GdSB) in every precision and the E4M3 product of bSB/GbSB in the
    FP8 form: bit-exact x, y, p, spins and energies against the oracle's strict binary32
    mode, because every partial sum of those products is exactly representable;
  - continuous products in the FP32 and BF16X2 forms: one step from an identical state
    within 1e-5 (relative, L2 over a replica) of the binary64 step; over 100 steps no
    further from the binary64 trajectory than the strict binary32 oracle is, times 4,
    floored at 1e-5.
"""
import sys

import numpy as np
import pytest

from paper_2508_17655_amd import gsb, instances

pytestmark = pytest.mark.gpu

FORM_OF = {"fp8": 1, "fp32": 0, "bf16x2": 2}  # oracle operand form of a continuous product


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def make(J, precision, c, init_mode=gsb.GSB_INIT_X):
    return gsb.GSB(J, precision=precision, c=c, init_mode=init_mode)


def oracle_start(orc, n, R, seed, init_mode):
    x, y = orc.init_state(n, R, seed, init_mode)
    return x, y, np.ones_like(x)


def check_exact(a, b, what):
    if not np.array_equal(a, b):
        bad = np.argwhere(a != b)
        raise AssertionError(f"{what}: {len(bad)} elements differ, first at {bad[0].tolist()}: "
                             f"{a[tuple(bad[0])]!r} vs {b[tuple(bad[0])]!r}")


@pytest.mark.parametrize("variant", ["dsb", "gdsb", "gbsb", "bsb"])
def test_small_exact_forms_bitexact(orc, variant):
    # N = 200, 16 replicas, 1000 steps, dt = 0.5, x and y ~ U(-0.1, 0.1): the small workload.
    n, R, M, dt, A, seed = 200, 16, 1000, 0.5, 0.2, 11
    say(f"case small-exact variant={variant} n={n} R={R} M={M}")
    J = instances.dense_pm1(n, 1)
    c = instances.paper_c(n)
    g = make(J, "fp8", c, gsb.GSB_INIT_XY)
    g.run(variant, A=A, dt=dt, replicas=R, steps=M, seed=seed)
    x, y, p, m = g.state()
    E = g.energy()
    s_best, e_best, r_best = g.best()
    spins = g.spins()
    g.close()
    assert m == M
    x0, y0, p0 = oracle_start(orc, n, R, seed, orc.INIT_XY)
    v = orc.VARIANTS[variant]
    form = orc.FORM_E4M3 if variant in ("bsb", "gbsb") else orc.FORM_EXACT
    xo, yo, po = orc.run(J, v, A=A, dt=dt, c=c, steps=M, x=x0, y=y0, p=p0, form=form, mode="fp32")
    check_exact(x, xo, "x"); check_exact(y, yo, "y"); check_exact(p, po, "p")
    so = orc.spins(xo)
    check_exact(spins, so, "spins")
    Eo = orc.energy(J, so)
    check_exact(E, Eo, "energies")
    assert r_best == orc.best(Eo) and e_best == Eo.min()
    check_exact(s_best, so[r_best], "best spins")


@pytest.mark.parametrize("precision", ["fp8", "bf16x2", "fp32"])
@pytest.mark.parametrize("variant", ["dsb", "gdsb"])
def test_ragged_sign_products_bitexact(orc, precision, variant):
    # n not a multiple of the 128-spin k-step and R not a multiple of the 128-replica
    # group: padding rows and padded replicas must not leak into the result.
    n, R, M, seed = 333, 200, 300, 5
    say(f"case ragged-sign precision={precision} variant={variant} n={n} R={R}")
    J = instances.dense_pm1(n, 2)
    c = instances.paper_c(n)
    g = make(J, precision, c)
    g.run(variant, A=0.3, dt=1.25, replicas=R, steps=M, seed=seed)
    x, y, p, _ = g.state()
    E = g.energy()
    g.close()
    x0, y0, p0 = oracle_start(orc, n, R, seed, orc.INIT_X)
    xo, yo, po = orc.run(J, orc.VARIANTS[variant], A=0.3, dt=1.25, c=c, steps=M, x=x0, y=y0, p=p0, mode="fp32")
    check_exact(x, xo, "x"); check_exact(y, yo, "y"); check_exact(p, po, "p")
    check_exact(E, orc.energy(J, orc.spins(xo)), "energies")


def test_chained_launches_equal_one_launch(orc):
    # M steps in one persistent launch == the same steps in several launches (the state,
    # operand and barrier hand-over between launches is exact) == oracle.
    n, R, M, seed = 256, 256, 240, 3
    say(f"case chained n={n} R={R} M={M}")
    J = instances.dense_pm1(n, 4)
    c = instances.paper_c(n)
    g = make(J, "fp8", c)
    g.init("gdsb", A=0.25, dt=1.25, replicas=R, steps=M, seed=seed)
    g.step(M)
    a = g.state()
    g.init("gdsb", A=0.25, dt=1.25, replicas=R, steps=M, seed=seed)
    for k in (1, 7, 32, 100, 100):
        g.step(k)
    b = g.state()
    # resume from a checkpoint taken at step 120
    g.init("gdsb", A=0.25, dt=1.25, replicas=R, steps=M, seed=seed)
    g.step(120)
    ck = g.state()
    g.init("gdsb", A=0.25, dt=1.25, replicas=R, steps=M, seed=seed + 1)
    g.set_state(ck[0], ck[1], ck[2], ck[3])
    g.step(M - 120)
    c2 = g.state()
    g.close()
    for u, v, w in zip(a[:3], b[:3], c2[:3]):
        check_exact(u, v, "chained")
        check_exact(u, w, "resumed")
    x0, y0, p0 = oracle_start(orc, n, R, seed, orc.INIT_X)
    xo = orc.run(J, orc.GDSB, A=0.25, dt=1.25, c=c, steps=M, x=x0, y=y0, p=p0, mode="fp32")[0]
    check_exact(a[0], xo, "x vs oracle")


def test_determinism(orc):
    n, R, M = 500, 384, 200
    say(f"case determinism n={n} R={R}")
    J = instances.dense_pm1(n, 6)
    g = make(J, "fp8", instances.paper_c(n))
    out = []
    for _ in range(2):
        g.run("gbsb", A=0.2, dt=1.25, replicas=R, steps=M, seed=77)
        out.append(g.state()[:3])
    g.close()
    for u, v in zip(*out):
        assert u.tobytes() == v.tobytes()


@pytest.mark.parametrize("variant", ["gdsb", "gbsb"])
def test_full_size_sampled_bitexact(orc, variant):
    # The benchmark launch: N = 2000 dense +-1, 1024 replicas, 2000 steps, dt = 1.25,
    # FP8 product.  Replicas are independent, so a sample of them is checked against the
    # oracle over the whole run, and all of them for the energy/spin consistency.
    n, R, M, A, seed = 2000, 1024, 2000, 0.2, 2024
    say(f"case full-size variant={variant} n={n} R={R} M={M}")
    J = instances.dense_pm1(n, 2)
    c = instances.paper_c(n)
    g = make(J, "fp8", c)
    g.run(variant, A=A, dt=1.25, replicas=R, steps=M, seed=seed)
    x, y, p, _ = g.state()
    E = g.energy()
    spins = g.spins()
    g.close()
    sample = np.array([0, 1, 517, 1023])
    x0, y0, p0 = oracle_start(orc, n, R, seed, orc.INIT_X)
    form = orc.FORM_E4M3 if variant == "gbsb" else orc.FORM_EXACT
    xo, yo, po = orc.run(J, orc.VARIANTS[variant], A=A, dt=1.25, c=c, steps=M, x=x0[sample], y=y0[sample],
                         p=p0[sample], form=form, mode="fp32")
    check_exact(x[sample], xo, "x"); check_exact(y[sample], yo, "y"); check_exact(p[sample], po, "p")
    # every replica: energies are those of its spins
    check_exact(spins, orc.spins(x), "spins")
    check_exact(E, orc.energy(J, spins), "energies")


@pytest.mark.parametrize("variant", ["dsb", "gdsb"])
def test_ferromagnet_largest_sign_products_bitexact(orc, variant):
    """The largest products the sign kernels hand over: a ferromagnet (J_ij = +1 for all
    i != j) at n = 2048, one full tile of 16 k-steps, where the spins align within a few
    steps and |sum_j J_ij s_j| = n - 1 = 2047 (the f16 hand-over holds it exactly)."""
    n, R, M, A, seed = 2048, 128, 60, 0.2, 77
    say(f"case ferromagnet variant={variant} n={n} R={R} M={M}")
    J = np.ones((n, n), dtype=np.float32) - np.eye(n, dtype=np.float32)
    c = instances.paper_c(n)
    g = make(J, "fp8", c)
    g.run(variant, A=A, dt=1.25, replicas=R, steps=M, seed=seed)
    x, y, p, _ = g.state()
    E = g.energy()
    g.close()
    sample = np.array([0, 77, 127])
    x0, y0, p0 = oracle_start(orc, n, R, seed, orc.INIT_X)
    xo, yo, po = orc.run(J, orc.VARIANTS[variant], A=A, dt=1.25, c=c, steps=M, x=x0[sample], y=y0[sample],
                         p=p0[sample], form=orc.FORM_EXACT, mode="fp32")
    check_exact(x[sample], xo, "x"); check_exact(y[sample], yo, "y"); check_exact(p[sample], po, "p")
    s = orc.spins(x)
    aligned = np.all(s == s[:, :1], axis=1)
    assert aligned.mean() > 0.9, "the case needs aligned replicas (products of magnitude n - 1)"
    check_exact(E, orc.energy(J, s), "energies")
    assert np.all(E[aligned] == -0.5 * n * (n - 1))


@pytest.mark.parametrize("variant", ["gbsb", "gdsb"])
def test_fp8_generic_kernel_bitexact(orc, variant):
    # N_p > 2048: the FP8 product runs in the generic kernel (FP4 J from L2), 2 k-step
    # rounds of the software pipeline and a ragged tail of 472 padded spins.
    n, R, M, A, seed = 2600, 128, 40, 0.25, 31
    say(f"case fp8 generic variant={variant} n={n} R={R} M={M}")
    J = instances.dense_pm1(n, 12)
    c = instances.paper_c(n)
    g = make(J, "fp8", c)
    g.run(variant, A=A, dt=1.25, replicas=R, steps=M, seed=seed)
    x, y, p, _ = g.state()
    E = g.energy()
    g.close()
    sample = np.array([0, 63, 127])
    x0, y0, p0 = oracle_start(orc, n, R, seed, orc.INIT_X)
    form = orc.FORM_E4M3 if variant == "gbsb" else orc.FORM_EXACT
    xo, yo, po = orc.run(J, orc.VARIANTS[variant], A=A, dt=1.25, c=c, steps=M, x=x0[sample], y=y0[sample],
                         p=p0[sample], form=form, mode="fp32")
    check_exact(x[sample], xo, "x"); check_exact(y[sample], yo, "y"); check_exact(p[sample], po, "p")
    check_exact(E, orc.energy(J, orc.spins(x)), "energies")


@pytest.mark.parametrize("n", [333, 1000, 1500, 2000])
def test_both_fp8_step_kernels_bitexact(orc, n):
    # The two FP8 step kernels for n_p <= 2048 (1: product and update in one wave per SIMD;
    # 2: in two waves per SIMD, J partly in LDS from n_p = 1536 on) give the same bits,
    # and the oracle's.
    R, M, A, seed = 200, 120, 0.2, 5  # 8 replica groups: each on one XCD
    say(f"case step kernels n={n} R={R} M={M}")
    J = instances.dense_pm1(n, 21)
    c = instances.paper_c(n)
    for variant in ("gbsb", "gdsb"):
        got = {}
        for k in (1, 2):
            g = gsb.GSB(J, precision="fp8", c=c, step_kernel=k)
            assert gsb.gsb_get(g.ctx, gsb.GSB_OPT_STEP_KERNEL) == k
            g.run(variant, A=A, dt=1.25, replicas=R, steps=M, seed=seed)
            got[k] = g.state()[:3] + (g.energy(),)
            g.close()
        for a, b, what in zip(got[1], got[2], ("x", "y", "p", "E")):
            check_exact(a, b, f"kernel 1 vs 2, {variant} {what}")
        sample = np.array([0, 47, 95, 150, 199])
        x0, y0, p0 = oracle_start(orc, n, R, seed, orc.INIT_X)
        form = orc.FORM_E4M3 if variant == "gbsb" else orc.FORM_EXACT
        xo, yo, po = orc.run(J, orc.VARIANTS[variant], A=A, dt=1.25, c=c, steps=M, x=x0[sample], y=y0[sample],
                             p=p0[sample], form=form, mode="fp32")
        x, y, p, _ = got[2]
        check_exact(x[sample], xo, "x"); check_exact(y[sample], yo, "y"); check_exact(p[sample], po, "p")


@pytest.mark.parametrize("case", range(12))
def test_fp8_kernels_on_seeded_random_shapes(orc, case):
    # n, replicas, steps and variant drawn from a seeded generator: padded rows, padded
    # replicas, one to several replica groups (padded grid or not), J partly in LDS or
    # not, launches of one step.  Both FP8 step kernels, bit for bit with each other and
    # with the oracle on sampled replicas.
    rng = np.random.default_rng(1000 + case)
    n = int(rng.integers(100, 2049))
    R = int(rng.integers(1, 301))
    M = int(rng.integers(1, 81))
    variant = ["bsb", "dsb", "gbsb", "gdsb"][int(rng.integers(0, 4))]
    A = float(rng.uniform(0.0, 0.5))
    say(f"case random shapes #{case}: n={n} R={R} M={M} {variant} A={A:.3f}")
    J = instances.dense_pm1(n, 50 + case)
    c = instances.paper_c(n)
    got = {}
    for k in (1, 2):
        g = gsb.GSB(J, precision="fp8", c=c, step_kernel=k)
        g.run(variant, A=A, dt=1.25, replicas=R, steps=M, seed=case)
        got[k] = g.state()[:3]
        g.close()
    for a, b, what in zip(got[1], got[2], ("x", "y", "p")):
        check_exact(a, b, f"kernel 1 vs 2 {what}")
    sample = np.unique(np.array([0, R // 2, R - 1]))
    x0, y0, p0 = oracle_start(orc, n, R, case, orc.INIT_X)
    form = orc.FORM_E4M3 if variant in ("bsb", "gbsb") else orc.FORM_EXACT
    xo, yo, po = orc.run(J, orc.VARIANTS[variant], A=A, dt=1.25, c=c, steps=M, x=x0[sample], y=y0[sample],
                         p=p0[sample], form=form, mode="fp32")
    x, y, p = got[2]
    check_exact(x[sample], xo, "x"); check_exact(y[sample], yo, "y"); check_exact(p[sample], po, "p")


def test_chained_launches_on_full_size_operand(orc):
    # The wave-specialised kernel's operand buffers keep their contents across launches
    # and runs of a context; every launch restarts the step tags of its operand words.
    # At n = 2000 (16 k-steps: first fragments checked together, later ones one by one),
    # runs of one launch and of launches of 1 to 7 steps, repeated on one context, give
    # the register-J kernel's bits.
    n, R, M, seed = 2000, 128, 40, 12
    say(f"case chained full size n={n} R={R} M={M}")
    J = instances.dense_pm1(n, 8)
    c = instances.paper_c(n)
    g2 = gsb.GSB(J, precision="fp8", c=c, step_kernel=2)
    g1 = gsb.GSB(J, precision="fp8", c=c, step_kernel=1)
    g1.run("gbsb", A=0.2, dt=1.25, replicas=R, steps=M, seed=seed)
    ref = g1.state()[:3]
    g1.close()
    for pieces in ((M,), (1, 2, 3, 4, 5, 6, 7, 12), (7, 7, 7, 7, 7, 5), (M,)):
        g2.init("gbsb", A=0.2, dt=1.25, replicas=R, steps=M, seed=seed)
        for k in pieces:
            g2.step(k)
        for a, b, what in zip(g2.state()[:3], ref, ("x", "y", "p")):
            check_exact(a, b, f"pieces {pieces}: {what}")
    g2.close()


@pytest.mark.parametrize("n,R,variant", [(1500, 300, "gbsb"), (2000, 100, "dsb"), (700, 380, "gdsb")])
def test_fp8_kernels_with_groups_across_xcds(orc, n, R, variant):
    # Without grid padding, 4 or 12 replica groups put the row blocks of a group on
    # different XCDs (workgroups go to the XCDs in turn), so the kernels take their
    # cross-XCD exchange: a group counter with device-scope fences every step.  Both FP8
    # step kernels, bit for bit with each other, with the padded grid and with the oracle.
    M, A, seed = 60, 0.2, 9
    say(f"case groups across XCDs n={n} R={R} M={M} {variant}")
    J = instances.dense_pm1(n, 31)
    c = instances.paper_c(n)
    got = {}
    for k, pad in ((1, False), (2, False), (2, True)):
        g = gsb.GSB(J, precision="fp8", c=c, step_kernel=k, grid_pad=pad)
        assert gsb.gsb_get(g.ctx, gsb.GSB_OPT_GRID_PAD) == (1 if pad else 0)
        g.run(variant, A=A, dt=1.25, replicas=R, steps=M, seed=seed)
        got[k, pad] = g.state()[:3]
        g.close()
    for key in ((1, False), (2, True)):
        for a, b, what in zip(got[key], got[2, False], ("x", "y", "p")):
            check_exact(a, b, f"{key} vs unpadded kernel 2, {what}")
    sample = np.unique(np.array([0, 5, R // 2, R - 1]))
    x0, y0, p0 = oracle_start(orc, n, R, seed, orc.INIT_X)
    form = orc.FORM_E4M3 if variant in ("bsb", "gbsb") else orc.FORM_EXACT
    xo, yo, po = orc.run(J, orc.VARIANTS[variant], A=A, dt=1.25, c=c, steps=M, x=x0[sample], y=y0[sample],
                         p=p0[sample], form=form, mode="fp32")
    x, y, p = got[2, False]
    check_exact(x[sample], xo, "x"); check_exact(y[sample], yo, "y"); check_exact(p[sample], po, "p")


@pytest.mark.parametrize("precision,kernel,variant,form", [("fp8", 1, "gbsb", "e4m3"), ("fp8", 2, "gbsb", "e4m3"),
                                                            ("fix16", 0, "gbsb", "fix16"), ("fp32", 0, "gdsb", "exact")])
def test_small_launch_on_padded_grid(orc, precision, kernel, variant, form):
    # 40 replicas are one or a few replica groups; the grid is padded to whole rounds of 8
    # groups (padding workgroups exit at once) so that each group shares one XCD.
    n, R, M, A, seed = 700, 40, 150, 0.2, 8
    say(f"case padded grid precision={precision} kernel={kernel} n={n} R={R} M={M}")
    J = instances.dense_pm1(n, 6)
    c = instances.paper_c(n)
    g = gsb.GSB(J, precision=precision, c=c, step_kernel=kernel)
    g.run(variant, A=A, dt=1.25, replicas=R, steps=M, seed=seed)
    x, y, p, _ = g.state()
    E = g.energy()
    g.close()
    sample = np.array([0, 17, 39])
    x0, y0, p0 = oracle_start(orc, n, R, seed, orc.INIT_X)
    f = {"e4m3": orc.FORM_E4M3, "fix16": orc.FORM_FIX16, "exact": orc.FORM_EXACT}[form]
    xo, yo, po = orc.run(J, orc.VARIANTS[variant], A=A, dt=1.25, c=c, steps=M, x=x0[sample], y=y0[sample],
                         p=p0[sample], form=f, mode="fp32")
    check_exact(x[sample], xo, "x"); check_exact(y[sample], yo, "y"); check_exact(p[sample], po, "p")
    check_exact(E, orc.energy(J, orc.spins(x)), "energies")


@pytest.mark.parametrize("kernel", [1, 2])
def test_operand_small_enough_for_l1(orc, kernel):
    # Regression: with XCD-local replica groups and an operand that fits in L1 (n_p = 512),
    # a workgroup-scope L1 invalidate let stale operand lines through now and then (whole
    # 16-replica tiles diverged, differently from run to run).  Every replica, 300 steps.
    n, R, M, seed = 333, 200, 300, 5
    say(f"case operand in L1 kernel={kernel} n={n} R={R} M={M}")
    J = instances.dense_pm1(n, 2)
    c = instances.paper_c(n)
    x0, y0, p0 = oracle_start(orc, n, R, seed, orc.INIT_X)
    xo, yo, po = orc.run(J, orc.DSB, A=0.3, dt=1.25, c=c, steps=M, x=x0, y=y0, p=p0, mode="fp32")
    for rep in range(3):
        g = gsb.GSB(J, precision="fp8", c=c, step_kernel=kernel)
        g.run("dsb", A=0.3, dt=1.25, replicas=R, steps=M, seed=seed)
        x, y, p, _ = g.state()
        g.close()
        check_exact(x, xo, f"x (run {rep})"); check_exact(y, yo, f"y (run {rep})"); check_exact(p, po, f"p (run {rep})")


@pytest.mark.parametrize("precision,variant,form", [("fp8", "gbsb", "e4m3"), ("fix16", "gbsb", "fix16"),
                                                     ("bf16x2", "gdsb", "exact"), ("fp32", "dsb", "exact")])
def test_more_replicas_than_one_launch_holds(orc, precision, variant, form):
    # At N = 2000 one co-resident launch holds 1024 replicas; 1100 replicas run as a
    # launch of 1024 and one of 128 (76 of them padding).  Replicas on both sides of the
    # split, and the last one, against the oracle.
    n, R, M, A, seed = 2000, 1100, 40, 0.2, 77
    say(f"case two launches precision={precision} variant={variant} n={n} R={R} M={M}")
    J = instances.dense_pm1(n, 2)
    c = instances.paper_c(n)
    g = make(J, precision, c)
    g.run(variant, A=A, dt=1.25, replicas=R, steps=M, seed=seed)
    x, y, p, _ = g.state()
    E = g.energy()
    g.close()
    assert x.shape == (R, n)
    sample = np.array([0, 1023, 1024, 1077, R - 1])
    x0, y0, p0 = oracle_start(orc, n, R, seed, orc.INIT_X)
    f = {"e4m3": orc.FORM_E4M3, "fix16": orc.FORM_FIX16, "exact": orc.FORM_EXACT}[form]
    xo, yo, po = orc.run(J, orc.VARIANTS[variant], A=A, dt=1.25, c=c, steps=M, x=x0[sample], y=y0[sample],
                         p=p0[sample], form=f, mode="fp32")
    check_exact(x[sample], xo, "x"); check_exact(y[sample], yo, "y"); check_exact(p[sample], po, "p")
    check_exact(E, orc.energy(J, orc.spins(x)), "energies")


@pytest.mark.parametrize("precision", ["fp32", "bf16x2"])
def test_continuous_forms_error_bounds(orc, precision):
    # bSB with a continuous product: one step from an identical state, and 100 steps.
    n, R, M, seed = 2000, 128, 2000, 9
    say(f"case continuous precision={precision} n={n} R={R}")
    J = instances.dense_pm1(n, 2)
    c = instances.paper_c(n)
    g = make(J, precision, c)
    g.init("bsb", dt=1.25, replicas=R, steps=M, seed=seed)
    samp = np.arange(4)
    x0, y0, p0 = oracle_start(orc, n, R, seed, orc.INIT_X)
    kw = dict(dt=1.25, c=c, steps=M)
    # 40 steps in binary64 to get a state off the initial one, then one step on both sides
    xs, ys, ps = orc.run(J, orc.BSB, x=x0, y=y0, p=p0, m_end=40, mode="fp64", **kw)
    g.set_state(xs.astype(np.float32), ys.astype(np.float32), ps.astype(np.float32), 40)
    g.step(1)
    xg = g.state()[0][samp]
    x64 = orc.run(J, orc.BSB, x=xs[samp].astype(np.float32), y=ys[samp].astype(np.float32),
                  p=ps[samp].astype(np.float32), m_begin=40, m_end=41, mode="fp64", **kw)[0]
    rel1 = np.linalg.norm(xg - x64, axis=1) / np.linalg.norm(x64, axis=1)
    say(f"  one-step relative error {rel1.max():.3e}")
    assert rel1.max() <= 1e-5
    # trajectory over the first 100 steps
    g.init("bsb", dt=1.25, replicas=R, steps=M, seed=seed)
    traj = []
    for _ in range(100):
        g.step(1)
        traj.append(g.state()[0][samp])
    g.close()
    traj = np.stack(traj, axis=1)
    t64 = orc.run(J, orc.BSB, x=x0[samp], y=y0[samp], p=p0[samp], m_end=100, mode="fp64", record=True, **kw)[3]
    t32 = orc.run(J, orc.BSB, x=x0[samp], y=y0[samp], p=p0[samp], m_end=100, mode="fp32", record=True, **kw)[3]
    e_gpu = np.linalg.norm(traj - t64, axis=2) / np.linalg.norm(t64, axis=2)
    e_f32 = np.linalg.norm(t32 - t64, axis=2) / np.linalg.norm(t64, axis=2)
    say(f"  100-step error gpu {e_gpu.max():.3e} strict-fp32 {e_f32.max():.3e}; "
        f"first step where strict fp32 exceeds 1e-5: {int(np.argmax(e_f32.max(0) > 1e-5))}")
    assert np.all(e_gpu <= np.maximum(1e-5, 4 * e_f32))


def test_real_weighted_energy_fp64(orc):
    # J_ij ~ N(0,1)/sqrt(N) (not exact in FP8): BF16X2 product; the final energy is binary64.
    n, R, M, seed = 300, 128, 200, 4
    say(f"case real-weighted n={n}")
    J = instances.dense_gaussian(n, 3)
    g = gsb.GSB(J)  # default: BF16X2, c = 1/lambda_max (App. A)
    lmax = g.get(gsb.GSB_OPT_LAMBDA_MAX)
    assert abs(lmax - np.linalg.eigvalsh(J.astype(np.float64))[-1]) < 1e-8
    dt = g.get(gsb.GSB_OPT_DT_STABLE)
    g.run("gbsb", A=0.2, dt=dt, replicas=R, steps=M, seed=seed)
    spins = g.spins()
    E = g.energy()
    g.close()
    Eo = orc.energy(J, spins)
    np.testing.assert_allclose(E, Eo, rtol=1e-13, atol=1e-12)


def test_real_weighted_bf16_one_step_error(orc):
    # J_ij ~ N(0,1)/sqrt(N) in the BF16X2 form: J itself is rounded to bf16 (relative
    # error <= 2^-9 per coupling, random in sign), x is split hi/lo.  One step from an
    # identical state against the binary64 step with the exact J: the coupling increment
    # dy = y' - y (c dt J x, minus the small p x dt term) is off by about 2^-9 / sqrt(3)
    # relative; bound 4e-3.
    n, R, M, seed = 2000, 128, 2000, 6
    say(f"case real-weighted bf16 one step n={n}")
    J = instances.dense_gaussian(n, 3)
    g = gsb.GSB(J)  # default precision for real J: BF16X2
    c = g.get(gsb.GSB_OPT_C)
    dt = g.get(gsb.GSB_OPT_DT_STABLE)
    g.init("gbsb", A=0.2, dt=dt, replicas=R, steps=M, seed=seed)
    samp = np.arange(4)
    x0, y0, p0 = oracle_start(orc, n, R, seed, orc.INIT_X)
    kw = dict(A=0.2, dt=dt, c=c, steps=M)
    xs, ys, ps = orc.run(J, orc.GBSB, x=x0, y=y0, p=p0, m_end=40, mode="fp64", **kw)
    xs, ys, ps = (v.astype(np.float32) for v in (xs, ys, ps))
    g.set_state(xs, ys, ps, 40)
    g.step(1)
    yg = g.state()[1][samp]
    g.close()
    y64 = orc.run(J, orc.GBSB, x=xs[samp], y=ys[samp], p=ps[samp], m_begin=40, m_end=41, mode="fp64", **kw)[1]
    d64 = y64 - ys[samp]
    rel = np.linalg.norm((yg - ys[samp]) - d64, axis=1) / np.linalg.norm(d64, axis=1)
    say(f"  one-step relative error of dy: {rel.max():.3e}")
    assert rel.max() <= 4e-3


def test_real_weighted_bf16_end_of_run(orc):
    """A whole run of the real-weighted instance (J_ij ~ N(0,1)/sqrt(N)) in the BF16X2 form
    against binary64 runs from the same start: with the exact J and with the bf16-rounded J
    the device uses.  The dynamics are chaotic, so a replica may end in another local
    minimum than its binary64 twin; what is bounded is the energy error of eq. (1) with the
    exact couplings, per replica and of the best replica (measured: at most 4.3e-5, median 0,
    best replica equal; at N = 2000 over 2000 steps the bench measures at most 0.5%)."""
    n, R, M, A, seed = 500, 16, 1000, 0.2, 41
    say(f"case real-weighted bf16 end of run n={n} R={R} M={M}")
    J = instances.dense_gaussian(n, 5)
    g = gsb.GSB(J, precision="bf16x2")
    c = g.get(gsb.GSB_OPT_C)
    dt = g.get(gsb.GSB_OPT_DT_STABLE)
    g.run("gbsb", A=A, dt=dt, replicas=R, steps=M, seed=seed)
    E = g.energy()
    s = g.spins()
    g.close()
    J64 = J.astype(np.float64)
    np.testing.assert_allclose(E, orc.energy(J64, s), rtol=1e-12)  # eq. (1) of its spins, binary64
    x0, y0, p0 = oracle_start(orc, n, R, seed, orc.INIT_X)
    for name, Jref in (("exact J", J64), ("bf16 J", orc.bf16_round(J).astype(np.float64))):
        x = orc.run(Jref, orc.GBSB, A=A, dt=dt, c=c, steps=M, x=x0, y=y0, p=p0, mode="fp64")[0]
        E_ref = orc.energy(J64, orc.spins(x))
        rel = np.abs(E - E_ref) / np.abs(E_ref)
        say(f"  {name}: energy relative error max {rel.max():.2e} median {np.median(rel):.2e}, "
            f"best {abs(E.min() - E_ref.min()) / abs(E_ref.min()):.2e}")
        assert rel.max() <= 5e-4 and np.median(rel) <= 1e-4
        assert abs(E.min() - E_ref.min()) <= 1e-6 * abs(E_ref.min())


def test_field_ancilla_energy(orc):
    n, R, M = 40, 128, 300
    say(f"case field n={n}")
    J = instances.dense_pm1(n, 8)
    h = np.where(np.arange(n) % 3 == 0, 1.0, -1.0).astype(np.float32)
    g = gsb.GSB(J, h, c=instances.paper_c(n + 1), precision="fp8")
    g.run("gdsb", A=0.2, dt=1.25, replicas=R, steps=M, seed=1)
    s = g.spins()
    E = g.energy()
    sb, eb, rb = g.best()
    g.close()
    # E = -1/2 s^T J s - h^T s for the returned (gauge-fixed) spins
    ref = orc.energy(J, s) - s.astype(np.float64) @ h.astype(np.float64)
    check_exact(E, ref, "energy with field")
    assert eb == ref.min() and rb == int(np.argmin(ref))


@pytest.mark.parametrize("R", [1, 63, 1000])
def test_best_replica_with_many_ties(orc, R):
    """gsb_best's argmin (a per-thread scan, a wavefront shuffle butterfly, then the four
    waves) on a 12-spin instance, where most replicas reach the same few energies: the
    lowest energy and, among its replicas, the lowest index (numpy's first occurrence)."""
    n, M = 12, 200
    say(f"case best-ties n={n} R={R}")
    J = instances.dense_pm1(n, 31)
    g = gsb.GSB(J, c=instances.paper_c(n), precision="fp8")
    g.run("gdsb", A=0.2, dt=1.25, replicas=R, steps=M, seed=5)
    E = g.energy()
    s = g.spins()
    sb, eb, rb = g.best()
    g.close()
    check_exact(E, orc.energy(J, s), "energies of the tie case")
    assert eb == E.min() and rb == int(np.argmin(E))
    np.testing.assert_array_equal(sb, s[rb])
    if R == 1000:
        assert np.sum(E == E.min()) > 1, "the case needs ties at the minimum"
