"""gsb_run_noalloc (the allocation-free run) against gsb_run, through the C ABI: the same
bits of x and of the energies, on calls in a row that share the library's device array
(the second call smaller than the first; a context that calls again after another one)."""
import sys

import numpy as np
import pytest

from paper_2508_17655_amd import gsb, instances

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def reference(J, precision, c, variant, A, dt, R, M, seed):
    g = gsb.GSB(J, precision=precision, c=c)
    g.run(variant, A=A, dt=dt, replicas=R, steps=M, seed=seed)
    x = g.state()[0]
    E = g.energy()
    g.close()
    return x, E


def noalloc(g, variant, A, dt, R, M, seed):
    import torch

    n_dyn = int(g.get(gsb.GSB_OPT_N_DYN))
    x = torch.full((R, n_dyn), float("nan"), dtype=torch.float32, device="cuda")
    E = torch.full((R,), float("nan"), dtype=torch.float64, device="cuda")
    gsb.gsb_set_stream(g.ctx, torch.cuda.current_stream().cuda_stream)
    gsb.gsb_run_noalloc(g.ctx, gsb.VARIANTS[variant], gsb.GSB_SCHED_LINEAR, A, dt, R, M, seed, x.data_ptr(),
                        E.data_ptr())
    return x.cpu().numpy(), E.cpu().numpy()


def check_same(a, b, what):
    if not np.array_equal(a, b):
        bad = np.argwhere(a != b)
        raise AssertionError(f"{what}: {len(bad)} elements differ, first at {bad[0].tolist()}")


def test_noalloc_equals_run_twice_then_smaller():
    # call 1: the benchmark shape (n = 2000 dense +-1, 1024 replicas) with the FP8 sign product
    n1, R1, M1 = 2000, 1024, 300
    say(f"case noalloc call 1 n={n1} R={R1} M={M1} gdsb fp8")
    J1 = instances.dense_pm1(n1, 2)
    c1 = instances.paper_c(n1)
    g1 = gsb.GSB(J1, precision="fp8", c=c1)
    x, E = noalloc(g1, "gdsb", 0.2, 1.25, R1, M1, 11)
    xr, Er = reference(J1, "fp8", c1, "gdsb", 0.2, 1.25, R1, M1, 11)
    check_same(x, xr, "x (call 1)")
    check_same(E, Er, "energies (call 1)")
    # call 2: smaller and ragged, another context (its J replaces the first one's in the array)
    n2, R2, M2 = 333, 200, 120
    say(f"case noalloc call 2 n={n2} R={R2} M={M2} gbsb fp8")
    J2 = instances.dense_pm1(n2, 9)
    c2 = instances.paper_c(n2)
    g2 = gsb.GSB(J2, precision="fp8", c=c2)
    x, E = noalloc(g2, "gbsb", 0.3, 1.25, R2, M2, 12)
    xr, Er = reference(J2, "fp8", c2, "gbsb", 0.3, 1.25, R2, M2, 12)
    check_same(x, xr, "x (call 2)")
    check_same(E, Er, "energies (call 2)")
    # call 3: the first context again, smaller (its J is uploaded again: another context ran since)
    say("case noalloc call 3 n=2000 R=128 M=200 gbsb fp8")
    x, E = noalloc(g1, "gbsb", 0.2, 1.25, 128, 200, 13)
    xr, Er = reference(J1, "fp8", c1, "gbsb", 0.2, 1.25, 128, 200, 13)
    check_same(x, xr, "x (call 3)")
    check_same(E, Er, "energies (call 3)")
    # call 4: the same context right after (its J is still in the array)
    say("case noalloc call 4 n=2000 R=64 M=100 dsb fp8")
    x, E = noalloc(g1, "dsb", 0.0, 1.25, 64, 100, 14)
    xr, Er = reference(J1, "fp8", c1, "dsb", 0.0, 1.25, 64, 100, 14)
    check_same(x, xr, "x (call 4)")
    check_same(E, Er, "energies (call 4)")
    g1.close()
    g2.close()


def test_noalloc_other_precision_and_field():
    # binary32 product with a field (ancilla spin): n_dyn = n + 1 columns of x
    n, R, M = 300, 100, 80
    say(f"case noalloc fp32 field n={n} R={R} M={M}")
    J = instances.dense_gaussian(n, 4)
    h = np.linspace(-0.5, 0.5, n).astype(np.float32)
    g = gsb.GSB(J, h, precision="fp32")
    x, E = noalloc(g, "gbsb", 0.2, 0.9, R, M, 21)
    g.close()
    gr = gsb.GSB(J, h, precision="fp32")
    gr.run("gbsb", A=0.2, dt=0.9, replicas=R, steps=M, seed=21)
    xr = gr.state()[0]
    Er = gr.energy()
    gr.close()
    assert x.shape == xr.shape == (R, n + 1)
    check_same(x, xr, "x (fp32, field)")
    check_same(E, Er, "energies (fp32, field)")


def test_noalloc_rejects_runs_beyond_the_array():
    import torch

    J = instances.dense_pm1(4000, 3)
    g = gsb.GSB(J, precision="fp8", c=instances.paper_c(4000))
    x = torch.empty((1024, 4000), dtype=torch.float32, device="cuda")
    E = torch.empty(1024, dtype=torch.float64, device="cuda")
    with pytest.raises(gsb.GsbError) as err:
        gsb.gsb_run_noalloc(g.ctx, gsb.GSB_GDSB, gsb.GSB_SCHED_LINEAR, 0.2, 1.25, 1024, 100, 1, x.data_ptr(),
                            E.data_ptr())
    assert err.value.status == gsb.GSB_EINVAL and "allocation-free" in str(err.value)
    # nothing was started: the context has no current run, and a normal run still works
    with pytest.raises(gsb.GsbError):
        gsb.gsb_energy(g.ctx)
    g.close()
