"""GPU parity of the 16-bit fixed-point product (FIX16: int8 hi/lo MFMA, exact int32
accumulation) against the oracle's FIX16 operand form, bit for bit."""
import sys

import numpy as np
import pytest

from paper_2508_17655_amd import instances

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _check_exact(a, b, what):
    a = np.asarray(a)
    b = np.asarray(b).astype(a.dtype)
    bad = np.flatnonzero(a.ravel() != b.ravel())
    assert bad.size == 0, f"{what}: {bad.size} mismatches, first at {bad[0]}: {a.ravel()[bad[0]]} vs {b.ravel()[bad[0]]}"


@pytest.mark.parametrize("variant", ["gbsb", "bsb", "gdsb", "dsb"])
def test_fix16_small_ragged_bitexact(orc, variant):
    from paper_2508_17655_amd import gsb
    n, R, M, A, seed = 333, 40, 150, 0.25, 17
    say(f"case fix16 small variant={variant} n={n} R={R} M={M}")
    J = instances.dense_pm1(n, 13)
    c = instances.paper_c(n)
    g = gsb.GSB(J, precision="fix16", c=c)
    g.run(variant, A=A, dt=1.25, replicas=R, steps=M, seed=seed)
    x, y, p, m = g.state()
    E = g.energy()
    g.close()
    x0, y0 = orc.init_state(n, R, seed, orc.INIT_X)
    xo, yo, po = orc.run(J.astype(np.float64), orc.VARIANTS[variant], A=A, dt=1.25, c=c, steps=M, x=x0, y=y0,
                         form=orc.FORM_FIX16, mode="fp32")
    _check_exact(x, xo, "x")
    _check_exact(y, yo, "y")
    _check_exact(p, po, "p")
    s = orc.spins(xo)
    _check_exact(E, orc.energy(J.astype(np.float64), s), "energies")


def test_fix16_full_size_sampled_bitexact(orc):
    from paper_2508_17655_amd import gsb
    n, R, M, A, seed = 2000, 1024, 2000, 0.2, 77
    say(f"case fix16 full-size n={n} R={R} M={M}")
    J = instances.dense_pm1(n, 2)
    c = instances.paper_c(n)
    g = gsb.GSB(J, precision="fix16", c=c)
    g.run("gbsb", A=A, dt=1.25, replicas=R, steps=M, seed=seed)
    x, y, p, _ = g.state()
    g.close()
    sample = np.array([0, 333, 1023])
    x0, y0 = orc.init_state(n, R, seed, orc.INIT_X)
    xo, yo, po = orc.run(J.astype(np.float64), orc.GBSB, A=A, dt=1.25, c=c, steps=M, x=x0[sample], y=y0[sample],
                         form=orc.FORM_FIX16, mode="fp32")
    _check_exact(x[sample], xo, "x")
    _check_exact(y[sample], yo, "y")
    _check_exact(p[sample], po, "p")


def test_fix16_requires_pm1_coupling():
    from paper_2508_17655_amd import gsb
    J = instances.dense_gaussian(32, 3)
    g = gsb.GSB(J)
    with pytest.raises(gsb.GsbError):
        gsb.gsb_set(g.ctx, gsb.GSB_OPT_PRECISION, gsb.GSB_PREC_FIX16)
    g.close()
