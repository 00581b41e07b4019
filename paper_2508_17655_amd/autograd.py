"""torch.autograd access to the binary32 dynamics (bSB, GbSB) of libgsb.

``Segment`` advances a run by ``count`` steps from a given state; its backward is the
library's reverse pass (gsb_vjp), which recomputes the segment's forward on the device
from the segment's start.  ``trajectory`` chains segments, so autograd keeps only the
segment boundaries: checkpointed recomputation over long trajectories.  Marshalling
only: the forward and reverse steps run in the library's kernels.
"""
from __future__ import annotations

import numpy as np
import torch

from . import gsb as _gsb


class Segment(torch.autograd.Function):
    """(x, y, p) at step m -> (x, y, p) at step m + count of the run held by `g` (a
    ``gsb.GSB`` initialised with gsb_init in the FP32 precision).  Tensors are
    [replicas, n_dyn] binary32.  On the GPU the state and the cotangents stay in device
    memory (gsb_set_state_device, gsb_state_device, gsb_vjp_device on torch's current
    stream); tensors on the host go through the host forms of the same calls."""

    @staticmethod
    def forward(ctx, x, y, p, g, m, count):
        ctx.g, ctx.m, ctx.count = g, m, count
        ctx.save_for_backward(x, y, p)
        if x.is_cuda:
            xs, ys, ps = (t.detach().to(torch.float32).contiguous() for t in (x, y, p))
            g.set_state_device(xs, ys, ps, m)
            g.step(count)
            out = tuple(torch.empty_like(xs) for _ in range(3))
            g.state_device(*out)
            return out
        xs, ys, ps = (t.detach().to("cpu", torch.float32).contiguous().numpy() for t in (x, y, p))
        g.set_state(xs, ys, ps, m)
        g.step(count)
        xo, yo, po, _ = g.state()
        return tuple(torch.from_numpy(v) for v in (xo, yo, po))

    @staticmethod
    def backward(ctx, gx, gy, gp):
        x, y, p = ctx.saved_tensors
        g = ctx.g
        if x.is_cuda:
            g.set_state_device(*(t.detach().to(torch.float32).contiguous() for t in (x, y, p)), ctx.m)
            cot = [torch.zeros_like(ref, dtype=torch.float32) if t is None
                   else t.detach().to(torch.float32).contiguous().clone() for t, ref in ((gx, x), (gy, y), (gp, p))]
            g.vjp_device(ctx.count, *cot)
            return (*cot, None, None, None)
        xs, ys, ps = (t.detach().to("cpu", torch.float32).contiguous().numpy() for t in (x, y, p))
        g.set_state(xs, ys, ps, ctx.m)
        cot = []
        for t, ref in ((gx, x), (gy, y), (gp, p)):
            cot.append(np.zeros(ref.shape, dtype=np.float32) if t is None
                       else t.detach().to("cpu", torch.float32).contiguous().numpy())
        xb, yb, pb = g.vjp(ctx.count, *cot)
        return torch.from_numpy(xb), torch.from_numpy(yb), torch.from_numpy(pb), None, None, None


def trajectory(g, x, y, p, steps: int, every: int = 50):
    """Advance (x, y, p) from step 0 by `steps` steps in segments of `every` steps."""
    m = 0
    while m < steps:
        k = min(every, steps - m)
        x, y, p = Segment.apply(x, y, p, g, m, k)
        m += k
    return x, y, p


def start(J, variant: str = "gbsb", *, A: float, dt: float, replicas: int, steps: int, seed: int, c=None,
          schedule: int = _gsb.GSB_SCHED_LINEAR, device=None):
    """A ``gsb.GSB`` in the FP32 precision with an initialised run, and its starting state
    as float32 tensors (x, y, p), each [replicas, n_dyn]: on the host, or (device="cuda")
    in device memory, copied there by the library."""
    g = _gsb.GSB(J, precision="fp32", c=c)
    g.init(variant, A=A, dt=dt, replicas=replicas, steps=steps, seed=seed, schedule=schedule)
    if device is not None and torch.device(device).type == "cuda":
        n = int(g.get(_gsb.GSB_OPT_N_DYN))
        x, y, p = (torch.empty((replicas, n), dtype=torch.float32, device=device) for _ in range(3))
        g.state_device(x, y, p)
        return g, x, y, p
    x, y, p, _ = g.state()
    return g, torch.from_numpy(x), torch.from_numpy(y), torch.from_numpy(p)
