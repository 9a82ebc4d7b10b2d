"""torch.autograd binding of the taped particle steps.

DepositFn.apply(u, d, run) returns the time-integrated momentum source of a
run of taped steps as a function of the fluid velocity field u and the
particle diameters d; its backward calls the library's hand-written adjoint
(st_backward), in which the deposit's transpose is a gather of dL/dS at the
particle's cell and the interpolation's transpose a scatter onto the field.
"""
from dataclasses import dataclass

import numpy as np
import torch

from .tracker import Tracker


@dataclass
class Run:
    """What DepositFn runs: a fresh tracker, the initial positions and
    velocities (float64 [P, 3], host or device), and the steps."""
    tracker: Tracker
    x0: object
    up0: object
    dt: float
    nsteps: int
    tape_every: int = 20
    nsub: int = 1


class DepositFn(torch.autograd.Function):
    """S_int = DepositFn.apply(u, d, run).

    u: fluid velocity [3, nz, ny, nx] float64 on the device (cast to the
    tracker's field precision for the forward run); d: diameters [P]
    float64.  The gradient with respect to u is float64, the sum over the
    taped steps (every step uses u)."""

    @staticmethod
    def forward(ctx, u, d, run):
        t = run.tracker
        if t.count() != 0:
            raise ValueError("DepositFn needs a tracker without particles")
        dev = t.device
        x0 = torch.as_tensor(run.x0, dtype=torch.float64).to(dev)
        up0 = torch.as_tensor(run.up0, dtype=torch.float64).to(dev)
        t.inject(x0, up0, d.detach().to(dev, torch.float64))
        uf = u.detach().to(t.field_dtype).contiguous()
        t.sources(reset=True)
        for _ in range(run.nsteps):
            t.step(uf, run.dt, nsub=run.nsub, tape=run.tape_every)
        ctx.run = run
        ctx.uf = uf  # the taped steps borrow this buffer until backward
        ctx.u_dtype = u.dtype
        return t.sources()

    @staticmethod
    def backward(ctx, gS):
        dU, dd = ctx.run.tracker.backward(gS.contiguous())
        ctx.uf = None
        return dU.to(ctx.u_dtype), dd, None
