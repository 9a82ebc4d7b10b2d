"""A second derivative of the particle step, independent of the oracle's own
reverse pass: the step written again with torch float64 operations on the
CPU and differentiated by torch's autograd, against or_adjoint_run.

The paper defines no adjoint; what both sides differentiate is the discrete
step of paper Sec. 2.1 (equation of motion, Stokes or Schiller-Naumann drag,
momentum source into the containing cell) and Sec. 2.5 (semi-implicit Euler,
trilinear or nearest-grid-point gather), with the sub-steps of Sec. 3.3 and
a field per step.  The forward below shares nothing with the oracle's C code
but the definitions; the cell index and the periodic wrap are piecewise
constant, so autograd sees them as constants, as the reverse pass does.
Agreement to 1e-12 of the largest entry (binary64 round-off of two
different evaluation orders) pins the reverse pass term by term.
"""
import math

import numpy as np
import pytest
import torch

from oracle.oracle import MeshParams, load as load_oracle


def _torch_run(mesh, fields, fs, dts, nsub, x0, up0, d):
    """Time-integrated source of the run, as a differentiable torch tensor."""
    n = torch.tensor(mesh.n, dtype=torch.int64)
    L = torch.tensor(mesh.L, dtype=torch.float64)
    h = L / n.to(torch.float64)
    V = float(h[0] * h[1] * h[2])
    g = torch.tensor(mesh.g, dtype=torch.float64)
    nx, ny, nz = mesh.n
    S = torch.zeros((3, nz, ny, nx), dtype=torch.float64)
    x, up = x0.clone(), up0.clone()
    comp = torch.arange(3)
    for step, k in enumerate(fs):
        F = fields[k]
        dt = dts[step] / nsub
        for _ in range(nsub):
            c0 = torch.remainder(torch.floor(x.detach() / h).to(torch.int64), n)  # [P, 3]
            if mesh.interp == 1:
                uf = F[:, c0[:, 2], c0[:, 1], c0[:, 0]].T
            else:
                s = x / h - 0.5
                i0 = torch.floor(s.detach())
                f = s - i0
                i0 = i0.to(torch.int64)
                uf = torch.zeros_like(x)
                for corner in range(8):
                    b = [(corner >> a) & 1 for a in range(3)]
                    w = torch.ones(x.shape[0], dtype=torch.float64)
                    idx = []
                    for a in range(3):
                        w = w * (f[:, a] if b[a] else 1.0 - f[:, a])
                        idx.append(torch.remainder(i0[:, a] + b[a], n[a]))
                    uf = uf + w[:, None] * F[:, idx[2], idx[1], idx[0]].T
            tau = mesh.rho_p * d ** 2 / (18.0 * mesh.mu_f)
            if mesh.drag == 1:
                slip = uf - up
                Re = mesh.rho_f * torch.sqrt((slip ** 2).sum(dim=1)) * d / mesh.mu_f
                tau = tau / (1.0 + 0.15 * Re ** 0.687)
            m = mesh.parcel_weight * mesh.rho_p * math.pi * d ** 3 / 6.0
            upn = (tau[:, None] * up + dt * uf + tau[:, None] * dt * g) / (tau[:, None] + dt)
            J = m[:, None] * (upn - up - g * dt)
            for a in range(3):
                S = S.index_put((comp[a].expand(x.shape[0]), c0[:, 2], c0[:, 1], c0[:, 0]),
                                -J[:, a] / V, accumulate=True)
            x = x + dt * upn
            x = torch.where(x >= L, x - L, x)
            x = torch.where(x < 0.0, x + L, x)
            x = torch.where(x == L, torch.zeros_like(x), x)
            up = upn
    return S


CASES = [
    # drag, interp, nsub, fields per step, step lengths
    (0, 0, 1, [0] * 5, [2e-4] * 5),
    (1, 0, 1, [0] * 5, [2e-4] * 5),
    (0, 0, 3, [0, 1, 0, 1], [2e-4, 1e-4, 3e-4, 2e-4]),
    (1, 0, 2, [0, 1, 2, 1], [2e-4, 1e-4, 3e-4, 2e-4]),
    (0, 1, 2, [0, 1, 1], [2e-4, 3e-4, 1e-4]),
    (1, 1, 1, [0, 0, 1, 1], [2e-4] * 4),
]


@pytest.mark.parametrize("drag,interp,nsub,fs,dts", CASES)
def test_autograd_matches_oracle_adjoint(drag, interp, nsub, fs, dts):
    orc = load_oracle()
    rng = np.random.default_rng(100 + 10 * drag + 3 * interp + nsub)
    mesh = MeshParams(n=(8, 6, 4), L=(0.01, 0.0075, 0.005), rho_p=1000.0, mu_f=1.8e-5,
                      parcel_weight=3.0, drag=drag, interp=interp, g=(0.5, -1.0, -9.81))
    nf = max(fs) + 1
    fields = rng.normal(0.0, 0.5, size=(nf, 3, 4, 6, 8))
    P = 12
    x0 = rng.random((P, 3)) * np.array(mesh.L)
    up0 = rng.normal(0.0, 0.3, size=(P, 3))
    d = np.exp(rng.normal(math.log(40e-6 if drag == 0 else 120e-6), 0.3, size=P))
    lam = rng.normal(size=(3, 4, 6, 8))

    Ft = torch.tensor(fields, requires_grad=True)
    dtt = torch.tensor(d, requires_grad=True)
    S = _torch_run(mesh, Ft, fs, dts, nsub, torch.tensor(x0), torch.tensor(up0), dtt)
    (S * torch.tensor(lam)).sum().backward()

    Ub, db = orc.adjoint_run(mesh, fields, fs, dts, nsub, x0, up0, d, lam)
    # the forward sources agree too (the same discrete step)
    So = np.zeros_like(lam)
    x, up = x0, up0
    for k, dt in zip(fs, dts):
        x, up, So = orc.run(mesh, fields[k], x, up, d, dt, 1, nsub=nsub, Su_int=So)
    assert np.abs(S.detach().numpy() - So).max() <= 1e-12 * np.abs(So).max()
    gU, gd = Ft.grad.numpy(), dtt.grad.numpy()
    assert np.abs(gU - Ub).max() <= 1e-12 * np.abs(Ub).max(), "dL/dU"
    assert np.abs(gd - db).max() <= 1e-12 * np.abs(db).max(), "dL/dd"
    # per entry above a floor of 1e-3 of the largest
    for g_, o_ in ((gU, Ub), (gd, db)):
        big = np.abs(o_) > 1e-3 * np.abs(o_).max()
        assert (np.abs(g_ - o_)[big] <= 1e-10 * np.abs(o_)[big]).all()
