"""Precision study: the three forms against binary64 truth.

The plume workload's recipe (4 Gaussian plumes, sigma 0.05 L, noise 0.1
m/s) at 64^3 with 2e6 droplets, 20 steps of 5e-5 s.  The oracle gets the
binary64 initial state and the binary64 field (the truth), so every form's
total error is measured: storage rounding of the state and the field plus
arithmetic.  Reported per form: worst position error (per L), worst
velocity error (m/s), worst per-cell source error (per the largest cell),
and the global momentum drift (sum of sources against the particles'
momentum change, per sum of |momentum change|).
"""
import numpy as np
import pytest

from gpu_helpers import min_image, oracle_mesh, state, tracker, workload
from oracle.oracle import load as load_oracle

pytestmark = pytest.mark.gpu


def test_precision_study():
    import torch
    w = workload("plume256", n=(64, 64, 64), P=2_000_000)
    x, up, d = w.particles()
    U = w.field()
    orc = load_oracle()
    xo, uo, So = orc.run(oracle_mesh(w), U, x, up, d, w.dt, w.nsteps)
    L = np.array(w.L)
    m = (w.parcel_weight * w.rho_p * np.pi / 6.0) * d ** 3
    rows = {}
    for form in ("fp64", "fp32_local", "fp32"):
        t = tracker(w, form)
        t.inject(x, up, d)
        Ud = torch.from_numpy(U if form == "fp64" else U.astype(np.float32)).cuda()
        for _ in range(w.nsteps):
            t.step(Ud, w.dt)
        s = state(t)
        S = t.sources().cpu().numpy()
        pos = float(np.abs(min_image(s["x"] - xo, L)).max() / L.max())
        vel = float(np.abs(s["up"] - uo).max())
        src = float(max(np.abs(S[c] - So[c]).max() / np.abs(So[c]).max() for c in range(3)))
        dP = (m[:, None] * (s["up"] - up)).sum(axis=0)
        drift = (S.reshape(3, -1).sum(axis=1) * np.prod(w.h) + dP
                 - w.nsteps * w.dt * np.array(w.g) * m.sum())
        drift = float(np.max(np.abs(drift) / np.abs(m[:, None] * (s["up"] - up)).sum(axis=0)))
        rows[form] = (pos, vel, src, drift)
        t.close()
    print("\nform        pos/L      vel[m/s]   src/max    momentum drift")
    for form, r in rows.items():
        print(f"{form:10s} {r[0]:.3e}  {r[1]:.3e}  {r[2]:.3e}  {r[3]:.3e}")
    assert rows["fp64"][0] < 1e-12 and rows["fp64"][3] < 1e-12
    assert rows["fp32_local"][0] < 1e-5 and rows["fp32_local"][1] < 1e-5
    assert rows["fp32"][0] < 1e-4
