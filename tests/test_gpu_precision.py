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


def test_precision_study_full_size():
    """The precision study at its full size: 256^3 mesh, 2e8 droplets in 4
    plumes, 20 steps.  The oracle cannot step 2e8 droplets, so the binary64
    form serves as the reference for all of them, and that form is itself
    checked against the oracle on 20 000 droplets sampled by id, advanced
    by the oracle from their binary64 initial state over all 20 steps.
    Reported per binary32 form, over every droplet and cell: worst position
    error (per L), worst velocity error (m/s), worst per-cell source error
    (per the largest cell), cell indices that differ from the binary64
    form's, and the global momentum drift."""
    import torch
    w = workload("plume256")
    L = np.array(w.L)
    U = w.field()
    rng = np.random.default_rng(256)
    sample = np.sort(rng.choice(w.P, 20_000, replace=False))
    bsz = 1 << 25
    s_x, s_d = [], []
    ref = None
    rows = {}
    for form in ("fp64", "fp32_local", "fp32"):
        t = tracker(w, form)
        for b in range(w.n_device_batches(bsz)):
            x, up, d = w.device_batch(b, bsz)
            if form == "fp64":
                sel = sample[(sample >= b * bsz) & (sample < (b + 1) * bsz)] - b * bsz
                ix = torch.from_numpy(sel).cuda()
                s_x.append(x[ix].cpu().numpy())
                s_d.append(d[ix].cpu().numpy())
            t.inject(x, up, d)
            del x, up, d
        Ud = torch.from_numpy(U if form == "fp64" else U.astype(np.float32)).cuda()
        for _ in range(w.nsteps):
            t.step(Ud, w.dt)
        s = t.particles()
        S = t.sources()
        assert torch.equal(s["id"], torch.arange(w.P, device="cuda"))
        m = (w.parcel_weight * w.rho_p * np.pi / 6.0) * s["d"] ** 3
        mv = m[:, None] * s["up"]           # droplets start at rest
        g = torch.tensor(w.g, dtype=torch.float64, device="cuda")
        drift = (S.reshape(3, -1).sum(dim=1) * float(np.prod(w.h)) + mv.sum(dim=0)
                 - w.nsteps * w.dt * g * m.sum())
        drift = float((drift.abs() / mv.abs().sum(dim=0)).max())
        if form == "fp64":
            xs, ds = np.concatenate(s_x), np.concatenate(s_d)
            orc = load_oracle()
            xo, uo, _ = orc.run(oracle_mesh(w), U, xs, np.zeros_like(xs), ds, w.dt, w.nsteps)
            ix = torch.from_numpy(sample).cuda()
            pos = np.abs(min_image(s["x"][ix].cpu().numpy() - xo, L)).max() / L.max()
            vel = np.abs(s["up"][ix].cpu().numpy() - uo).max()
            print(f"\nfp64 form against the oracle on {sample.size} droplets: "
                  f"pos/L {pos:.3e}, vel {vel:.3e} m/s, momentum drift {drift:.3e}")
            assert pos < 1e-12 and vel < 1e-12 and drift < 1e-12
            ref = {"x": s["x"], "up": s["up"], "cell": s["cell"], "S": S}
            del s
        else:
            Lt = torch.tensor(L, dtype=torch.float64, device="cuda")
            dx = s["x"] - ref["x"]
            dx = dx - torch.round(dx / Lt) * Lt
            pos = float(dx.abs().max()) / L.max()
            vel = float((s["up"] - ref["up"]).abs().max())
            src = max(float((S[c] - ref["S"][c]).abs().max() / ref["S"][c].abs().max())
                      for c in range(3))
            cells = int((s["cell"] != ref["cell"]).any(dim=1).sum())
            rows[form] = (pos, vel, src, cells, drift)
            del s, dx
        t.close()
        del S, Ud
        torch.cuda.empty_cache()
    print("form        pos/L      vel[m/s]   src/max    cells differing  momentum drift")
    for form, r in rows.items():
        print(f"{form:10s} {r[0]:.3e}  {r[1]:.3e}  {r[2]:.3e}  {r[3]:15d}  {r[4]:.3e}")
    assert rows["fp32_local"][0] < 1e-5 and rows["fp32_local"][1] < 1e-5
    assert rows["fp32"][0] < 1e-4
    assert rows["fp32_local"][4] < 1e-6
