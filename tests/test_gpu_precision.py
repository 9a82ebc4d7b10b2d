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

from gpu_helpers import (displacement_bound, in_window, lockstep_window, min_image, oracle_mesh,
                         state, tracker, window_index, workload)
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
    plumes, 20 steps.  The binary64 form is checked against the oracle: on
    20 000 droplets sampled by id, advanced by the oracle from their binary64
    initial state over all 20 steps; and in every cell of a 12^3-cell window
    on a plume's flank, the oracle running, over all 20 steps, every droplet
    that starts close enough to reach the window (the distance a droplet can
    cover bounds the margin).  It then serves as the reference for all
    droplets and cells: reported per binary32 form, worst position error (per
    L), worst velocity error (m/s), worst per-cell source error (per the
    largest cell), cell indices that differ from the binary64 form's, and the
    global momentum drift.  Every form also takes one more lockstep step
    whose sources are checked against the oracle in every cell of a window."""
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
    orc = load_oracle()
    mesh = oracle_mesh(w)
    centre = np.floor(w.plume_centres()[0] / w.h).astype(int)
    win_lo, win_size = tuple(int(v) for v in centre + np.array([13, 0, 0]) - 6), 12
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
        if form == "fp64":
            # the droplets that can reach the window within the run
            s = t.particles()
            reach = displacement_bound(w, U, 0.0, float(s["d"].max()), w.nsteps, w.dt)
            margin = int(np.ceil(reach / w.h.min())) + 1
            sel = in_window(s["cell"], win_lo, win_size, w.n, margin)
            w_x, w_d = s["x"][sel].cpu().numpy(), s["d"][sel].cpu().numpy()
            del s, sel
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
            _, _, Sw = orc.run_par(mesh, U, w_x, np.zeros_like(w_x), w_d, w.dt, w.nsteps)
            wi = window_index(win_lo, win_size, w.n)
            Sg = S.cpu().numpy()
            werr = max(float(np.abs(Sg[c][wi] - Sw[c][wi]).max() / np.abs(Sw[c][wi]).max())
                       for c in range(3))
            print(f"\nfp64 form against the oracle in a {win_size}^3-cell window, all "
                  f"{w_x.shape[0]} droplets within {margin} cells of it over 20 steps: "
                  f"largest source error {werr:.3e}")
            assert werr < 1e-10
            del Sg
            xs, ds = np.concatenate(s_x), np.concatenate(s_d)
            xo, uo, _ = orc.run(mesh, U, xs, np.zeros_like(xs), ds, w.dt, w.nsteps)
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
        del S
        torch.cuda.empty_cache()
        err, k = lockstep_window(t, orc, mesh, Ud, U if form == "fp64" else
                                 U.astype(np.float32).astype(np.float64), w.dt,
                                 (int(centre[0]) - 8, int(centre[1]) - 8, int(centre[2]) - 8), 16,
                                 {"fp64": 1e-10, "fp32_local": 1e-6, "fp32": 1e-4}[form])
        print(f"{form}: lockstep step, 16^3 cells at a plume centre, {k} droplets, largest "
              f"source error {err:.3e}")
        del Ud
        torch.cuda.empty_cache()
    print("form        pos/L      vel[m/s]   src/max    cells differing  momentum drift")
    for form, r in rows.items():
        print(f"{form:10s} {r[0]:.3e}  {r[1]:.3e}  {r[2]:.3e}  {r[3]:15d}  {r[4]:.3e}")
    assert rows["fp32_local"][0] < 1e-5 and rows["fp32_local"][1] < 1e-5
    assert rows["fp32"][0] < 1e-4
    assert rows["fp32_local"][4] < 1e-6
