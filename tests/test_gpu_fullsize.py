"""Parity at the benchmark's full size and launch configuration.

tg128: 128^3 mesh, 1e7 droplets, FP32 chunk-local form, the same tracker
configuration bench.py times.  After warm-up steps the oracle advances a
random sample of 20 000 particles, one by one, from the GPU's state with the
field the GPU used, and the sample is compared with the GPU's next state;
the deposited source is checked over all particles through the momentum
balance (sum of sources = minus the particles' drag impulse).
"""
import numpy as np
import pytest

from gpu_helpers import (BAND, face_distance, fields, lockstep_window, min_image, oracle_mesh,
                         tracker, workload)
from oracle.oracle import load as load_oracle

pytestmark = pytest.mark.gpu


def _sample(s, idx):
    return {k: v[idx].cpu().numpy() for k, v in s.items()}


def test_tg128_sampled_parity():
    import torch
    w = workload("tg128")
    t = tracker(w, "fp32_local")
    for b in range(w.n_batches()):
        t.inject(*w.batch(b))
    Udev, Uor = fields(w, "fp32_local")
    for _ in range(5):
        t.step(Udev, w.dt)
    rng = np.random.default_rng(128)
    idx = torch.from_numpy(rng.choice(w.P, 20000, replace=False)).cuda()
    orc = load_oracle()
    mesh = oracle_mesh(w)
    L = np.array(w.L)
    for step in range(3):
        s0 = t.particles()
        a = _sample(s0, idx)
        t.sources(reset=True)
        t.step(Udev, w.dt)
        s1 = t.particles()
        b = _sample(s1, idx)
        xo, uo, _ = orc.run(mesh, Uor, a["x"], a["up"], a["d"], w.dt, 1)
        pos = np.abs(min_image(b["x"] - xo, L)).max() / L.max()
        vel = np.abs(b["up"] - uo).max()
        near = (face_distance(xo, w.h) < BAND).any(axis=1)
        co = orc.cells(mesh, xo)
        assert np.array_equal(co[~near], b["cell"][~near])
        assert pos < 1e-5 and vel < 1e-5, (pos, vel)
        # all particles: sum of the step's sources = minus the drag impulse
        S = t.sources(reset=True)
        m = (w.parcel_weight * w.rho_p * np.pi / 6.0) * s0["d"] ** 3
        g = torch.tensor(w.g, dtype=torch.float64, device="cuda")
        J = (m[:, None] * (s1["up"] - s0["up"] - g * w.dt)).sum(dim=0)
        scale = (m[:, None] * (s1["up"] - s0["up"])).abs().sum(dim=0)
        Ssum = S.reshape(3, -1).sum(dim=1) * float(np.prod(w.h))
        resid = ((Ssum + J).abs() / scale).cpu().numpy()
        print("step", step, "pos", pos, "vel", vel, "band", int(near.sum()), "balance", resid)
        assert np.all(resid < 1e-6)
    assert np.array_equal(s1["id"].cpu().numpy(), np.arange(w.P))
    del s0, s1
    # one more lockstep step, every source of a 32^3-cell window against the
    # oracle stepping every droplet that starts the step in it
    err, k = lockstep_window(t, orc, mesh, Udev, Uor, w.dt, (40, 72, 8), 32, 1e-6)
    print(f"window of 32^3 cells: {k} droplets, largest source error {err:.3e}")
    t.close()


def test_plume512_coupled_sampled_parity():
    """plume512: 512^3 mesh, 1.4e9 droplets (60 % in one plume), FP32
    chunk-local form, 10 steps with the field rotated by 1 degree per step on
    the second stream, in the configuration bench.py times.  The oracle
    advances 20 000 droplets sampled by id from the GPU's stored initial
    state through the same rotating schedule; over all droplets the sum of
    the sources is checked against minus their drag impulse."""
    import torch
    w = workload("plume512")
    t = tracker(w, "fp32_local")
    for b in range(w.n_device_batches()):
        x, up, d = w.device_batch(b)
        t.inject(x, up, d)
        del x, up, d
    rng = np.random.default_rng(512)
    idx = torch.from_numpy(np.sort(rng.choice(w.P, 20000, replace=False))).cuda()
    s = t.particles()
    a = _sample(s, idx)
    assert not a["up"].any()                      # droplets start at rest
    del s
    torch.cuda.empty_cache()
    U0dev, U0 = fields(w, "fp32_local")
    cs = w.rotation()
    t.run_coupled(U0dev, cs, w.dt, timed=False)
    s = t.particles()
    b = _sample(s, idx)
    c = w.parcel_weight * w.rho_p * np.pi / 6.0
    f64 = dict(dtype=torch.float64, device="cuda")
    mu, scale, M = torch.zeros(3, **f64), torch.zeros(3, **f64), torch.zeros((), **f64)
    for i in range(0, w.P, 1 << 26):
        m = c * s["d"][i:i + (1 << 26)] ** 3
        p = m[:, None] * s["up"][i:i + (1 << 26)]
        mu += p.sum(dim=0)
        scale += p.abs().sum(dim=0)
        M += m.sum()
        del m, p
    del s
    g = torch.tensor(w.g, **f64)
    J = mu - w.nsteps * w.dt * g * M               # drag impulse of all droplets
    S = t.sources()
    Ssum = S.reshape(3, -1).sum(dim=1) * float(np.prod(w.h))
    resid = ((Ssum + J).abs() / scale).cpu().numpy()
    del S
    orc = load_oracle()
    mesh = oracle_mesh(w)
    # one more step with the next field of the schedule (rotated on the host,
    # rounded to binary32), every source of two windows against the oracle
    # stepping every droplet that starts the step in them: 16^3 cells at the
    # plume's centre and 32^3 cells of the uniform background
    th = np.deg2rad(w.rotate_deg * w.nsteps)
    Un = np.stack([np.cos(th) * U0[0] - np.sin(th) * U0[1],
                   np.sin(th) * U0[0] + np.cos(th) * U0[1], U0[2]]).astype(np.float32)
    Undev = torch.from_numpy(Un).cuda()
    centre = tuple(int(v) for v in np.floor(w.plume_centres()[0] / w.h))
    for lo, size in [(tuple(c - 8 for c in centre), 16),
                     (tuple((c + 256) % 512 for c in centre), 32)]:
        err, k = lockstep_window(t, orc, mesh, Undev, Un.astype(np.float64), w.dt, lo, size,
                                 1e-6)
        print(f"window of {size}^3 cells at {lo}: {k} droplets, largest source error {err:.3e}")
    t.close()
    xo, uo, _ = orc.run_rotating(mesh, U0, cs, a["x"], a["up"], a["d"], w.dt, w.nsteps)
    L = np.array(w.L)
    pos = np.abs(min_image(b["x"] - xo, L)).max() / L.max()
    vel = np.abs(b["up"] - uo).max()
    print("plume512 coupled: pos", pos, "vel", vel, "balance", resid)
    assert pos < 1e-5 and vel < 1e-5, (pos, vel)
    assert np.all(resid < 1e-6)
