"""GPU adjoint (st_backward) against the FP64 oracle adjoint and central
finite differences of the GPU forward run.

Loss: L = sum (S_int - T)^2 over the time-integrated source, T built from a
run with the diameters scaled by 1.1; so dL/dS_int = 2 (S_int - T).
Gradients are compared with the oracle's in relative L2 norm and entry by
entry: the largest entry difference over the largest reference entry, and
the relative difference of every entry above a floor of 1e-3 of the largest.
The bounds are 1e-4 (norm and largest entry) for the FP32 chunk-local form
(forward in binary32, adjoint in binary64) and near round-off for the FP64
form; FD samples whose per-step cells change between the +h and -h runs are
excluded and counted.
"""
import numpy as np
import pytest

from gpu_helpers import fields, oracle_mesh, state, tracker, workload
from oracle.oracle import load as load_oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def orc():
    return load_oracle()


def _case(P=4000, n=(16, 16, 16), nsteps=30):
    return workload("adj64", n=n, P=P, nsteps=nsteps, noise=0.2)


def _forward(w, form, x, up, d, U, K, drag="stokes", interp="trilinear"):
    import torch
    t = tracker(w, form, drag=drag, interp=interp)
    t.inject(x, up, d)
    s0 = state(t)
    for _ in range(w.nsteps):
        t.step(U, w.dt, tape=K)
    S = t.sources()
    return t, s0, S


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


# entry-by-entry bounds: (largest difference / largest entry, relative
# difference of entries above 1e-3 of the largest)
ENTRY_TOL = {"fp64": (1e-9, 1e-7), "fp32_local": (1e-4, 1e-2)}


def _entrywise(g, ref, form, what):
    """Asserts the entry-by-entry bounds of the form; returns the two errors."""
    scale = np.abs(ref).max()
    emax = float(np.abs(g - ref).max() / scale)
    big = np.abs(ref) > 1e-3 * scale
    erel = float((np.abs(g - ref)[big] / np.abs(ref)[big]).max())
    print(f"{form} {what}: largest-entry error {emax:.3e}, worst relative error above the "
          f"floor {erel:.3e} over {int(big.sum())} entries")
    tmax, trel = ENTRY_TOL[form]
    assert emax <= tmax, (what, emax)
    assert erel <= trel, (what, erel)
    return emax, erel


def _far_from_faces(orc, mesh, Uor, fs, dts, nsub, x0, up0, d, band=1e-4):
    """Droplets whose oracle trajectory never starts a sub-step within `band`
    cell widths of a face (only those can deposit into another cell in a
    binary32 forward)."""
    h = mesh.h
    near = np.zeros(x0.shape[0], dtype=bool)
    x, u = x0, up0
    for k, dt in zip(fs, dts):
        for _ in range(nsub):
            q = x / h
            f = q - np.floor(q)
            near |= (np.minimum(f, 1.0 - f) < band).any(axis=1)
            x, u, _ = orc.run_par(mesh, Uor[k], x, u, d, dt / nsub, 1)
    return ~near


def _entrywise_far(orc, w, form, mesh, Ud, Uor, fs, dts, nsub, s0, lam, K,
                   drag="stokes", interp="trilinear", dd_full=None):
    """Entry-by-entry comparison for a binary32 forward.  The gradient for a
    given dL/dS_int is a sum over droplets, so the droplets that stay away
    from the faces are run again on their own (from the stored initial state,
    which re-injection reproduces exactly) and their adjoint is compared with
    the oracle's reverse pass over the same droplets, entry by entry; the
    droplets left out are counted."""
    import torch
    keep = _far_from_faces(orc, mesh, Uor, fs, dts, nsub, s0["x"], s0["up"], s0["d"])
    n = int(keep.sum())
    t = tracker(w, form, capacity=n, drag=drag, interp=interp)
    t.inject(s0["x"][keep], s0["up"][keep], s0["d"][keep])
    for k, dt in zip(fs, dts):
        t.step(Ud[k], dt, nsub=nsub, tape=K)
    dU, dd = (g.cpu().numpy() for g in t.backward(torch.from_numpy(lam).cuda()))
    t.close()
    oU, od = orc.adjoint_run_par(mesh, np.stack(Uor), fs, dts, nsub, s0["x"][keep],
                                 s0["up"][keep], s0["d"][keep], lam)
    print(f"per entry on the {n} of {keep.size} droplets away from the faces:")
    _entrywise(dU, oU.sum(axis=0), form, "dL/du")
    _entrywise(dd, od, form, "dL/dd")
    if dd_full is not None:
        # a droplet's dL/dd does not depend on the other droplets
        assert np.array_equal(dd, dd_full[keep])
    assert n > keep.size // 2
    return keep


def _entrywise_all(orc, w, form, mesh, Ud, Uor, fs, dts, nsub, s0, lam, K, dU, dd, oU, od,
                   drag="stokes", interp="trilinear"):
    if form == "fp64":
        _entrywise(dU, oU, form, "dL/du")
        _entrywise(dd, od, form, "dL/dd")
    else:
        _entrywise_far(orc, w, form, mesh, Ud, Uor, fs, dts, nsub, s0, lam, K, drag, interp,
                       dd_full=dd)


def _target(w, form, x, up, d, U, drag="stokes", interp="trilinear"):
    t = tracker(w, form, drag=drag, interp=interp)
    t.inject(x, up, d * 1.1)
    for _ in range(w.nsteps):
        t.step(U, w.dt)
    T = t.sources().cpu().numpy()
    t.close()
    return T


@pytest.mark.parametrize("form,tol,drag", [
    ("fp64", 1e-9, "stokes"), ("fp32_local", 1e-4, "stokes"),
    ("fp64", 1e-9, "schiller_naumann"), ("fp32_local", 1e-4, "schiller_naumann")])
def test_adjoint_matches_oracle(orc, form, tol, drag):
    import torch
    w = _case()
    if drag == "schiller_naumann":
        # larger droplets: slip Reynolds numbers of order one
        import dataclasses
        w = dataclasses.replace(w, d_median=60e-6)
    x, up, d = w.particles()
    Udev, Uor = fields(w, form)
    T = _target(w, form, x, up, d, Udev, drag)
    t, s0, S = _forward(w, form, x, up, d, Udev, K=7, drag=drag)
    lam = 2.0 * (S.cpu().numpy() - T)
    before = state(t)
    dU, dd = t.backward(torch.from_numpy(lam).cuda())
    after = state(t)
    for k in before:
        assert np.array_equal(before[k], after[k]), f"state restored after backward: {k}"
    dU, dd = dU.cpu().numpy(), dd.cpu().numpy()
    # the oracle differentiates from the GPU's stored initial state
    mesh = oracle_mesh(w, drag=drag)
    oU, od = orc.adjoint(mesh, Uor, s0["x"], s0["up"], s0["d"], w.dt, w.nsteps, lam)
    eU, ed = _rel(dU, oU), _rel(dd, od)
    print(form, drag, "adjoint rel L2: dU", eU, "dd", ed)
    assert eU < tol and ed < tol
    t.close()
    _entrywise_all(orc, w, form, mesh, [Udev], [Uor], [0] * w.nsteps, [w.dt] * w.nsteps, 1, s0,
                   lam, 7, dU, dd, oU, od, drag=drag)


@pytest.mark.parametrize("form,tol,interp,P", [
    ("fp64", 1e-9, "ngp", 4000), ("fp32_local", 1e-4, "ngp", 4000),
    ("fp64", 1e-9, "trilinear", 40000), ("fp32_local", 1e-4, "trilinear", 40000)])
def test_adjoint_ngp_and_crowded_chunks(orc, form, tol, interp, P):
    # nearest grid point (one corner per particle); and 5000 droplets per
    # chunk, so that the trilinear scatter runs over several batches
    import torch
    w = _case(P=P, nsteps=12 if P > 10000 else 30)
    x, up, d = w.particles()
    Udev, Uor = fields(w, form)
    T = _target(w, form, x, up, d, Udev, interp=interp)
    t, s0, S = _forward(w, form, x, up, d, Udev, K=5, interp=interp)
    lam = 2.0 * (S.cpu().numpy() - T)
    dU, dd = t.backward(torch.from_numpy(lam).cuda())
    dU, dd = dU.cpu().numpy(), dd.cpu().numpy()
    mesh = oracle_mesh(w, interp=1 if interp == "ngp" else 0)
    oU, od = orc.adjoint(mesh, Uor, s0["x"], s0["up"], s0["d"], w.dt, w.nsteps, lam)
    eU, ed = _rel(dU, oU), _rel(dd, od)
    print(form, interp, P, "adjoint rel L2: dU", eU, "dd", ed)
    assert eU < tol and ed < tol
    t.close()
    _entrywise_all(orc, w, form, mesh, [Udev], [Uor], [0] * w.nsteps, [w.dt] * w.nsteps, 1, s0,
                   lam, 5, dU, dd, oU, od, interp=interp)


@pytest.mark.parametrize("form,drag,interp,nsub,fs", [
    ("fp64", "stokes", "trilinear", 3, [0] * 10),
    ("fp32_local", "stokes", "trilinear", 3, [0] * 10),
    ("fp64", "schiller_naumann", "trilinear", 1, [0, 1, 2, 1, 0, 2, 2, 1, 0, 1]),
    ("fp32_local", "schiller_naumann", "trilinear", 2, [0, 1, 2, 1, 0, 2, 2, 1, 0, 1]),
    ("fp64", "stokes", "ngp", 3, [0, 1, 1, 0, 1, 0, 0, 1, 1, 0]),
    ("fp32_local", "schiller_naumann", "ngp", 2, [0, 1, 1, 0, 1, 0, 0, 1, 1, 0])])
def test_adjoint_substeps_and_fields(orc, form, drag, interp, nsub, fs):
    """Taped steps of nsub sub-steps each, and taped steps that read
    different fields (and step lengths): st_backward's dL/du is the sum over
    the taped sub-steps of the gradient with respect to the field each read,
    against the oracle's reverse pass over the same sub-steps and fields."""
    import dataclasses
    import torch
    w = _case(P=4000, nsteps=len(fs))
    if drag == "schiller_naumann":
        w = dataclasses.replace(w, d_median=60e-6)
    x, up, d = w.particles()
    rng = np.random.default_rng(17 + nsub)
    nf = max(fs) + 1
    U64 = [w.field()] + [w.field() + rng.normal(0.0, 0.3, size=w.field().shape)
                         for _ in range(nf - 1)]
    dts = [w.dt * (1.0 + 0.5 * ((k * 7) % 3 - 1)) for k in range(len(fs))]
    if form == "fp64":
        Ud = [torch.from_numpy(u).cuda() for u in U64]
        Uor = U64
    else:
        Ud = [torch.from_numpy(u.astype(np.float32)).cuda() for u in U64]
        Uor = [u.astype(np.float32).astype(np.float64) for u in U64]
    ti = "ngp" if interp == "ngp" else "trilinear"
    tt = tracker(w, form, drag=drag, interp=ti)
    tt.inject(x, up, d * 1.1)
    for k, dt in zip(fs, dts):
        tt.step(Ud[k], dt, nsub=nsub)
    T = tt.sources().cpu().numpy()
    tt.close()
    t = tracker(w, form, drag=drag, interp=ti)
    t.inject(x, up, d)
    s0 = state(t)
    for k, dt in zip(fs, dts):
        t.step(Ud[k], dt, nsub=nsub, tape=4)
    lam = 2.0 * (t.sources().cpu().numpy() - T)
    dU, dd = (g.cpu().numpy() for g in t.backward(torch.from_numpy(lam).cuda()))
    t.close()
    mesh = oracle_mesh(w, interp=1 if interp == "ngp" else 0, drag=drag)
    oU, od = orc.adjoint_run(mesh, np.stack(Uor), fs, dts, nsub, s0["x"], s0["up"], s0["d"], lam)
    oU = oU.sum(axis=0)
    tol = 1e-9 if form == "fp64" else 1e-4
    eU, ed = _rel(dU, oU), _rel(dd, od)
    print(form, drag, interp, nsub, nf, "adjoint rel L2: dU", eU, "dd", ed)
    assert eU < tol and ed < tol
    _entrywise_all(orc, w, form, mesh, Ud, Uor, fs, dts, nsub, s0, lam, 4, dU, dd, oU, od,
                   drag=drag, interp=ti)


def test_checkpoint_interval_does_not_change_gradient():
    import torch
    w = _case(P=3000, nsteps=12)
    x, up, d = w.particles()
    Udev, _ = fields(w, "fp64")
    lam = None
    grads = []
    for K in (1, 5, 12, 50):
        t, _, S = _forward(w, "fp64", x, up, d, Udev, K)
        if lam is None:
            lam = torch.sin(S * 1e3).contiguous()
        grads.append([g.cpu().numpy() for g in t.backward(lam)])
        t.close()
    for g in grads[1:]:
        assert _rel(g[0], grads[0][0]) < 1e-12 and _rel(g[1], grads[0][1]) < 1e-12


@pytest.mark.parametrize("form", ["fp64", "fp32_local"])
def test_repeated_taped_runs_reuse_buffers(form):
    """st_backward keeps the checkpoint buffers and its workspace for the next
    taped run: a second and a third taped run on the same tracker (other
    checkpoint intervals, so the workspace grows and is reused) give the
    gradients of a fresh tracker started from the same state, and
    st_tape_clear releases everything without disturbing the next run."""
    import torch
    w = _case(P=3000, nsteps=8)
    x, up, d = w.particles()
    Udev, _ = fields(w, form)
    a = tracker(w, form)
    a.inject(x, up, d)
    b = tracker(w, form)
    b.inject(x, up, d)
    lam = None
    for cycle, K in enumerate((4, 8, 3)):
        for _ in range(w.nsteps):
            a.step(Udev, w.dt, tape=K)
        Sa = a.sources(reset=True)
        if lam is None:
            lam = torch.sin(Sa * 1e3).contiguous()
        ga = [g.cpu().numpy() for g in a.backward(lam)]
        # the fresh reference: the same start state (b untaped to here), then
        # the same taped run in a tracker that never kept a tape
        c = tracker(w, form)
        sb = state(b)
        order = np.argsort(sb["id"])
        c.inject(sb["x"][order], sb["up"][order], sb["d"][order])
        for _ in range(w.nsteps):
            c.step(Udev, w.dt, tape=K)
            b.step(Udev, w.dt)
        c.sources(reset=True)
        b.sources(reset=True)
        gc = [g.cpu().numpy() for g in c.backward(lam)]
        c.close()
        tol = 1e-12 if form == "fp64" else 1e-6
        assert _rel(ga[0], gc[0]) < tol and _rel(ga[1], gc[1]) < tol, (cycle, K)
        if cycle == 1:
            a.tape_clear()   # nothing taped: releases the kept buffers
    a.close()
    b.close()


@pytest.mark.parametrize("form", ["fp64", "fp32_local"])
def test_tape_reserve(form):
    """st_tape_reserve allocates a taped run's checkpoints and its backward's
    workspace ahead: the run and its gradients match those of a tracker that
    allocates as it goes (checkpoints every 3 of 8 steps, and a second run
    with more checkpoints than were reserved), and reserving is refused
    while a tape is recorded and for invalid intervals."""
    import torch
    from paper_2603_26691_amd._native import STError
    w = _case(P=3000, nsteps=8)
    x, up, d = w.particles()
    Udev, _ = fields(w, form)
    lam = None
    for K, reserve in ((3, w.nsteps), (2, 4)):
        a = tracker(w, form)
        a.inject(x, up, d)
        a.tape_reserve(K, reserve)
        b = tracker(w, form)
        b.inject(x, up, d)
        for k in range(w.nsteps):
            a.step(Udev, w.dt, tape=K)
            b.step(Udev, w.dt, tape=K)
            if k == 0:
                with pytest.raises(STError):
                    a.tape_reserve(K, w.nsteps)   # a tape is recorded
        Sa, Sb = a.sources(), b.sources()
        # (the deposit's additions are ordered by atomics)
        assert float((Sa - Sb).norm() / Sb.norm()) < 1e-12
        if lam is None:
            lam = torch.sin(Sa * 1e3).contiguous()
        ga = [g.cpu().numpy() for g in a.backward(lam)]
        gb = [g.cpu().numpy() for g in b.backward(lam)]
        tol = 1e-12 if form == "fp64" else 1e-6
        assert _rel(ga[0], gb[0]) < tol and _rel(ga[1], gb[1]) < tol, K
        for bad in ((0, 8), (3, -1)):
            with pytest.raises(STError):
                a.tape_reserve(*bad)
        a.close()
        b.close()


@pytest.mark.parametrize("form,tol", [("fp64", 1e-9), ("fp32_local", 1e-4)])
def test_adjoint_across_full_rebins(orc, form, tol):
    """A plume spreading over a small mesh overflows its chunks' room, so full
    re-bins re-sort the store inside the taped segments: the adjoint records,
    indexed by each particle's slot in its segment's checkpoint, follow the
    particles through the re-sorted layouts (against the oracle adjoint)."""
    import torch
    import dataclasses
    w = _case(P=40000, n=(32, 32, 32), nsteps=24)
    w = dataclasses.replace(w, plumes=1, plume_fraction=1.0, plume_sigma=0.05, dt=4e-4, U0=3.0)
    x, up, d = w.particles()
    Udev, Uor = fields(w, form)
    t = tracker(w, form)
    t.inject(x, up, d)
    t.step(Udev, w.dt)          # places the injected droplets (a full re-bin)
    t.sources(reset=True)
    s0 = state(t)
    r0 = t.stats()["repacks"]
    for _ in range(w.nsteps):
        t.step(Udev, w.dt, tape=5)
    r1 = t.stats()["repacks"]
    S = t.sources()
    lam = torch.sin(S * 1e3).contiguous()
    dU, dd = (g.cpu().numpy() for g in t.backward(lam))
    t.close()
    print(form, "full re-bins during the taped steps:", r1 - r0)
    assert r1 - r0 >= 5   # (12 on the MI355X)
    mesh = oracle_mesh(w)
    oU, od = orc.adjoint(mesh, Uor, s0["x"], s0["up"], s0["d"], w.dt, w.nsteps,
                         lam.cpu().numpy())
    eU, ed = _rel(dU, oU), _rel(dd, od)
    print(form, "adjoint rel L2 across full re-bins: dU", eU, "dd", ed)
    assert eU < tol and ed < tol


@pytest.mark.parametrize("E", [2, 4])
@pytest.mark.parametrize("interp", ["trilinear", "ngp"])
def test_adjoint_small_chunks(orc, E, interp):
    """Chunks of 2^3 and 4^3 cells (their own tile sizes, node sums and fold
    of the per-chunk sums into dL/du), FP64 form, against the oracle
    adjoint."""
    import dataclasses
    import torch
    w = dataclasses.replace(_case(P=4000), chunk_edge=E)
    x, up, d = w.particles()
    Udev, Uor = fields(w, "fp64")
    t = tracker(w, "fp64", interp=interp)
    t.inject(x, up, d)
    s0 = state(t)
    for _ in range(w.nsteps):
        t.step(Udev, w.dt, tape=7)
    S = t.sources()
    lam = torch.sin(S * 1e3).contiguous()
    dU, dd = (g.cpu().numpy() for g in t.backward(lam))
    t.close()
    mesh = oracle_mesh(w, interp=1 if interp == "ngp" else 0)
    oU, od = orc.adjoint(mesh, Uor, s0["x"], s0["up"], s0["d"], w.dt, w.nsteps,
                         lam.cpu().numpy())
    print(E, interp, "adjoint rel L2: dU", _rel(dU, oU), "dd", _rel(dd, od))
    _entrywise(dU, oU, "fp64", "dL/du")
    _entrywise(dd, od, "fp64", "dL/dd")


def test_adjoint_against_finite_differences():
    """Central differences of the GPU's own FP64 forward (h = 1e-3 relative
    for diameters, 1e-3 m/s for field entries) on 32 sampled entries."""
    import torch
    w = _case(P=2000, nsteps=10)
    x, up, d = w.particles()
    Udev, _ = fields(w, "fp64")
    T = _target(w, "fp64", x, up, d, Udev)

    def run(dd, U):
        t = tracker(w, "fp64")
        t.inject(x, up, dd)
        cells = []
        for _ in range(w.nsteps):
            cells.append(state(t)["cell"])
            t.step(U, w.dt)
        S = t.sources().cpu().numpy()
        t.close()
        return float(np.sum((S - T) ** 2)), np.stack(cells)

    t, _, S = _forward(w, "fp64", x, up, d, Udev, K=4)
    lam = torch.from_numpy(2.0 * (S.cpu().numpy() - T)).cuda()
    dU, dd = (g.cpu().numpy() for g in t.backward(lam))
    t.close()
    _, cells0 = run(d, Udev)
    rng = np.random.default_rng(3)
    checked = skipped = 0
    for p in rng.choice(w.P, 16, replace=False):
        h = 1e-3 * d[p]
        dp_, dm_ = d.copy(), d.copy()
        dp_[p] += h
        dm_[p] -= h
        Lp, cp = run(dp_, Udev)
        Lm, cm = run(dm_, Udev)
        if not (np.array_equal(cp, cells0) and np.array_equal(cm, cells0)):
            skipped += 1
            continue
        fd = (Lp - Lm) / (2 * h)
        assert abs(fd - dd[p]) <= 2e-4 * abs(fd) + 1e-6 * np.abs(dd).max(), (p, fd, dd[p])
        checked += 1
    flat = np.argsort(-np.abs(dU).ravel())[:16]
    for q in flat:
        idx = np.unravel_index(q, dU.shape)
        Up, Um = Udev.clone(), Udev.clone()
        Up[idx] += 1e-3
        Um[idx] -= 1e-3
        Lp, cp = run(d, Up)
        Lm, cm = run(d, Um)
        if not (np.array_equal(cp, cells0) and np.array_equal(cm, cells0)):
            skipped += 1
            continue
        fd = (Lp - Lm) / 2e-3
        assert abs(fd - dU[idx]) <= 2e-4 * abs(fd) + 1e-6 * np.abs(dU).max(), (idx, fd, dU[idx])
        checked += 1
    print("FD checked", checked, "skipped", skipped)
    assert checked >= 24


def test_autograd_function():
    import torch
    import paper_2603_26691_amd as pkg
    from paper_2603_26691_amd.autograd import Run
    w = _case(P=2000, nsteps=8)
    x, up, d = w.particles()
    U = torch.from_numpy(w.field()).cuda().requires_grad_(True)
    dd = torch.from_numpy(d).cuda().requires_grad_(True)
    T = torch.from_numpy(_target(w, "fp32_local", x, up, d, U.detach().float())).cuda()
    run = Run(tracker(w, "fp32_local"), x, up, w.dt, w.nsteps, tape_every=3)
    S = pkg.DepositFn.apply(U, dd, run)
    loss = ((S - T) ** 2).sum()
    loss.backward()
    # a fresh binary32 copy of the field; the tracker keeps it alive while taped
    t2, _, S2 = _forward(w, "fp32_local", x, up, d, U.detach().float().contiguous(), K=3)
    gU, gd = (g.cpu().numpy() for g in t2.backward((2.0 * (S2 - T)).contiguous()))
    # the same run twice: the binary32 tile sums of dL/du depend on the order
    # of their atomic adds, so the two agree to binary32 rounding
    assert _rel(U.grad.cpu().numpy(), gU) < 1e-6
    assert _rel(dd.grad.cpu().numpy(), gd) < 1e-12
    run.tracker.close()
    t2.close()


def test_adjoint_full_size(orc):
    """Forward + adjoint at the differentiation workload's full size: 64^3,
    1e6 droplets, 200 steps of 5e-5 s, checkpoints every 20, FP32
    chunk-local forward, against the oracle's reverse pass over every droplet
    (its particle-parallel driver), from the GPU's stored initial state and
    the binary32 field, with the full dL/dS_int.  A droplet that the oracle's
    trajectory brings within 1e-4 cell widths of a face at the start of some
    step may deposit into the neighbouring cell in the binary32 forward; such
    droplets are left out of the per-droplet dL/dd comparison and counted,
    and their share of dL/du is what separates the two gradients beyond
    binary32 rounding.  The FP64 form's adjoint of the same problem is
    compared with the oracle as well."""
    import torch
    w = workload("adj64")
    x, up, d = w.particles()
    Udev, Uor = fields(w, "fp32_local")
    T = _target(w, "fp32_local", x, up, d, Udev)
    t, s0, S = _forward(w, "fp32_local", x, up, d, Udev, K=20)
    lam = 2.0 * (S.cpu().numpy() - T)
    lam_dev = torch.from_numpy(lam).cuda()
    dU, dd = [g.cpu().numpy() for g in t.backward(lam_dev)]
    t.close()
    # the FP64 form from the binary32 form's stored initial state, as the oracle
    t64, _, _ = _forward(w, "fp64", s0["x"], s0["up"], s0["d"], torch.from_numpy(Uor).cuda(),
                         K=20)
    dU64, dd64 = [g.cpu().numpy() for g in t64.backward(lam_dev)]
    t64.close()

    mesh = oracle_mesh(w)
    fs, dts = [0] * w.nsteps, [w.dt] * w.nsteps
    oU, od = orc.adjoint_run_par(mesh, Uor[None], fs, dts, 1, s0["x"], s0["up"], s0["d"], lam)
    oU = oU[0]
    eU, ed = _rel(dU, oU), _rel(dd, od)
    eU64, ed64 = _rel(dU64, oU), _rel(dd64, od)
    print(f"full size against the oracle over all {w.P} droplets: dL/du {eU:.3e}, dL/dd "
          f"{ed:.3e}; FP64 form: dL/du {eU64:.3e}, dL/dd {ed64:.3e}")
    assert eU < 1e-4 and ed < 1e-4
    assert eU64 < 1e-9 and ed64 < 1e-9
    _entrywise(dU64, oU, "fp64", "dL/du (FP64 form)")
    _entrywise(dd64, od, "fp64", "dL/dd (FP64 form)")
    _entrywise_far(orc, w, "fp32_local", mesh, [Udev], [Uor], fs, dts, 1, s0, lam, 20,
                   dd_full=dd)


def test_finite_differences_full_size():
    """Central differences (h = 1e-3 relative for diameters, 1e-6 m/s for
    field entries) of the GPU's FP64 forward at the differentiation
    workload's full size (64^3, 1e6 droplets, 200 steps) on 32 entries: 16
    random diameters and 16 field entries taken in order of decreasing
    gradient, against its adjoint with checkpoints every 20 steps.  An entry
    whose perturbed runs change any droplet's cell at any step is skipped,
    counted and replaced by the next one (the deposit cell is piecewise
    constant); at most 64 entries of each kind are tried.  A field entry
    moves every droplet near its node, dozens of them here: at 1e-3 m/s one
    of them crosses a face in the perturbed runs for nearly every entry,
    hence the smaller step, at which binary64 central differences are still
    accurate to far below the tolerance."""
    hU = 1e-6
    import torch
    w = workload("adj64")
    x, up, d = w.particles()
    Udev, _ = fields(w, "fp64")
    T = torch.from_numpy(_target(w, "fp64", x, up, d, Udev)).cuda()

    def run(dd, U, base=None):
        t = tracker(w, "fp64")
        t.inject(x, up, dd)
        cells, same = [], True
        for k in range(w.nsteps):
            c = t.particles()["cell"]
            if base is None:
                cells.append(c)
            elif same:
                same = torch.equal(c, base[k])
            t.step(U, w.dt)
        Lv = float(((t.sources() - T) ** 2).sum())
        t.close()
        return Lv, (cells if base is None else same)

    t, _, S = _forward(w, "fp64", x, up, d, Udev, K=20)
    lam = (2.0 * (S - T)).contiguous()
    dU, dd = (g.cpu().numpy() for g in t.backward(lam))
    t.close()
    _, cells0 = run(d, Udev)
    rng = np.random.default_rng(64)
    checked = skipped = 0
    for p in rng.choice(w.P, 64, replace=False):
        if checked == 16:
            break
        h = 1e-3 * d[p]
        dp_, dm_ = d.copy(), d.copy()
        dp_[p] += h
        dm_[p] -= h
        Lp, sp = run(dp_, Udev, cells0)
        Lm, sm = run(dm_, Udev, cells0)
        if not (sp and sm):
            skipped += 1
            continue
        fd = (Lp - Lm) / (2 * h)
        assert abs(fd - dd[p]) <= 2e-4 * abs(fd) + 1e-6 * np.abs(dd).max(), (p, fd, dd[p])
        checked += 1
    n_dd = checked
    for q in np.argsort(-np.abs(dU).ravel())[:64]:
        if checked == n_dd + 16:
            break
        idx = np.unravel_index(q, dU.shape)
        Up, Um = Udev.clone(), Udev.clone()
        Up[idx] += hU
        Um[idx] -= hU
        Lp, sp = run(d, Up, cells0)
        Lm, sm = run(d, Um, cells0)
        if not (sp and sm):
            skipped += 1
            continue
        fd = (Lp - Lm) / (2 * hU)
        assert abs(fd - dU[idx]) <= 2e-4 * abs(fd) + 1e-6 * np.abs(dU).max(), (idx, fd, dU[idx])
        checked += 1
    print("full-size FD checked", n_dd, "diameters and", checked - n_dd, "field entries;",
          "skipped", skipped)
    assert n_dd == 16 and checked == 32
