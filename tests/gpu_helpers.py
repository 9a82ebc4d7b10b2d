"""Shared pieces of the GPU parity tests: trackers built from a workload,
the oracle stepped from the GPU's own state (lockstep), and comparisons
that exclude, and count, particles within 1e-6 cell widths of a face."""
import dataclasses
import math

import numpy as np

from oracle.oracle import MeshParams, load as load_oracle
from workloads import synth

FORMS = ("fp64", "fp32_local", "fp32")
BAND = 1e-6  # cell widths


def band(form, n):
    """Cell widths around a face within which the two sides may place a
    particle in different cells.  The FP32-everywhere form takes a cell from
    the binary32 product x * fl(n / L), within 2^-23 * n cells of x n / L,
    and its positions carry a binary32 rounding of up to 2^-24 * n cells: a
    band of 2^-21 * n cells holds both with a factor of 2 to spare."""
    return max(BAND, 2.0 ** -21 * max(n)) if form == "fp32" else BAND


def workload(name="tg32", **kw):
    w = synth.get(name)
    return dataclasses.replace(w, **kw) if kw else w


DRAGS = ("stokes", "schiller_naumann")   # oracle drag codes 0, 1


def oracle_mesh(w, interp=0, drag="stokes"):
    return MeshParams(interp=interp, drag=DRAGS.index(drag), **w.mesh_kwargs())


def tracker(w, form, capacity=None, interp="trilinear", drag="stokes"):
    import paper_2603_26691_amd as pkg
    return pkg.Tracker(w.n, w.L, capacity or max(w.P, 1), form=form, interp=interp,
                       chunk_edge=w.chunk_edge, rho_f=w.rho_f, mu_f=w.mu_f, g=w.g,
                       rho_p=w.rho_p, parcel_weight=w.parcel_weight, drag=drag)


def fields(w, form):
    """(device field for the tracker, float64 field the oracle gets)."""
    import torch
    U = w.field()
    if form == "fp64":
        return torch.from_numpy(U).cuda(), U
    U32 = U.astype(np.float32)
    return torch.from_numpy(U32).cuda(), U32.astype(np.float64)


def state(t):
    s = t.particles()
    return {k: v.cpu().numpy() for k, v in s.items()}


def face_distance(x, h):
    """Distance of each coordinate to the nearest cell face, in cell widths."""
    q = x / h
    f = q - np.floor(q)
    return np.minimum(f, 1.0 - f)


def min_image(dx, L):
    L = np.asarray(L)
    return dx - np.round(dx / L) * L


def lockstep_check(t, orc, mesh, Udev, Uor, dt, nsteps, tol, nsub=1, band_=BAND, ngp=False):
    """Steps the tracker and, from the GPU's state at every step, the oracle.

    tol: dict with keys pos (/L), vel (/1 m/s), src (per-cell, relative to the
    largest cell); band_: the face band in cell widths (band()); ngp: the
    field is taken from the start cell (nearest grid point), so a particle
    whose start cell differs between the two sides (within the band) gets a
    different field value and is left out of every comparison (counted).
    Returns the worst errors and the counts of excluded particles and
    cells."""
    L = np.array(mesh.L)
    h = mesh.h
    worst = {"pos": 0.0, "vel": 0.0, "src": 0.0, "band_cells": 0, "band_src_cells": 0,
             "compared": 0, "band_start_cells": 0}
    t.sources(reset=True)
    s0 = state(t)
    for _ in range(nsteps):
        t.step(Udev, dt, nsub=nsub)
        s1 = state(t)
        Sg = t.sources(reset=True).cpu().numpy()
        xo, uo, So = orc.run(mesh, Uor, s0["x"], s0["up"], s0["d"], dt, 1, nsub=nsub)
        assert np.array_equal(s1["id"], np.arange(s1["id"].shape[0])), "ids are a permutation"
        assert np.array_equal(s1["d"], s0["d"]), "diameters travel with their particles"
        # start cells: they differ between the two sides only within the band
        c0o = orc.cells(mesh, s0["x"])
        diff0 = (c0o != s0["cell"]).any(axis=1)
        assert not (diff0 & ~(face_distance(s0["x"], h) < band_).any(axis=1)).any()
        keep_p = ~diff0 if ngp else np.ones(diff0.shape, dtype=bool)
        worst["band_start_cells"] += int(diff0.sum())
        dpos = np.abs(min_image(s1["x"] - xo, L))[keep_p] / L
        dvel = np.abs(s1["up"] - uo)[keep_p]
        if dpos.size:
            worst["pos"] = max(worst["pos"], float(dpos.max()))
            worst["vel"] = max(worst["vel"], float(dvel.max()))
        # cells after the step: bit-exact away from the faces
        co = orc.cells(mesh, xo)
        near = (face_distance(xo, h) < band_).any(axis=1) | ~keep_p
        mism = (co != s1["cell"]).any(axis=1)
        assert not (mism & ~near).any(), \
            f"cell mismatch away from faces: {np.argwhere(mism & ~near)[:5].ravel()}"
        worst["band_cells"] += int(near.sum())
        worst["compared"] += int((~near).sum())
        # sources: a particle whose start-of-step cell differs between the
        # two sides (only possible within the band) puts its impulse in
        # different cells; those cells are left out and counted
        keep = np.ones(Sg.shape[1:], dtype=bool)
        for p in np.nonzero(diff0)[0]:
            for c in (c0o[p], s0["cell"][p]):
                keep[c[2], c[1], c[0]] = False
        worst["band_src_cells"] += int((~keep).sum())
        for comp in range(3):
            ref = So[comp]
            scale = np.abs(ref).max()
            if scale == 0:
                continue
            err = np.abs(Sg[comp] - ref)[keep].max() / scale
            worst["src"] = max(worst["src"], float(err))
        s0 = s1
    assert worst["pos"] <= tol["pos"], worst
    assert worst["vel"] <= tol["vel"], worst
    assert worst["src"] <= tol["src"], worst
    return worst


def sphere_mass(d, w=1.0, rho_p=1000.0):
    return w * rho_p * math.pi * d ** 3 / 6.0


def in_window(cell, lo, size, n, margin=0):
    """Mask of cells (int [P, 3], torch or numpy) inside the periodic window of
    cells [lo - margin, lo + size + margin) per axis."""
    ok = None
    for a in range(3):
        r = (cell[:, a] - (lo[a] - margin)) % n[a]
        m = r < size + 2 * margin
        ok = m if ok is None else ok & m
    return ok


def window_index(lo, size, n):
    """Index arrays (z, y, x) of the window's cells in a [nz, ny, nx] field."""
    ax = [(np.arange(size) + lo[a]) % n[a] for a in range(3)]
    return np.ix_(ax[2], ax[1], ax[0])


def lockstep_window(t, orc, mesh, Udev, Uor, dt, lo, size, tol):
    """One lockstep step checked per cell over a window of cells, at any size:
    a cell's source comes only from the droplets whose cell at the start of
    the step is that cell, so the oracle steps exactly the droplets that the
    GPU holds in the window (their stored state promoted to binary64) and the
    two sources must agree in every window cell to `tol` of the largest.  A
    droplet on a face that the two sides place in different cells (binary32
    cell arithmetic, within the face band) leaves both cells out.  Returns
    (error, droplets in the window)."""
    import torch
    t.sources(reset=True)
    s = t.particles()
    sel = in_window(s["cell"], lo, size, mesh.n)
    xs, us, ds, cs = (s[k][sel].cpu().numpy() for k in ("x", "up", "d", "cell"))
    del s, sel
    co = orc.cells(mesh, xs)
    split = np.nonzero((co != cs).any(axis=1))[0]
    keep = np.ones(tuple(mesh.n[::-1]), dtype=bool)
    for p in split:
        for c in (co[p], cs[p]):
            keep[c[2], c[1], c[0]] = False
    torch.cuda.empty_cache()
    t.step(Udev, dt)
    S = t.sources(reset=True).cpu().numpy()
    _, _, So = orc.run_par(mesh, Uor, xs, us, ds, dt, 1)
    wi = window_index(lo, size, mesh.n)
    kw = keep[wi]
    err = 0.0
    for c in range(3):
        ref = So[c][wi]
        scale = np.abs(ref).max()
        if scale > 0:
            err = max(err, float(np.abs(S[c][wi] - ref)[kw].max() / scale))
    assert err <= tol, (err, tol, lo, size)
    return err, xs.shape[0]


def displacement_bound(w, U, up0_max, d_max, nsteps, dt):
    """Largest distance [m] a droplet can travel in nsteps steps of dt (Stokes
    drag): each velocity update is a convex combination of the old velocity
    and u_f + tau g, so |u_p| never exceeds max(|u_p0|, max|u_f| + tau_max |g|)."""
    tau_max = w.rho_p * d_max ** 2 / (18.0 * w.mu_f)
    umax = float(np.sqrt((np.asarray(U) ** 2).sum(axis=0)).max())
    vmax = max(up0_max, umax + tau_max * float(np.linalg.norm(w.g)))
    return nsteps * dt * vmax
