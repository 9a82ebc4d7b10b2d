"""Seeded synthetic inputs shaped like the paper's particle-laden flows.

This module only draws inputs: the mesh and material parameters, a
cell-centred fluid velocity field, and particle positions, velocities and
diameters.  It holds none of the method's arithmetic, and both the oracle
side and the GPU side take their inputs from here.

Recipe (stand-ins for the OpenFOAM cloud-chamber and scaling cases of the
paper, Sec. 3.2 and Sec. 4, whose flow fields are not available):
  * field: Taylor-Green-like cell-centred velocity
        u = U0 (sin kx cos ky cos kz, -cos kx sin ky cos kz, 0),
    k = 2 pi / L per axis, evaluated at the cell centres (i + 1/2) h, plus
    optionally i.i.d. N(0, noise^2) per cell and component;
  * positions: uniform on the periodic box, or Gaussian plumes (wrapped),
    giving strongly uneven occupancy of the 8^3-cell chunks;
  * diameters: lognormal, median 20 um, sigma_ln 0.4 (water droplets);
  * initial particle velocity 0.
Random streams come from numpy SeedSequence: the field noise and the plume
centres from SeedSequence(seed), the particles batch by batch from
SeedSequence([seed, batch]) so that any batch can be drawn on its own.
"""
from dataclasses import dataclass, field
import math

import numpy as np

BATCH = 1 << 22  # particles per independently seeded batch


@dataclass
class Workload:
    name: str
    n: tuple
    P: int
    nsteps: int
    dt: float
    seed: int
    L: tuple = (0.1, 0.1, 0.1)
    U0: float = 1.0
    noise: float = 0.0          # std of the per-cell field perturbation [m/s]
    plumes: int = 0             # number of Gaussian plumes (0 = uniform)
    plume_fraction: float = 1.0  # share of particles in plumes
    plume_sigma: float = 0.05   # plume std as a fraction of L
    nsub: int = 1
    rotate_deg: float = 0.0     # field rotation about z per step (coupled run)
    d_median: float = 20e-6
    d_sigma_ln: float = 0.4
    rho_f: float = 1.2
    mu_f: float = 1.8e-5
    rho_p: float = 1000.0
    g: tuple = (0.0, 0.0, -9.81)
    parcel_weight: float = 1.0
    chunk_edge: int = 8

    # ------------------------------------------------------------------
    def mesh_kwargs(self):
        """Plain mesh/material parameters, for either side's own mesh type."""
        return dict(n=tuple(self.n), L=tuple(self.L), rho_f=self.rho_f, mu_f=self.mu_f,
                    g=tuple(self.g), rho_p=self.rho_p, parcel_weight=self.parcel_weight)

    @property
    def h(self):
        return np.array(self.L, dtype=np.float64) / np.array(self.n, dtype=np.float64)

    def scaled(self, P=None, nsteps=None, n=None, name=None):
        """Same recipe with another particle count, step count or mesh."""
        kw = dict(self.__dict__)
        if P is not None:
            kw["P"] = int(P)
        if nsteps is not None:
            kw["nsteps"] = int(nsteps)
        if n is not None:
            kw["n"] = tuple(n)
        kw["name"] = name or self.name
        return Workload(**kw)

    # ------------------------------------------------------------------
    def field(self):
        """Cell-centred fluid velocity, float64 [3, nz, ny, nx]."""
        nx, ny, nz = self.n
        Lx, Ly, Lz = self.L
        xc = (np.arange(nx) + 0.5) * (Lx / nx)
        yc = (np.arange(ny) + 0.5) * (Ly / ny)
        zc = (np.arange(nz) + 0.5) * (Lz / nz)
        kx, ky, kz = 2 * math.pi / Lx, 2 * math.pi / Ly, 2 * math.pi / Lz
        sx, cx = np.sin(kx * xc), np.cos(kx * xc)
        sy, cy = np.sin(ky * yc), np.cos(ky * yc)
        cz = np.cos(kz * zc)
        U = np.empty((3, nz, ny, nx), dtype=np.float64)
        U[0] = self.U0 * cz[:, None, None] * cy[None, :, None] * sx[None, None, :]
        U[1] = -self.U0 * cz[:, None, None] * sy[None, :, None] * cx[None, None, :]
        U[2] = 0.0
        if self.noise > 0:
            rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(self.seed).spawn(2)[0]))
            for c in range(3):
                U[c] += rng.normal(0.0, self.noise, size=(nz, ny, nx))
        return U

    def plume_centres(self):
        if self.plumes == 0:
            return np.zeros((0, 3))
        rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(self.seed).spawn(2)[1]))
        return rng.random((self.plumes, 3)) * np.array(self.L)

    def n_batches(self):
        return (self.P + BATCH - 1) // BATCH

    def batch(self, b):
        """Particles [b*BATCH, min(P, (b+1)*BATCH)): (x [k,3], up [k,3], d [k]) float64."""
        start = b * BATCH
        k = min(self.P, start + BATCH) - start
        if k <= 0:
            z = np.zeros((0, 3))
            return z, z.copy(), np.zeros(0)
        ss = np.random.SeedSequence([self.seed, b])
        r_pos, r_d, r_sel = [np.random.Generator(np.random.PCG64(s)) for s in ss.spawn(3)]
        L = np.array(self.L, dtype=np.float64)
        x = r_pos.random((k, 3)) * L
        if self.plumes > 0:
            centres = self.plume_centres()
            in_plume = r_sel.random(k) < self.plume_fraction
            which = r_sel.integers(0, self.plumes, size=k)
            m = int(in_plume.sum())
            off = r_pos.normal(0.0, 1.0, size=(m, 3)) * (self.plume_sigma * L)
            x[in_plume] = np.mod(centres[which[in_plume]] + off, L)
            # np.mod can round a tiny negative offset up to exactly L.
            x = np.where(x >= L, 0.0, x)
        d = np.exp(r_d.normal(math.log(self.d_median), self.d_sigma_ln, size=k))
        up = np.zeros((k, 3), dtype=np.float64)
        return x, up, d

    def particles(self, count=None):
        """The first `count` particles (all by default), concatenated over batches."""
        count = self.P if count is None else min(int(count), self.P)
        xs, us, ds = [], [], []
        b = 0
        got = 0
        while got < count:
            x, up, d = self.batch(b)
            take = min(count - got, x.shape[0])
            xs.append(x[:take]); us.append(up[:take]); ds.append(d[:take])
            got += take
            b += 1
        if not xs:
            z = np.zeros((0, 3))
            return z, z.copy(), np.zeros(0)
        return np.concatenate(xs), np.concatenate(us), np.concatenate(ds)

    def device_batch(self, b, batch=1 << 25, device="cuda"):
        """Particles [b*batch, min(P, (b+1)*batch)) drawn on the GPU with torch's
        seeded generator (same recipe, different random stream from batch()):
        (x [k,3], up [k,3], d [k]) float64 device tensors.  For workloads too
        large to draw on the host; a sample copied back is a valid oracle input."""
        import torch
        start = b * batch
        k = min(self.P, start + batch) - start
        f64 = torch.float64
        if k <= 0:
            z = torch.zeros((0, 3), dtype=f64, device=device)
            return z, z.clone(), torch.zeros(0, dtype=f64, device=device)
        seed = int(np.random.SeedSequence([self.seed, b, 77]).generate_state(1, np.uint64)[0])
        g = torch.Generator(device=device)
        g.manual_seed(seed)
        L = torch.tensor(self.L, dtype=f64, device=device)
        x = torch.rand((k, 3), generator=g, dtype=f64, device=device) * L
        if self.plumes > 0:
            centres = torch.from_numpy(self.plume_centres()).to(device)
            in_plume = torch.rand(k, generator=g, dtype=f64, device=device) < self.plume_fraction
            which = torch.randint(0, self.plumes, (k,), generator=g, device=device)
            off = torch.randn((k, 3), generator=g, dtype=f64, device=device) * (self.plume_sigma * L)
            xp = torch.remainder(centres[which] + off, L)
            x = torch.where(in_plume[:, None], xp, x)
            x = torch.where(x >= L, torch.zeros_like(x), x)
        d = torch.exp(torch.randn(k, generator=g, dtype=f64, device=device) * self.d_sigma_ln
                      + math.log(self.d_median))
        up = torch.zeros((k, 3), dtype=f64, device=device)
        return x.contiguous(), up, d

    def n_device_batches(self, batch=1 << 25):
        return (self.P + batch - 1) // batch

    def rotation(self, nsteps=None, first=0):
        """(cos theta_n, sin theta_n) for n = first .. first+nsteps-1, flattened."""
        nsteps = self.nsteps if nsteps is None else nsteps
        th = np.deg2rad(self.rotate_deg * np.arange(first, first + nsteps, dtype=np.float64))
        return np.stack([np.cos(th), np.sin(th)], axis=1).reshape(-1)


def f32_round(a):
    """Round to binary32 and widen back exactly (what an FP32 form stores)."""
    return np.asarray(a, dtype=np.float32).astype(np.float64)


CONFIGS = {
    # 0: plain method, FP64; 32^3, 1e5 droplets, 100 steps of 1e-4 s.
    "tg32": Workload("tg32", n=(32, 32, 32), P=100_000, nsteps=100, dt=1e-4, seed=0),
    # 1: plain method at scale; 128^3 with noise, 1e7 droplets, 50 steps of 5e-5 s.
    "tg128": Workload("tg128", n=(128, 128, 128), P=10_000_000, nsteps=50, dt=5e-5, seed=1,
                      noise=0.1),
    # 2: precision study; 256^3, 2e8 droplets in 4 plumes (sigma 0.05 L), 20 steps.
    "plume256": Workload("plume256", n=(256, 256, 256), P=200_000_000, nsteps=20, dt=5e-5,
                         seed=2, noise=0.1, plumes=4),
    # 3: differentiation; 64^3, 1e6 droplets, 200 steps of 5e-5 s.
    "adj64": Workload("adj64", n=(64, 64, 64), P=1_000_000, nsteps=200, dt=5e-5, seed=3),
    # 4: largest single-GPU case; 512^3, 1.4e9 droplets, 60 % in one plume,
    #    field rotated 1 degree per step on a second stream.
    "plume512": Workload("plume512", n=(512, 512, 512), P=1_400_000_000, nsteps=10, dt=5e-5,
                         seed=4, noise=0.1, plumes=1, plume_fraction=0.6, rotate_deg=1.0),
}
CONFIG_ORDER = ["tg32", "tg128", "plume256", "adj64", "plume512"]


def get(name_or_index):
    if isinstance(name_or_index, int):
        return CONFIGS[CONFIG_ORDER[name_or_index]]
    return CONFIGS[name_or_index]
