"""Bit-exact deposit on the dyadic workload (tests/dyadic.py), in all three
forms: every impulse and every partial sum is a binary fraction that binary32
holds exactly, so the per-cell sources the GPU deposits (paper Sec. 2.1
momentum source, Sec. 2.5 deposit into the containing cell) must equal the
oracle's bit for bit, whatever order the LDS and global atomics add them in;
so must positions, velocities and cells.  Sparse chunks (one work item each)
and crowded ones (several work items, whose sums meet in global atomics),
chunk edges 8 and 4, trilinear over one step and nearest grid point over
three (particles crossing chunks in between)."""
import numpy as np
import pytest

import dyadic
from oracle.oracle import MeshParams, load as load_oracle

pytestmark = pytest.mark.gpu

CASES = [
    # mesh, particles, chunk edge, interpolation, steps
    ((32, 32, 32), 60_000, 8, "trilinear", 1),
    ((32, 32, 32), 60_000, 8, "ngp", 3),
    ((16, 16, 16), 200_000, 8, "trilinear", 1),   # 25 000 per chunk: several work items
    ((16, 16, 16), 200_000, 8, "ngp", 3),
    ((16, 8, 24), 30_000, 4, "trilinear", 1),
    ((16, 8, 24), 30_000, 4, "ngp", 3),
]


@pytest.mark.parametrize("form", ["fp64", "fp32_local", "fp32"])
@pytest.mark.parametrize("n,P,E,interp,nsteps", CASES)
def test_dyadic_deposit_bit_exact(form, n, P, E, interp, nsteps):
    import torch
    import paper_2603_26691_amd as pkg
    kw = dyadic.mesh_kwargs(n)
    U, x, up, d = dyadic.case(n, P, seed=sum(n) + P + E)
    t = pkg.Tracker(n, kw["L"], P, form=form, interp=interp, chunk_edge=E, rho_f=kw["rho_f"],
                    mu_f=kw["mu_f"], g=kw["g"], rho_p=kw["rho_p"],
                    parcel_weight=kw["parcel_weight"])
    t.inject(x, up, d)
    Udev = torch.from_numpy(U if form == "fp64" else U.astype(np.float32)).cuda()
    for _ in range(nsteps):
        t.step(Udev, dyadic.DT)
    S = t.sources().cpu().numpy()
    s = {k: v.cpu().numpy() for k, v in t.particles().items()}
    movers = t.stats()["movers"]
    t.close()
    orc = load_oracle()
    mesh = MeshParams(interp=1 if interp == "ngp" else 0, **kw)
    xo, uo, So = orc.run(mesh, U, x, up, d, dyadic.DT, nsteps)
    assert np.array_equal(S, So), \
        f"{np.count_nonzero(S != So)} cells differ, largest {np.abs(S - So).max()}"
    assert np.array_equal(s["x"], xo) and np.array_equal(s["up"], uo)
    assert np.array_equal(s["cell"], orc.cells(mesh, xo))
    assert np.array_equal(s["id"], np.arange(P))
    assert np.count_nonzero(So) > 1000
    if nsteps > 1:
        assert movers > 0, "particles crossed chunks"
