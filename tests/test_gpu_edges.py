"""GPU edge cases of the step against the FP64 oracle (through the C ABI):
droplets that cross several chunks (and the periodic domain) in one step,
chunks holding exactly one work item's worth of droplets and one more, and a
tracker with no droplets at all (stepped, read back and differentiated).
Tolerances as in the lockstep parity tests.
"""
import numpy as np
import pytest

from gpu_helpers import FORMS, band, fields, lockstep_check, oracle_mesh, state, tracker, workload
from oracle.oracle import load as load_oracle

pytestmark = pytest.mark.gpu

TOL = {
    "fp64": {"pos": 1e-13, "vel": 1e-12, "src": 1e-10},
    "fp32_local": {"pos": 1e-5, "vel": 1e-5, "src": 1e-6},
    "fp32": {"pos": 1e-5, "vel": 1e-5, "src": 1e-4},
}
# (vel is per 1 m/s; the far-mover test scales it by its largest speed)
KSEG = 16384   # droplets per work item of the step kernel


@pytest.fixture(scope="module")
def orc():
    return load_oracle()


@pytest.mark.parametrize("form", FORMS)
def test_lockstep_far_movers(orc, form):
    # 2-cell chunks, a 20 m/s field and initial speeds up to ~100 m/s with
    # dt = 2 ms: most droplets cross several chunks per step, some the whole
    # (periodic) domain
    w = workload("tg32", n=(16, 16, 16), L=(0.1, 0.1, 0.1), P=20000, noise=0.5, U0=20.0,
                 chunk_edge=2)
    x, _, d = w.particles()
    rng = np.random.default_rng(11)
    up = rng.normal(0.0, 10.0, size=x.shape)
    up[:50] *= 10.0
    t = tracker(w, form)
    t.inject(x, up, d)
    Udev, Uor = fields(w, form)
    # velocities of up to a few hundred m/s: their tolerance scales with the
    # largest speed (binary32 keeps about 1e-7 of it per operation)
    vmax = float(np.abs(up).max())
    tol = dict(TOL[form], vel=TOL[form]["vel"] * vmax)
    # FP32 everywhere: a position of up to L + vmax dt carries a binary32
    # rounding of up to 2^-24 of it, which the face band has to cover
    bnd = band(form, w.n)
    if form == "fp32":
        bnd = max(bnd, 2.0 ** -21 * (max(w.L) + vmax * 2e-3) / min(w.h))
    out = lockstep_check(t, orc, oracle_mesh(w), Udev, Uor, 2e-3, 3, tol, band_=bnd)
    print(form, vmax, out, t.stats())
    assert t.stats()["movers"] > w.P // 2
    t.close()


@pytest.mark.parametrize("form", FORMS)
def test_lockstep_item_boundaries(orc, form):
    # 16^3 mesh of 8^3-cell chunks: chunk (0,0,0) holds exactly one work item
    # of droplets, chunk (1,0,0) one more (a second item of one droplet),
    # chunk (0,1,0) a ragged few, the rest none
    w = workload("tg32", n=(16, 16, 16), L=(0.1, 0.1, 0.1), P=2 * KSEG + 8, noise=0.1)
    rng = np.random.default_rng(12)
    ce = 8 * w.L[0] / w.n[0]          # chunk width
    lo = [np.array([0.0, 0.0, 0.0]), np.array([ce, 0.0, 0.0]), np.array([0.0, ce, 0.0])]
    counts = [KSEG, KSEG + 1, 7]
    # keep away from the chunk faces so that no droplet leaves in two short steps
    x = np.concatenate([lo[k] + ce * (0.05 + 0.9 * rng.random((counts[k], 3)))
                        for k in range(3)])
    up = np.zeros_like(x)
    d = np.exp(rng.normal(np.log(20e-6), 0.4, x.shape[0]))
    t = tracker(w, form)
    t.inject(x, up, d)
    Udev, Uor = fields(w, form)
    out = lockstep_check(t, orc, oracle_mesh(w), Udev, Uor, 1e-4, 2, TOL[form],
                         band_=band(form, w.n))
    print(form, out)
    assert t.stats()["items"] == 4 and t.stats()["movers"] == 0
    t.close()


def test_no_droplets():
    import torch
    w = workload("tg32", n=(16, 16, 16), P=0)
    t = tracker(w, "fp32_local", capacity=100)
    Udev, _ = fields(w, "fp32_local")
    for _ in range(3):
        t.step(Udev, 1e-4, tape=2)
    assert t.count() == 0
    s = state(t)
    assert s["x"].shape == (0, 3) and s["id"].shape == (0,)
    assert float(torch.abs(t.sources()).max()) == 0.0
    dU, dd = t.backward(torch.ones(tuple(Udev.shape), dtype=torch.float64, device="cuda"))
    assert dd.shape == (0,) and float(torch.abs(dU).max()) == 0.0
    st = t.stats()
    assert st["particles"] == 0 and st["items"] == 0
    # droplets injected after empty steps step normally
    x, up, d = workload("tg32", n=(16, 16, 16), P=50).particles()
    t.inject(x, up, d)
    t.step(Udev, 1e-4)
    assert t.count() == 50
    t.close()
