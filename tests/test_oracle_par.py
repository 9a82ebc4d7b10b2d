"""The oracle's particle-parallel drivers against the serial oracle: particle
states and per-particle gradients bitwise equal, per-cell sums equal up to
the order of their additions."""
import math

import numpy as np

from oracle.oracle import MeshParams, load as load_oracle


def _case(seed, P=3000, n=(16, 8, 12)):
    rng = np.random.default_rng(seed)
    mesh = MeshParams(n=n, L=(0.02, 0.01, 0.015), drag=1)
    U = rng.normal(0.0, 0.5, size=mesh.field_shape)
    x = rng.random((P, 3)) * np.array(mesh.L)
    up = rng.normal(0.0, 0.2, size=(P, 3))
    d = np.exp(rng.normal(math.log(40e-6), 0.4, size=P))
    return mesh, U, x, up, d


def test_run_par_equals_serial():
    orc = load_oracle()
    mesh, U, x, up, d = _case(1)
    xs, us, Ss = orc.run(mesh, U, x, up, d, 1e-4, 5, nsub=2)
    for threads in (1, 3, 8):
        xp, upp, Sp = orc.run_par(mesh, U, x, up, d, 1e-4, 5, nsub=2, threads=threads)
        assert np.array_equal(xp, xs) and np.array_equal(upp, us)
        assert np.abs(Sp - Ss).max() <= 1e-13 * np.abs(Ss).max()


def test_adjoint_run_par_equals_serial():
    orc = load_oracle()
    mesh, U, x, up, d = _case(2, P=800)
    rng = np.random.default_rng(3)
    F = np.stack([U, U + rng.normal(0.0, 0.2, size=U.shape)])
    fs, dts = [0, 1, 1, 0], [1e-4, 2e-4, 1e-4, 1.5e-4]
    lam = rng.normal(size=mesh.field_shape)
    Us, ds = orc.adjoint_run(mesh, F, fs, dts, 2, x, up, d, lam)
    for threads in (1, 5):
        Up, dp = orc.adjoint_run_par(mesh, F, fs, dts, 2, x, up, d, lam, threads=threads)
        assert np.array_equal(dp, ds)
        assert np.abs(Up - Us).max() <= 1e-13 * np.abs(Us).max()
