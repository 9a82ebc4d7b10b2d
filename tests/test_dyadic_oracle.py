"""The oracle on the dyadic workload (tests/dyadic.py) against exact rational
arithmetic: the impulse m (u_p' - u_p - g dt) of every particle, deposited
with the opposite sign, divided by the cell volume, into the cell that held
it at the start of the step (paper Sec. 2.1 momentum source, Sec. 2.5), and
the semi-implicit Euler update, evaluated with Python fractions.  Every value
is a binary fraction, so the oracle's binary64 result must be exactly equal,
in every cell and for every particle."""
from fractions import Fraction as Fr
import math

import numpy as np

import dyadic
from oracle.oracle import MeshParams, load as load_oracle


def test_dyadic_constants_are_exact():
    orc = load_oracle()
    mesh = MeshParams(**dyadic.mesh_kwargs((16, 16, 16)))
    assert orc.tau(mesh, dyadic.D) == dyadic.DT          # response time 2^-10 s
    assert orc.mass(mesh, dyadic.D) == dyadic.D ** 3     # parcel mass d^3


def test_dyadic_step_equals_exact_arithmetic():
    orc = load_oracle()
    n = (16, 8, 16)
    for interp in (0, 1):
        mesh = MeshParams(interp=interp, **dyadic.mesh_kwargs(n))
        U, x, up, d = dyadic.case(n, 600, seed=5 + interp)
        xo, uo, So = orc.run(mesh, U, x, up, d, dyadic.DT, 1)
        h, dt, tau, m = Fr(dyadic.H), Fr(dyadic.DT), Fr(dyadic.DT), Fr(dyadic.D) ** 3
        V = h ** 3
        g = [Fr(v) for v in dyadic.G]
        S = {}
        for p in range(x.shape[0]):
            X = [Fr(v) for v in x[p]]
            c0 = [math.floor(X[a] / h) % n[a] for a in range(3)]
            if interp == 1:
                uf = [Fr(U[a, c0[2], c0[1], c0[0]]) for a in range(3)]
            else:
                s = [X[a] / h - Fr(1, 2) for a in range(3)]
                i0 = [math.floor(v) for v in s]
                f = [s[a] - i0[a] for a in range(3)]
                uf = [Fr(0)] * 3
                for k in range(8):
                    b = [(k >> a) & 1 for a in range(3)]
                    w = Fr(1)
                    for a in range(3):
                        w *= f[a] if b[a] else 1 - f[a]
                    c = [(i0[a] + b[a]) % n[a] for a in range(3)]
                    uf = [uf[a] + w * Fr(U[a, c[2], c[1], c[0]]) for a in range(3)]
            Up = [Fr(v) for v in up[p]]
            un = [(tau * Up[a] + dt * uf[a] + tau * dt * g[a]) / (tau + dt) for a in range(3)]
            J = [m * (un[a] - Up[a] - g[a] * dt) for a in range(3)]
            for a in range(3):
                key = (a, c0[2], c0[1], c0[0])
                S[key] = S.get(key, Fr(0)) - J[a] / V
            L = [h * n[a] for a in range(3)]
            Xn = [X[a] + dt * un[a] for a in range(3)]
            Xn = [v - L[a] if v >= L[a] else (v + L[a] if v < 0 else v) for a, v in enumerate(Xn)]
            assert [Fr(v) for v in xo[p]] == Xn, f"position of particle {p}"
            assert [Fr(v) for v in uo[p]] == un, f"velocity of particle {p}"
        want = np.zeros_like(So)
        for key, v in S.items():
            want[key] = float(v)
            assert Fr(want[key]) == v, "exact sums are binary fractions"
        assert np.array_equal(So, want), f"per-cell sources, interp {interp}"
        assert np.count_nonzero(So) > 100
