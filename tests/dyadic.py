"""A dyadic workload: every quantity of the particle step is a binary
fraction with few significant bits, so every product, quotient and sum the
step takes (paper Sec. 2.1 impulse and momentum source, Sec. 2.5
semi-implicit Euler and deposit into the containing cell) is exact in
binary32 and binary64 alike, and the per-cell sums of the deposited source
are the same in any summation order.

Choices (cell width h = 2^-7 m, dt = 2^-10 s):
  * diameter d = 2^-6 m, particle density 2^10 kg/m^3, viscosity mu with
    fl(18 mu) = 2^8: the response time rho_p d^2 / (18 mu) = 2^-10 s = dt,
    so the implicit drag step halves the slip;
  * parcel weight w with fl(fl(w rho_p) pi) = 6: the parcel mass
    w rho_p pi d^3 / 6 = d^3 = 2^-18 kg;
  * positions on multiples of h/4 (a quarter of them exactly on a face),
    velocities and field values on multiples of 2^-2 m/s, gravity -8 m/s^2;
  * with trilinear interpolation one step is exact (the weights are
    multiples of 2^-6 at the start); with nearest grid point several steps
    are (the gathered value is a field value).
"""
import math

import numpy as np

H = 2.0 ** -7
DT = 2.0 ** -10
D = 2.0 ** -6
RHO_P = 1024.0
G = (0.0, 0.0, -8.0)


def _nudge(v, ok):
    """The double nearest v (within 64 ulp) for which ok(v) holds."""
    for k in range(64):
        for s in (1, -1):
            c = v
            for _ in range(k):
                c = math.nextafter(c, s * math.inf)
            if ok(c):
                return c
    raise ValueError("no exact constant found")


# viscosity with fl(18 mu) == 2^8 and parcel weight with fl(fl(w rho_p) pi) == 6
MU = _nudge(256.0 / 18.0, lambda m: 18.0 * m == 256.0)
W = _nudge(6.0 / (math.pi * RHO_P), lambda w: (w * RHO_P) * math.pi == 6.0)


def mesh_kwargs(n):
    return dict(n=tuple(n), L=tuple(v * H for v in n), rho_f=1.2, mu_f=MU, g=G, rho_p=RHO_P,
                parcel_weight=W)


def case(n, P, seed):
    """(field [3, nz, ny, nx], x [P, 3], up [P, 3], d [P]) on the dyadic grid."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = n
    U = rng.integers(-8, 8, size=(3, nz, ny, nx)).astype(np.float64) * 0.25
    q = rng.integers(0, 4 * np.array(n), size=(P, 3))     # quarter cells
    x = q.astype(np.float64) * (H / 4)
    up = rng.integers(-4, 4, size=(P, 3)).astype(np.float64) * 0.25
    d = np.full(P, D)
    return U, x, up, d
