"""Plant plausible mistakes in copies of the oracle; each must fail a pin.

Every mutant below is one textual change to oracle/st_oracle.c (a dropped
term, a wrong sign or index, a transposed operand).  The copy is compiled
with gcc into a temporary directory and the pins run in a child process, so
a mutant that indexes out of bounds cannot take the test run down.
"""
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(ROOT, "oracle", "st_oracle.c")

MUTANTS = {
    "gravity dropped from the velocity update":
        ("+ tau * dt * m->g[a]) / (tau + dt)", ") / (tau + dt)"),
    "gravity sign in the velocity update":
        ("+ tau * dt * m->g[a]) / (tau + dt)", "- tau * dt * m->g[a]) / (tau + dt)"),
    "position advanced with the old velocity":
        ("x[a] = x[a] + dt * up_new[a];", "x[a] = x[a] + dt * up[a];"),
    "response time factor 9 instead of 18":
        ("(18.0 * m->mu_f)", "(9.0 * m->mu_f)"),
    "response time with rho_f":
        ("return m->rho_p * d * d / (18.0", "return m->rho_f * d * d / (18.0"),
    "impulse without the gravity term":
        ("J[a] = mass * (up_new[a] - up[a] - m->g[a] * dt);",
         "J[a] = mass * (up_new[a] - up[a]);"),
    "deposit sign":
        ("-= J[a] / V;", "+= J[a] / V;"),
    "deposit into the end-of-step cell":
        ("    int32_t c0[3];\n    or_cell(m, x, c0);\n    double ufp[3];",
         "    int32_t c0[3];\n    { double xe[3]; for (int q = 0; q < 3; ++q) xe[q] = x[q] + dt * up[q];"
         " or_wrap(m, xe); or_cell(m, xe, c0); }\n    double ufp[3];"),
    "no half-cell shift to the cell centres":
        ("double s = x[a] / h - 0.5;", "double s = x[a] / h;"),
    "trilinear weights swapped":
        ("om[a][0] = 1.0 - f;\n        om[a][1] = f;", "om[a][0] = f;\n        om[a][1] = 1.0 - f;"),
    "field layout x and z transposed":
        ("((c * (int64_t)m->n[2] + k) * m->n[1] + j) * m->n[0] + i",
         "((c * (int64_t)m->n[2] + i) * m->n[1] + j) * m->n[0] + k"),
    "no wrap at the upper boundary":
        ("if (x[a] >= m->L[a]) x[a] -= m->L[a];", ""),
    "cell by rounding instead of floor":
        ("double q = floor(x[a] / width(m, a));", "double q = round(x[a] / width(m, a));"),
    "cell width of the wrong axis":
        ("double q = floor(x[a] / width(m, a));", "double q = floor(x[a] / width(m, 0));"),
    "mass with d^2":
        ("OR_PI * d * d * d / 6.0", "OR_PI * d * d / 6.0"),
    "cell volume from one axis":
        ("return width(m, 0) * width(m, 1) * width(m, 2);",
         "return width(m, 0) * width(m, 0) * width(m, 0);"),
    "negative index wrap off by one":
        ("return r < 0 ? r + n : r;", "return r < 0 ? r + n - 1 : r;"),
    "sub-step length not divided":
        ("double dts = dt / nsub;", "double dts = dt;"),
    "rotation sign":
        ("Un[q] = c * ux - s * uy;", "Un[q] = c * ux + s * uy;"),
    "adjoint: position term dropped from the velocity cotangent":
        ("wbar[a] = ubar[a] + dt * xbar[a] + mass * Jbar[a];",
         "wbar[a] = ubar[a] + mass * Jbar[a];"),
    "adjoint: interpolation-gradient term dropped":
        ("for (int a = 0; a < 3; ++a) xbar[a] += st.dw[k8][a] * dot;", ";"),
    "adjoint: response-time cotangent sign":
        ("taubar += wbar[a] * (up[a] + dt * m->g[a] - up_new[a]) / D;",
         "taubar -= wbar[a] * (up[a] + dt * m->g[a] - up_new[a]) / D;"),
    "adjoint: mass cotangent dropped":
        ("mbar += Jbar[a] * (up_new[a] - up[a] - m->g[a] * dt);", ";"),
    "adjoint: field cotangent scaled by tau":
        ("ufbar[a] = dt / D * wbar[a];", "ufbar[a] = tau / D * wbar[a];"),
    "adjoint: impulse term sign in the old-velocity cotangent":
        ("ubar[a] = -mass * Jbar[a] + tau / D * wbar[a];",
         "ubar[a] = mass * Jbar[a] + tau / D * wbar[a];"),
    "adjoint: deposit transpose sign":
        ("Jbar[a] = -lambda[", "Jbar[a] = lambda["),
    "adjoint: lower-corner weight gradient sign":
        ("dom[a][0] = -1.0 / h;", "dom[a][0] = 1.0 / h;"),
    "adjoint: dm/dd factor":
        ("mbar * 3.0 * mass / d[p]", "mbar * 2.0 * mass / d[p]"),
    "adjoint: dtau/dd factor":
        ("tausbar * 2.0 * tau_s / d[p]", "tausbar * tau_s / d[p]"),
    "adjoint: sub-step length not divided":
        ("double dt = dt_of_step[n] / nsub;", "double dt = dt_of_step[n];"),
    "adjoint: every sub-step reversed from the state at its step's start":
        ("const double *x = xs + per * k + 3 * p;",
         "const double *x = xs + per * (k - k % nsub) + 3 * p;"),
    "adjoint: every step read with the first step's field":
        ("const double *Uf = fields + (size_t)field_of_step[n] * 3 * nc;\n            double *Ub",
         "const double *Uf = fields;\n            double *Ub"),
    "adjoint: every field's gradient added to the first field":
        ("double *Ub = Ubar + (size_t)field_of_step[n] * 3 * nc;", "double *Ub = Ubar;"),
    "adjoint: trilinear stencil in the reverse of nearest-grid-point steps":
        ("            stencil st;\n            make_stencil(m, x, &st);\n            double ufp[3], up_new[3];",
         "            stencil st;\n            { or_mesh tm = *m; tm.interp = 0; make_stencil(&tm, x, &st); }\n"
         "            double ufp[3], up_new[3];"),
    "Schiller-Naumann exponent":
        ("0.15 * pow(slip_reynolds(m, d, slip), 0.687)", "0.15 * pow(slip_reynolds(m, d, slip), 0.786)"),
    "Schiller-Naumann coefficient":
        ("1.0 + 0.15 * pow(", "1.0 + 0.015 * pow("),
    "Schiller-Naumann Reynolds number with the radius":
        ("m->rho_f * s * d / m->mu_f", "m->rho_f * s * 0.5 * d / m->mu_f"),
    "Schiller-Naumann Reynolds number without the fluid density":
        ("m->rho_f * s * d / m->mu_f", "s * d / m->mu_f"),
    "Schiller-Naumann Reynolds number from one slip component":
        ("double s = sqrt(slip[0] * slip[0] + slip[1] * slip[1] + slip[2] * slip[2]);",
         "double s = fabs(slip[0]);"),
    "Schiller-Naumann factor multiplies the response time":
        ("double tau = or_tau(m, d) / or_drag_factor(m, d, slip);",
         "double tau = or_tau(m, d) * or_drag_factor(m, d, slip);"),
    "Schiller-Naumann slip from the particle velocity alone":
        ("double slip[3] = {ufp[0] - up[0], ufp[1] - up[1], ufp[2] - up[2]};",
         "double slip[3] = {-up[0], -up[1], -up[2]};"),
    "adjoint: Schiller-Naumann slip cotangent sign":
        ("ufbar[a] += sbar;", "ufbar[a] -= sbar;"),
    "adjoint: Schiller-Naumann diameter term dropped":
        ("if (Re > 0.0) db += Rebar * Re / d[p];", ";"),
    "adjoint: Schiller-Naumann factor left out of the Stokes cotangent":
        ("double tausbar = taubar / f;", "double tausbar = taubar;"),
    "adjoint: Schiller-Naumann derivative exponent":
        ("pow(Re, 0.687 - 1.0)", "pow(Re, 0.687)"),
    "Hilbert: invert and exchange swapped":
        ("if (X[i] & Q) {\n                X[0] ^= P;", "if (!(X[i] & Q)) {\n                X[0] ^= P;"),
    "Hilbert: Gray encoding from the wrong neighbour":
        ("for (int i = 1; i < 3; ++i) X[i] ^= X[i - 1];", "for (int i = 1; i < 3; ++i) X[i - 1] ^= X[i];"),
    "Hilbert: correction mask from x instead of z":
        ("if (X[2] & Q) t ^= Q - 1;", "if (X[0] & Q) t ^= Q - 1;"),
    "Hilbert: axes interleaved z first":
        ("h = (h << 1) | (int64_t)((X[i] >> level) & 1u);", "h = (h << 1) | (int64_t)((X[2 - i] >> level) & 1u);"),
    "Hilbert: undo loop stops one level early":
        ("for (uint32_t Q = M; Q > 1; Q >>= 1) {\n        const uint32_t P = Q - 1;",
         "for (uint32_t Q = M; Q > 2; Q >>= 1) {\n        const uint32_t P = Q - 1;"),
    "segments: voxel of a particle by modulo":
        ("const int64_t v = v0 + k * nv / per_seg;", "const int64_t v = v0 + k % nv;"),
    "segments: start rounded up":
        ("const int64_t v0 = sg * V / nseg, v1", "const int64_t v0 = (sg * V + nseg - 1) / nseg, v1"),
    "segments: voxel width from side - 1":
        ("* (L[a] / (double)side);", "* (L[a] / (double)(side - 1));"),
    "bounding boxes: partition off by one":
        ("const int64_t p = (id[q] - id0) / per_part;", "const int64_t p = (id[q] - id0 + 1) / per_part;"),
    "bounding boxes: min and max swapped":
        ("if (x[3 * q + a] < box[6 * p + a]) box[6 * p + a] = x[3 * q + a];",
         "if (x[3 * q + a] > box[6 * p + a]) box[6 * p + a] = x[3 * q + a];"),
    "extrapolator-corrector: corrector sign":
        ("double correction = S_last[i] - ext_prev[i];", "double correction = S_last[i] + ext_prev[i];"),
    "extrapolator-corrector: linear coefficients swapped":
        ("2.0 * S_last[i] - S_prev2[i]", "2.0 * S_prev2[i] - S_last[i]"),
    "extrapolator-corrector: history not advanced":
        ("S_prev2[i] = S_last[i];", ";"),
    "extrapolator-corrector: extrapolation not remembered":
        ("ext_prev[i] = extrapolation;", ";"),
    "extrapolator-corrector: constant extrapolator uses the older source":
        ("if (kind == 1) extrapolation = S_last[i];", "if (kind == 1) extrapolation = S_prev2[i];"),
}


def _build_and_pin(name, old, new, tmp):
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation site not found for {name!r}"
    mutated = src.replace(old, new, 1)
    tag = str(abs(hash(name)))
    csrc = os.path.join(tmp, f"m{tag}.c")
    lib = os.path.join(tmp, f"m{tag}.so")
    with open(csrc, "w") as f:
        f.write(mutated)
    subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
                    "-fopenmp", csrc, os.path.join(ROOT, "oracle", "st_oracle_par.c"),
                    "-I", tmp, "-o", lib, "-lm"], check=True, capture_output=True)
    r = subprocess.run([sys.executable, os.path.join(HERE, "oracle_pins.py"), lib],
                       capture_output=True, text=True, timeout=120)
    out = r.stdout.strip().splitlines()[-1] if r.stdout.strip() else ""
    return name, r.returncode, out


def _tmpdir_with_header(tmp):
    shutil.copy(os.path.join(ROOT, "oracle", "st_oracle.h"), tmp)
    return tmp


def test_every_mutant_fails_a_pin():
    with tempfile.TemporaryDirectory() as tmp:
        _tmpdir_with_header(tmp)
        with cf.ThreadPoolExecutor(max_workers=6) as ex:
            futs = [ex.submit(_build_and_pin, k, o, n, tmp) for k, (o, n) in MUTANTS.items()]
            results = [f.result() for f in futs]
    survivors = []
    for name, rc, out in results:
        # a crash (nonzero return) also counts as caught
        if rc == 0 and out == "ALL_PASSED":
            survivors.append(name)
    assert not survivors, f"mutants not caught by any pin: {survivors}"


def test_unmutated_copy_passes():
    with tempfile.TemporaryDirectory() as tmp:
        _tmpdir_with_header(tmp)
        name, rc, out = _build_and_pin("identity", "st_oracle.h", "st_oracle.h", tmp)
    assert rc == 0 and out == "ALL_PASSED", out
