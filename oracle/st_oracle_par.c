/*
 * Particle-parallel drivers of the FP64 CPU oracle.  TEST INFRASTRUCTURE
 * ONLY (the tests, the smoke check and the CPU-baseline leg of the benchmark
 * load it; the product library never does).
 *
 * Particles do not interact given the fluid field (the paper's droplets do
 * not collide), so a run over np particles is the same as runs over any
 * partition of them, except for the order in which their deposits are
 * summed per cell.  Each driver splits the particles into nthreads
 * contiguous ranges, runs the serial oracle (st_oracle.c) on every range
 * with a private source or gradient array, and adds the private arrays in
 * range order.  No arithmetic of the method lives here: particle states and
 * per-particle gradients are bitwise those of the serial oracle, per-cell
 * sums differ from it only by the order of the additions.
 */
#include "st_oracle.h"

#include <omp.h>
#include <stdlib.h>
#include <string.h>

static int64_t cells_of(const or_mesh *m) { return (int64_t)m->n[0] * m->n[1] * m->n[2]; }

/* out += sum over t of part[t] (in t order), each of n values */
static void add_parts(double *out, const double *part, int nt, int64_t n)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double s = out[i];
        for (int t = 0; t < nt; ++t) s += part[(size_t)t * n + i];
        out[i] = s;
    }
}

int or_run_par(const or_mesh *m, const double *Uf, int64_t np, double *x, double *up,
               const double *d, double dt, int32_t nsteps, int32_t nsub, double *Su_int,
               int32_t nthreads)
{
    if (nthreads < 1 || np < 0) return -1;
    const int64_t n3 = 3 * cells_of(m);
    double *part = (double *)calloc((size_t)nthreads * (size_t)n3, sizeof(double));
    if (!part) return -1;
#pragma omp parallel for num_threads(nthreads) schedule(static, 1)
    for (int t = 0; t < nthreads; ++t) {
        const int64_t p0 = np * t / nthreads, p1 = np * (t + 1) / nthreads;
        or_run(m, Uf, p1 - p0, x + 3 * p0, up + 3 * p0, d + p0, dt, nsteps, nsub,
               part + (size_t)t * n3);
    }
    add_parts(Su_int, part, nthreads, n3);
    free(part);
    return 0;
}

int or_adjoint_run_par(const or_mesh *m, int32_t nfields, const double *fields,
                       int32_t nsteps, const int32_t *field_of_step, const double *dt_of_step,
                       int32_t nsub, int64_t np, const double *x0, const double *up0,
                       const double *d, const double *lambda, double *Ubar, double *dbar,
                       int32_t nthreads)
{
    if (nthreads < 1 || nfields < 1 || np < 0) return -1;
    const int64_t n3 = (int64_t)nfields * 3 * cells_of(m);
    double *part = (double *)calloc((size_t)nthreads * (size_t)n3, sizeof(double));
    if (!part) return -1;
    int bad = 0;
#pragma omp parallel for num_threads(nthreads) schedule(static, 1) reduction(| : bad)
    for (int t = 0; t < nthreads; ++t) {
        const int64_t p0 = np * t / nthreads, p1 = np * (t + 1) / nthreads;
        if (or_adjoint_run(m, nfields, fields, nsteps, field_of_step, dt_of_step, nsub,
                           p1 - p0, x0 + 3 * p0, up0 + 3 * p0, d + p0, lambda,
                           part + (size_t)t * n3, dbar + p0) != 0)
            bad |= 1;
    }
    if (!bad) add_parts(Ubar, part, nthreads, n3);
    free(part);
    return bad ? -1 : 0;
}
