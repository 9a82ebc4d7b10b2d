/*
 * Plain FP64 CPU oracle for the per-particle Lagrangian time step of
 * SCALE-TRACK (arXiv 2603.26691).  TEST INFRASTRUCTURE ONLY: only the test
 * suite, the smoke check and the CPU-baseline leg of the benchmark may load
 * it; the product library never does.  It shares no code with the HIP
 * implementation.  See st_oracle.h for the definitions it follows.
 *
 * Written for a reader checking it against the paper by eye: one particle
 * at a time, in id order, no blocking, no reordering, no fusion.
 */
#include "st_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

static const double OR_PI = 3.14159265358979323846;

static double width(const or_mesh *m, int a) { return m->L[a] / m->n[a]; }

static double cell_volume(const or_mesh *m)
{
    return width(m, 0) * width(m, 1) * width(m, 2);
}

static int64_t n_cells(const or_mesh *m)
{
    return (int64_t)m->n[0] * m->n[1] * m->n[2];
}

/* Euclidean remainder: the periodic image of index i on an axis of n cells. */
static int64_t wrap_index(int64_t i, int64_t n)
{
    int64_t r = i % n;
    return r < 0 ? r + n : r;
}

/* Flat index of cell (i, j, k), component c, in a [3][n2][n1][n0] field. */
static int64_t field_index(const or_mesh *m, int c, int64_t i, int64_t j,
                           int64_t k)
{
    return ((c * (int64_t)m->n[2] + k) * m->n[1] + j) * m->n[0] + i;
}

void or_cell(const or_mesh *m, const double x[3], int32_t c[3])
{
    /* The particle's cell is the one whose half-open interval
     * [i h, (i+1) h) holds it; a point on a face belongs to the upper cell. */
    for (int a = 0; a < 3; ++a) {
        double q = floor(x[a] / width(m, a));
        c[a] = (int32_t)wrap_index((int64_t)q, m->n[a]);
    }
}

void or_cells(const or_mesh *m, int64_t np, const double *x, int32_t *c)
{
    for (int64_t p = 0; p < np; ++p) or_cell(m, x + 3 * p, c + 3 * p);
}

void or_wrap(const or_mesh *m, double x[3])
{
    for (int a = 0; a < 3; ++a) {
        if (x[a] >= m->L[a]) x[a] -= m->L[a];
        if (x[a] < 0.0) x[a] += m->L[a];
        if (x[a] == m->L[a]) x[a] = 0.0;
    }
}

double or_tau(const or_mesh *m, double d)
{
    /* Stokes response time of a sphere. */
    return m->rho_p * d * d / (18.0 * m->mu_f);
}

double or_mass(const or_mesh *m, double d)
{
    /* Mass of a parcel of spheres of diameter d. */
    return m->parcel_weight * m->rho_p * OR_PI * d * d * d / 6.0;
}

static double slip_reynolds(const or_mesh *m, double d, const double slip[3])
{
    double s = sqrt(slip[0] * slip[0] + slip[1] * slip[1] + slip[2] * slip[2]);
    return m->rho_f * s * d / m->mu_f;
}

double or_drag_factor(const or_mesh *m, double d, const double slip[3])
{
    if (m->drag != 1) return 1.0;
    return 1.0 + 0.15 * pow(slip_reynolds(m, d, slip), 0.687);
}

/*
 * Interpolation stencil at position x: 8 corner cells (x-index fastest in
 * the corner number), their weights and the weights' gradient with respect
 * to x.  Trilinear: the cell centres sit at (i + 1/2) h; with
 * s = x/h - 1/2, i0 = floor(s), f = s - i0 the corner weights along one
 * axis are (1 - f) for i0 and f for i0 + 1.  Nearest grid point: the
 * containing cell with weight 1 (the other 7 weights are 0).
 */
typedef struct {
    int64_t cell[8][3];
    double w[8];
    double dw[8][3];
} stencil;

static void make_stencil(const or_mesh *m, const double x[3], stencil *st)
{
    if (m->interp == 1) {
        int32_t c[3];
        or_cell(m, x, c);
        memset(st, 0, sizeof *st);
        for (int k = 0; k < 8; ++k)
            for (int a = 0; a < 3; ++a) st->cell[k][a] = c[a];
        st->w[0] = 1.0;
        return;
    }
    int64_t i0[3];
    double om[3][2], dom[3][2];
    for (int a = 0; a < 3; ++a) {
        double h = width(m, a);
        double s = x[a] / h - 0.5;
        double fl = floor(s);
        double f = s - fl;
        i0[a] = (int64_t)fl;
        om[a][0] = 1.0 - f;
        om[a][1] = f;
        dom[a][0] = -1.0 / h;
        dom[a][1] = 1.0 / h;
    }
    for (int k = 0; k < 8; ++k) {
        int b[3] = {k & 1, (k >> 1) & 1, (k >> 2) & 1};
        for (int a = 0; a < 3; ++a)
            st->cell[k][a] = wrap_index(i0[a] + b[a], m->n[a]);
        st->w[k] = om[0][b[0]] * om[1][b[1]] * om[2][b[2]];
        st->dw[k][0] = dom[0][b[0]] * om[1][b[1]] * om[2][b[2]];
        st->dw[k][1] = om[0][b[0]] * dom[1][b[1]] * om[2][b[2]];
        st->dw[k][2] = om[0][b[0]] * om[1][b[1]] * dom[2][b[2]];
    }
}

void or_interp(const or_mesh *m, const double *Uf, const double x[3],
               double uf_at_p[3])
{
    stencil st;
    make_stencil(m, x, &st);
    for (int c = 0; c < 3; ++c) {
        double acc = 0.0;
        for (int k = 0; k < 8; ++k)
            acc += st.w[k] * Uf[field_index(m, c, st.cell[k][0],
                                            st.cell[k][1], st.cell[k][2])];
        uf_at_p[c] = acc;
    }
}

void or_interp_many(const or_mesh *m, const double *Uf, int64_t np,
                    const double *x, double *uf_at_p)
{
    for (int64_t p = 0; p < np; ++p)
        or_interp(m, Uf, x + 3 * p, uf_at_p + 3 * p);
}

void or_interp_transpose(const or_mesh *m, const double x[3],
                         const double a[3], double *Ubar)
{
    stencil st;
    make_stencil(m, x, &st);
    for (int c = 0; c < 3; ++c)
        for (int k = 0; k < 8; ++k)
            Ubar[field_index(m, c, st.cell[k][0], st.cell[k][1],
                             st.cell[k][2])] += st.w[k] * a[c];
}

/*
 * One sub-step of one particle.  Semi-implicit Euler for
 * m du_p/dt = m (u_f - u_p)/tau + m g:
 *     u_p' = (tau u_p + dt u_f + tau dt g) / (tau + dt)
 *     x'   = x + dt u_p'            (wrapped periodically)
 *     J    = m (u_p' - u_p - g dt)  (drag impulse on the particle)
 * and the fluid receives -J in the cell that held the particle at the start
 * of the sub-step: Su_int[c0] -= J / V_cell.
 */
static void particle_substep(const or_mesh *m, const double *Uf, double x[3],
                             double up[3], double d, double dt,
                             double *Su_int)
{
    int32_t c0[3];
    or_cell(m, x, c0);
    double ufp[3];
    or_interp(m, Uf, x, ufp);
    double slip[3] = {ufp[0] - up[0], ufp[1] - up[1], ufp[2] - up[2]};
    double tau = or_tau(m, d) / or_drag_factor(m, d, slip);
    double mass = or_mass(m, d);
    double V = cell_volume(m);
    double up_new[3], J[3];
    for (int a = 0; a < 3; ++a) {
        up_new[a] = (tau * up[a] + dt * ufp[a] + tau * dt * m->g[a]) / (tau + dt);
        J[a] = mass * (up_new[a] - up[a] - m->g[a] * dt);
    }
    for (int a = 0; a < 3; ++a) {
        x[a] = x[a] + dt * up_new[a];
        up[a] = up_new[a];
        Su_int[field_index(m, a, c0[0], c0[1], c0[2])] -= J[a] / V;
    }
    or_wrap(m, x);
}

void or_step(const or_mesh *m, const double *Uf, int64_t np, double *x,
             double *up, const double *d, double dt, int32_t nsub,
             double *Su_int)
{
    double dts = dt / nsub;
    for (int32_t s = 0; s < nsub; ++s)
        for (int64_t p = 0; p < np; ++p)
            particle_substep(m, Uf, x + 3 * p, up + 3 * p, d[p], dts, Su_int);
}

void or_run(const or_mesh *m, const double *Uf, int64_t np, double *x,
            double *up, const double *d, double dt, int32_t nsteps,
            int32_t nsub, double *Su_int)
{
    for (int32_t n = 0; n < nsteps; ++n)
        or_step(m, Uf, np, x, up, d, dt, nsub, Su_int);
}

void or_run_rotating(const or_mesh *m, const double *U0, const double *cs,
                     int64_t np, double *x, double *up, const double *d,
                     double dt, int32_t nsteps, double *Su_int)
{
    int64_t nc = n_cells(m);
    double *Un = (double *)malloc(sizeof(double) * 3 * nc);
    if (!Un) return;
    for (int32_t n = 0; n < nsteps; ++n) {
        double c = cs[2 * n], s = cs[2 * n + 1];
        /* Rotation of the velocity vector about the z axis. */
        for (int64_t q = 0; q < nc; ++q) {
            double ux = U0[q], uy = U0[nc + q], uz = U0[2 * nc + q];
            Un[q] = c * ux - s * uy;
            Un[nc + q] = s * ux + c * uy;
            Un[2 * nc + q] = uz;
        }
        or_step(m, Un, np, x, up, d, dt, 1, Su_int);
    }
    free(Un);
}

void or_ec_estimate(int64_t n, int32_t kind, const double *S_last, double *S_prev2,
                    double *ext_prev, double *applied)
{
    for (int64_t i = 0; i < n; ++i) {
        double correction = S_last[i] - ext_prev[i];
        double extrapolation = 0.0;
        if (kind == 1) extrapolation = S_last[i];
        if (kind == 2) extrapolation = 2.0 * S_last[i] - S_prev2[i];
        applied[i] = correction + extrapolation;
        ext_prev[i] = extrapolation;
        S_prev2[i] = S_last[i];
    }
}

int or_adjoint_run(const or_mesh *m, int32_t nfields, const double *fields,
                   int32_t nsteps, const int32_t *field_of_step,
                   const double *dt_of_step, int32_t nsub, int64_t np,
                   const double *x0, const double *up0, const double *d,
                   const double *lambda, double *Ubar, double *dbar)
{
    if (nfields < 1 || nsteps < 0 || nsub < 1 || np < 0) return -1;
    for (int32_t n = 0; n < nsteps; ++n)
        if (field_of_step[n] < 0 || field_of_step[n] >= nfields || !(dt_of_step[n] > 0.0))
            return -1;
    int64_t nc = n_cells(m);
    /* Forward pass, keeping the state at the start of every sub-step: the
     * step n is nsub sub-steps of dt_n / nsub with its field held fixed. */
    int64_t nss = (int64_t)nsteps * nsub;
    size_t per = (size_t)np * 3;
    double *xs = (double *)malloc(sizeof(double) * per * (size_t)(nss + 1));
    double *us = (double *)malloc(sizeof(double) * per * (size_t)(nss + 1));
    double *scratch = (double *)calloc((size_t)3 * nc, sizeof(double));
    if (!xs || !us || !scratch) {
        free(xs); free(us); free(scratch);
        return -1;
    }
    memcpy(xs, x0, sizeof(double) * per);
    memcpy(us, up0, sizeof(double) * per);
    for (int64_t k = 0; k < nss; ++k) {
        int32_t n = (int32_t)(k / nsub);
        const double *Uf = fields + (size_t)field_of_step[n] * 3 * nc;
        double dts = dt_of_step[n] / nsub;
        memcpy(xs + per * (k + 1), xs + per * k, sizeof(double) * per);
        memcpy(us + per * (k + 1), us + per * k, sizeof(double) * per);
        or_step(m, Uf, np, xs + per * (k + 1), us + per * (k + 1), d, dts, 1,
                scratch);
    }

    double V = cell_volume(m);
    for (int64_t p = 0; p < np; ++p) {
        double xbar[3] = {0, 0, 0}, ubar[3] = {0, 0, 0}, db = 0.0;
        double tau_s = or_tau(m, d[p]);
        double mass = or_mass(m, d[p]);
        /* Sub-steps newest first; each reads the field of its step and adds
         * that field's gradient. */
        for (int64_t k = nss - 1; k >= 0; --k) {
            int32_t n = (int32_t)(k / nsub);
            const double *Uf = fields + (size_t)field_of_step[n] * 3 * nc;
            double *Ub = Ubar + (size_t)field_of_step[n] * 3 * nc;
            double dt = dt_of_step[n] / nsub;
            const double *x = xs + per * k + 3 * p;
            const double *up = us + per * k + 3 * p;
            /* Recompute the forward quantities of this sub-step. */
            int32_t c0[3];
            or_cell(m, x, c0);
            stencil st;
            make_stencil(m, x, &st);
            double ufp[3], up_new[3];
            or_interp(m, Uf, x, ufp);
            double slip[3] = {ufp[0] - up[0], ufp[1] - up[1], ufp[2] - up[2]};
            double f = or_drag_factor(m, d[p], slip);
            double tau = tau_s / f;
            double D = tau + dt;
            for (int a = 0; a < 3; ++a)
                up_new[a] = (tau * up[a] + dt * ufp[a] + tau * dt * m->g[a]) / D;

            /* Deposit: Su_int[c0] -= J/V, so Jbar = -lambda[c0] / V. */
            double Jbar[3], wbar[3], ufbar[3];
            double mbar = 0.0, taubar = 0.0;
            for (int a = 0; a < 3; ++a)
                Jbar[a] = -lambda[field_index(m, a, c0[0], c0[1], c0[2])] / V;
            for (int a = 0; a < 3; ++a) {
                /* Everything that reads u_p': the next state's velocity, the
                 * position update x' = x + dt u_p' and the impulse. */
                wbar[a] = ubar[a] + dt * xbar[a] + mass * Jbar[a];
                mbar += Jbar[a] * (up_new[a] - up[a] - m->g[a] * dt);
                ufbar[a] = dt / D * wbar[a];
                taubar += wbar[a] * (up[a] + dt * m->g[a] - up_new[a]) / D;
                ubar[a] = -mass * Jbar[a] + tau / D * wbar[a];
            }
            /* tau = tau_s / f: the Stokes part and, for Schiller-Naumann, the
             * drag factor f = 1 + 0.15 Re^0.687 with Re = rho_f |s| d / mu_f
             * of the slip s = u_f - u_p (dRe/ds = Re s / |s|^2, dRe/dd = Re/d;
             * at zero slip the derivative is taken as zero). */
            double tausbar = taubar / f;
            double Rebar = 0.0, Re = 0.0;
            if (m->drag == 1) {
                double s2 = slip[0] * slip[0] + slip[1] * slip[1] + slip[2] * slip[2];
                Re = slip_reynolds(m, d[p], slip);
                if (Re > 0.0) {
                    double fbar = -taubar * tau / f;
                    Rebar = fbar * 0.15 * 0.687 * pow(Re, 0.687 - 1.0);
                    for (int a = 0; a < 3; ++a) {
                        double sbar = Rebar * Re * slip[a] / s2;
                        ufbar[a] += sbar;
                        ubar[a] -= sbar;
                    }
                }
            }
            /* Interpolation: u_f(x) = sum_k w_k(x) U[k] (nearest grid point:
             * one corner of weight 1, whose weight does not depend on x). */
            for (int k8 = 0; k8 < 8; ++k8) {
                double dot = 0.0;
                for (int c = 0; c < 3; ++c) {
                    int64_t q = field_index(m, c, st.cell[k8][0], st.cell[k8][1],
                                            st.cell[k8][2]);
                    Ub[q] += st.w[k8] * ufbar[c];
                    dot += Uf[q] * ufbar[c];
                }
                if (m->interp != 1)
                    for (int a = 0; a < 3; ++a) xbar[a] += st.dw[k8][a] * dot;
            }
            /* tau = rho_p d^2/(18 mu): dtau/dd = 2 tau/d;
             * m = w rho_p pi d^3/6:   dm/dd = 3 m/d. */
            db += tausbar * 2.0 * tau_s / d[p] + mbar * 3.0 * mass / d[p];
            if (Re > 0.0) db += Rebar * Re / d[p];
        }
        dbar[p] = db;
    }
    free(xs);
    free(us);
    free(scratch);
    return 0;
}

int or_adjoint(const or_mesh *m, const double *Uf, int64_t np,
               const double *x0, const double *up0, const double *d,
               double dt, int32_t nsteps, const double *lambda, double *Ubar,
               double *dbar)
{
    /* One field and one sub-step per step: the general reverse pass. */
    int32_t *fs = (int32_t *)calloc((size_t)(nsteps > 0 ? nsteps : 1), sizeof(int32_t));
    double *dts = (double *)malloc(sizeof(double) * (size_t)(nsteps > 0 ? nsteps : 1));
    if (!fs || !dts) {
        free(fs); free(dts);
        return -1;
    }
    for (int32_t n = 0; n < nsteps; ++n) dts[n] = dt;
    int r = or_adjoint_run(m, 1, Uf, nsteps, fs, dts, 1, np, x0, up0, d, lambda,
                           Ubar, dbar);
    free(fs);
    free(dts);
    return r;
}

/* ------------------------------------------------------------------------ */
/* Hilbert curve and segments (Sec. 2.2)                                     */
/* ------------------------------------------------------------------------ */

int64_t or_hilbert_index(int32_t order, const int32_t xyz[3])
{
    /* Skilling's axes-to-transpose: undo the rotations and reflections from
     * the most significant bit down, then Gray-encode. */
    uint32_t X[3] = {(uint32_t)xyz[0], (uint32_t)xyz[1], (uint32_t)xyz[2]};
    const uint32_t M = 1u << (order - 1);
    for (uint32_t Q = M; Q > 1; Q >>= 1) {
        const uint32_t P = Q - 1;
        for (int i = 0; i < 3; ++i) {
            if (X[i] & Q) {
                X[0] ^= P;                       /* invert low bits of x */
            } else {
                const uint32_t t = (X[0] ^ X[i]) & P;   /* exchange with x */
                X[0] ^= t;
                X[i] ^= t;
            }
        }
    }
    for (int i = 1; i < 3; ++i) X[i] ^= X[i - 1];
    uint32_t t = 0;
    for (uint32_t Q = M; Q > 1; Q >>= 1)
        if (X[2] & Q) t ^= Q - 1;
    for (int i = 0; i < 3; ++i) X[i] ^= t;
    /* interleave: bit b of the index, counted from the top, comes from axis
     * (b mod 3) at bit level (order - 1 - b / 3) */
    int64_t h = 0;
    for (int level = order - 1; level >= 0; --level)
        for (int i = 0; i < 3; ++i) h = (h << 1) | (int64_t)((X[i] >> level) & 1u);
    return h;
}

int or_hilbert_positions(int32_t order, int64_t nseg, int64_t seg_begin, int64_t seg_end,
                         int64_t per_seg, const double L[3], const double *u, double *x)
{
    if (order < 1 || order > 10 || nseg < 1 || per_seg < 1 || seg_begin < 0 ||
        seg_end > nseg || seg_begin > seg_end)
        return -1;
    const int64_t side = (int64_t)1 << order;
    const int64_t V = side * side * side;
    if (nseg > V) return -1;
    /* table: curve position -> voxel, by inverting the index over the lattice */
    int32_t *vox = (int32_t *)malloc(sizeof(int32_t) * 3 * (size_t)V);
    if (!vox) return -1;
    for (int32_t k = 0; k < side; ++k)
        for (int32_t j = 0; j < side; ++j)
            for (int32_t i = 0; i < side; ++i) {
                const int32_t c[3] = {i, j, k};
                const int64_t h = or_hilbert_index(order, c);
                vox[3 * h] = i;
                vox[3 * h + 1] = j;
                vox[3 * h + 2] = k;
            }
    int64_t n = 0;
    for (int64_t sg = seg_begin; sg < seg_end; ++sg) {
        const int64_t v0 = sg * V / nseg, v1 = (sg + 1) * V / nseg;
        const int64_t nv = v1 - v0;
        for (int64_t k = 0; k < per_seg; ++k, ++n) {
            const int64_t v = v0 + k * nv / per_seg;
            for (int a = 0; a < 3; ++a)
                x[3 * n + a] = ((double)vox[3 * v + a] + u[3 * n + a]) * (L[a] / (double)side);
        }
    }
    free(vox);
    return 0;
}

void or_bounding_boxes(int64_t np, const double *x, const int64_t *id, int64_t id0,
                       int64_t per_part, int64_t nparts, double *box)
{
    for (int64_t p = 0; p < nparts; ++p)
        for (int a = 0; a < 3; ++a) {
            box[6 * p + a] = INFINITY;
            box[6 * p + 3 + a] = -INFINITY;
        }
    for (int64_t q = 0; q < np; ++q) {
        if (id[q] < id0) continue;
        const int64_t p = (id[q] - id0) / per_part;
        if (p >= nparts) continue;
        for (int a = 0; a < 3; ++a) {
            if (x[3 * q + a] < box[6 * p + a]) box[6 * p + a] = x[3 * q + a];
            if (x[3 * q + a] > box[6 * p + 3 + a]) box[6 * p + 3 + a] = x[3 * q + a];
        }
    }
}
