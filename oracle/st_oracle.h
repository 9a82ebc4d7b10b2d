/*
 * Plain FP64 CPU oracle for the per-particle Lagrangian time step of
 * SCALE-TRACK (Schmalfuss, Lesnik, Rusche, Niedermeier, arXiv 2603.26691).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this code; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no source, header, constant or helper
 * with the HIP implementation.
 *
 * What is computed (paper, Sec. 2.1 "Governing equations" and Sec. 2.5
 * "Further implementation details"):
 *   - Newton's law for a particle, dx_p/dt = u_p and m_p du_p/dt = sum F
 *     (Sec. 2.1, particle equations of motion), with drag plus gravity as
 *     the forces (the paper keeps only drag; gravity comes from the workload
 *     definition and is a documented reading).  The drag is Stokes drag or
 *     the paper's Schiller-Naumann correction of it (Sec. 2.1);
 *   - semi-implicit Euler: drag implicit, gravity explicit, position advanced
 *     with the new velocity (Sec. 2.5); with Schiller-Naumann the correction
 *     factor is taken from the slip at the start of the step;
 *   - the momentum source S_u = (1/V_cell) d(m_p u_p)/dt of Sec. 2.1, read as
 *     the fluid receiving minus the drag impulse, deposited into the cell
 *     that contains the particle at the start of the step (Sec. 2.5);
 *   - fluid velocity at the particle: trilinear interpolation of the
 *     cell-centred field (default) or the paper's nearest-grid-point scheme
 *     (Sec. 2.5);
 *   - a fixed number of sub-steps per call with the field held fixed
 *     (Sec. 3.3).
 *
 * Precision: everything in IEEE binary64; particles processed in id order,
 * sources summed in id order.  Mesh: n[0] x n[1] x n[2] uniform periodic
 * cells on [0,L0) x [0,L1) x [0,L2).  Fields are laid out [3][n2][n1][n0]
 * (component, z, y, x; x fastest).
 */
#ifndef ST_ORACLE_H
#define ST_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t n[3];          /* cells per axis */
    int32_t interp;        /* 0 = trilinear, 1 = nearest grid point */
    int32_t drag;          /* 0 = Stokes, 1 = Schiller-Naumann (Sec. 2.1) */
    int32_t reserved;
    double  L[3];          /* domain extent per axis [m] */
    double  rho_f;         /* fluid density [kg/m^3] (Reynolds number only) */
    double  mu_f;          /* fluid dynamic viscosity [Pa s] */
    double  g[3];          /* gravitational acceleration [m/s^2] */
    double  rho_p;         /* particle material density [kg/m^3] */
    double  parcel_weight; /* droplets represented by one parcel (Sec. 3.2) */
} or_mesh;

/* Cell index of position x along each axis: floor(x_a / h_a) modulo n_a. */
void or_cell(const or_mesh *m, const double x[3], int32_t c[3]);

/* or_cell for np positions ([np][3] -> [np][3]). */
void or_cells(const or_mesh *m, int64_t np, const double *x, int32_t *c);

/* Periodic wrap of a position that moved by less than one domain length. */
void or_wrap(const or_mesh *m, double x[3]);

/* Fluid velocity at x from the cell-centred field Uf ([3][n2][n1][n0]). */
void or_interp(const or_mesh *m, const double *Uf, const double x[3],
               double uf_at_p[3]);

/* or_interp for np positions ([np][3] -> [np][3]). */
void or_interp_many(const or_mesh *m, const double *Uf, int64_t np,
                    const double *x, double *uf_at_p);

/* Transpose of or_interp: Ubar[corner] += weight * a (per component). */
void or_interp_transpose(const or_mesh *m, const double x[3],
                         const double a[3], double *Ubar);

/* Response time tau_p = rho_p d^2 / (18 mu_f) and parcel mass
 * m_p = w rho_p pi d^3 / 6. */
double or_tau(const or_mesh *m, double d);
double or_mass(const or_mesh *m, double d);

/* Drag factor f relative to Stokes drag for the slip u_f - u_p: 1 (Stokes) or
 * 1 + 0.15 Re^0.687 with Re = rho_f |u_f - u_p| d / mu_f (Schiller-Naumann).
 * A step uses the effective response time tau / f, f taken with the slip at
 * the start of the step (drag coefficient explicit, velocity implicit). */
double or_drag_factor(const or_mesh *m, double d, const double slip[3]);

/* One call of the Lagrangian step on np particles: nsub sub-steps of dt/nsub
 * with the field held fixed.  x, up updated in place ([np][3]); the time
 * integrated momentum source of every sub-step is added to Su_int
 * ([3][n2][n1][n0]), i.e. Su_int[c0] -= J / V_cell. */
void or_step(const or_mesh *m, const double *Uf, int64_t np, double *x,
             double *up, const double *d, double dt, int32_t nsub,
             double *Su_int);

/* nsteps calls of or_step with the same field. */
void or_run(const or_mesh *m, const double *Uf, int64_t np, double *x,
            double *up, const double *d, double dt, int32_t nsteps,
            int32_t nsub, double *Su_int);

/* nsteps steps with a field that turns about z: step n uses
 * U^n = R_z(theta_n) U^0 with (cos theta_n, sin theta_n) = cs[2n], cs[2n+1]. */
void or_run_rotating(const or_mesh *m, const double *U0, const double *cs,
                     int64_t np, double *x, double *up, const double *d,
                     double dt, int32_t nsteps, double *Su_int);

/* Extrapolator-corrector for sources that arrive one step late (paper
 * Sec. 2.4).  At the current step only the actual source of the previous
 * step, S_last, is available.  The corrector is S_last minus the
 * extrapolation that stood in for it one step earlier (ext_prev); the
 * extrapolation for the current step is 0 (kind 0, zero), S_last (kind 1,
 * constant) or 2 S_last - S_prev2 (kind 2, linear), S_prev2 being the actual
 * source one step further back.  The source to apply is corrector plus
 * extrapolation; then ext_prev <- extrapolation, S_prev2 <- S_last.  All
 * arrays hold n values (cells times components); ext_prev and S_prev2 start
 * at zero. */
void or_ec_estimate(int64_t n, int32_t kind, const double *S_last, double *S_prev2,
                    double *ext_prev, double *applied);

/* Hilbert index of voxel (x, y, z) on the 2^order lattice per axis
 * (paper Sec. 2.2, particle initialisation along a Hilbert curve): the
 * published transpose algorithm of Skilling (AIP Conf. Proc. 707, 2004),
 * axes to transpose, then the transpose's bits interleaved most significant
 * first (x before y before z).  order 1..10. */
int64_t or_hilbert_index(int32_t order, const int32_t xyz[3]);

/* Placement of particles by Hilbert segments (Sec. 2.2): the 8^order voxels in
 * curve order are cut into nseg consecutive segments, segment s holding
 * voxels [floor(s V / nseg), floor((s+1) V / nseg)), V = 8^order.  Particle k
 * (0 <= k < per_seg) of segment s lies in the segment's voxel
 * floor(k nv / per_seg) (nv voxels in the segment: counts per voxel differ by
 * at most one and every segment holds exactly per_seg particles), at
 * x_a = (c_a + u_a) (L_a / 2^order) with u in [0,1)^3 given.  Writes the
 * positions of segments [seg_begin, seg_end) in order ([n][3],
 * n = (seg_end - seg_begin) per_seg).  The voxel of a curve position is found
 * by inverting or_hilbert_index over the whole lattice.  Returns 0, or -1 on
 * bad arguments or when the table cannot be allocated. */
int or_hilbert_positions(int32_t order, int64_t nseg, int64_t seg_begin, int64_t seg_end,
                         int64_t per_seg, const double L[3], const double *u, double *x);

/* Axis-aligned bounding boxes of particle partitions: partition p holds the
 * particles with id in [id0 + p per_part, id0 + (p+1) per_part); box p is
 * (min x, min y, min z, max x, max y, max z) over them (Sec. 2.2, chunk
 * bounding boxes).  An empty partition gets min = +inf, max = -inf. */
void or_bounding_boxes(int64_t np, const double *x, const int64_t *id, int64_t id0,
                       int64_t per_part, int64_t nparts, double *box);

/* Reverse-mode derivative of a run of or_step calls starting from (x0, up0),
 * for a loss whose derivative with respect to the time-integrated source
 * Su_int is lambda ([3][n2][n1][n0]).  The paper defines no adjoint: this is
 * the derivative of the discrete step above, taken by reversing its
 * operations (the deposit's transpose is a gather of lambda in the
 * start-of-sub-step cell, the interpolation's transpose a scatter onto the
 * field; the cell index and the periodic wrap are piecewise constant and
 * contribute nothing).  Step n (0 <= n < nsteps) is nsub sub-steps of
 * dt_of_step[n] / nsub with the field fields[field_of_step[n]] held fixed
 * (fields: [nfields][3][n2][n1][n0]).  Adds dL/d(field k) to
 * Ubar[k] ([nfields][3][n2][n1][n0]) and writes dL/dd to dbar ([np]).
 * Returns 0, or -1 on bad arguments or if the forward tape could not be
 * allocated. */
int or_adjoint_run(const or_mesh *m, int32_t nfields, const double *fields,
                   int32_t nsteps, const int32_t *field_of_step,
                   const double *dt_of_step, int32_t nsub, int64_t np,
                   const double *x0, const double *up0, const double *d,
                   const double *lambda, double *Ubar, double *dbar);

/* or_adjoint_run with one field and one sub-step of dt per step (nsteps
 * calls of or_step with nsub = 1). */
int or_adjoint(const or_mesh *m, const double *Uf, int64_t np,
               const double *x0, const double *up0, const double *d,
               double dt, int32_t nsteps, const double *lambda, double *Ubar,
               double *dbar);

/* Particle-parallel drivers (st_oracle_par.c): the same computations as
 * or_run and or_adjoint_run, with the particles split into nthreads
 * contiguous ranges run on their own threads and the per-range source or
 * gradient arrays added in range order.  Particle states and dL/dd are
 * bitwise those of the serial calls; per-cell sums differ only by the order
 * of the additions.  Return 0, or -1 on bad arguments or allocation
 * failure. */
int or_run_par(const or_mesh *m, const double *Uf, int64_t np, double *x, double *up,
               const double *d, double dt, int32_t nsteps, int32_t nsub, double *Su_int,
               int32_t nthreads);
int or_adjoint_run_par(const or_mesh *m, int32_t nfields, const double *fields,
                       int32_t nsteps, const int32_t *field_of_step, const double *dt_of_step,
                       int32_t nsub, int64_t np, const double *x0, const double *up0,
                       const double *d, const double *lambda, double *Ubar, double *dbar,
                       int32_t nthreads);

#ifdef __cplusplus
}
#endif
#endif
