/*
 * scaletrack: the per-particle Lagrangian time step of SCALE-TRACK
 * (Schmalfuss, Lesnik, Rusche, Niedermeier, arXiv 2603.26691) as a C-ABI
 * library for AMD Instinct MI355X (gfx950).
 *
 * The library tracks point particles ("parcels", paper Sec. 3.2) through a
 * given cell-centred fluid velocity field on a uniform periodic Cartesian
 * mesh and returns the momentum source they feed back to the fluid
 * (paper Sec. 2.1, particle equations of motion and momentum source; Sec. 2.5,
 * what the Lagrangian solver needs from and returns to the Eulerian solver).
 * One call of st_step, per particle:
 *   1. gathers the fluid velocity at the particle (trilinear interpolation of
 *      the cell-centred field, or the paper's nearest-grid-point scheme,
 *      Sec. 2.5);
 *   2. integrates m du_p/dt = m (u_f - u_p)/tau + m g with semi-implicit
 *      Euler (drag implicit, gravity explicit, position with the new
 *      velocity; Sec. 2.5), tau = rho_p d^2 / (18 mu_f) (Stokes drag), or
 *      tau divided by the Schiller-Naumann factor 1 + 0.15 Re^0.687,
 *      Re = rho_f |u_f - u_p| d / mu_f, taken from the slip at the start of
 *      the step (Sec. 2.1, drag force);
 *   3. moves the particle (periodic wrap) and re-bins it into its new cell
 *      and 8^3-cell chunk;
 *   4. deposits the reacting momentum, minus the drag impulse
 *      J = m (u_p' - u_p - g dt), divided by the cell volume, into the cell
 *      that held the particle at the start of the step (Sec. 2.1 momentum
 *      source, Sec. 2.5 deposit into the containing cell).
 *
 * Conventions for every entry point:
 *   - Return value is an st_status.  Argument errors are detected on the
 *     host, before anything is enqueued, and leave the state unchanged;
 *     st_last_error(ctx) then holds a message.  No exception or abort crosses
 *     this boundary.  A failed HIP call surfaces as ST_ERR_DEVICE.
 *   - Work is ordered on the caller's HIP stream (hip_stream, a hipStream_t;
 *     NULL = the default stream).  Pointers passed in are borrowed until the
 *     stream has reached the call's completion.  Outputs go to caller-owned
 *     buffers.
 *   - "on_device" non-zero means the pointer is device memory on the
 *     context's device; zero means host memory (the call then synchronises
 *     the stream before returning).
 *   - Fields are [3][n2][n1][n0]: component, z, y, x, with x fastest.
 *     Positions and velocities are [count][3].  Particle order inside the
 *     library is private; everything user visible is indexed by the particle
 *     id, which is the injection order (0, 1, 2, ...).
 *   - One context per host thread; the library is not internally
 *     thread-safe.
 */
#ifndef SCALETRACK_ST_H
#define SCALETRACK_ST_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct st_ctx st_ctx; /* opaque; owns every device buffer it uses */

typedef enum {
    ST_OK = 0,
    ST_ERR_INVALID = 1,   /* bad argument; nothing was enqueued */
    ST_ERR_OOM = 2,       /* device allocation failed */
    ST_ERR_DEVICE = 3,    /* a HIP call failed */
    ST_ERR_STATE = 4,     /* call not valid in the current state */
    ST_ERR_CAPACITY = 5   /* particle count would exceed the capacity */
} st_status;

typedef enum {
    /* particle state, field, interpolation and sources in binary64 */
    ST_FORM_FP64 = 0,
    /* particle state and interpolation in binary32, positions stored as
     * chunk-local offsets (the chunk origin is exact, implied by the chunk
     * index); impulses, source accumulation and totals in binary64 */
    ST_FORM_FP32_LOCAL = 1,
    /* everything in binary32, sources included; positions stored as
     * coordinates in metres, a particle's cell taken from the binary32
     * product x * fl32(n / L) (clamped to [0, n)).  Steps cannot be taped
     * in this form. */
    ST_FORM_FP32 = 2
} st_form;

typedef enum {
    ST_DRAG_STOKES = 0,           /* f = 1 */
    ST_DRAG_SCHILLER_NAUMANN = 1  /* f = 1 + 0.15 Re^0.687 (paper Sec. 2.1) */
} st_drag;

typedef struct {
    int32_t n[3];          /* cells per axis; each a multiple of chunk_edge */
    int32_t chunk_edge;    /* cells per chunk edge: 2, 4 or 8 */
    double  L[3];          /* domain extent per axis [m]; origin at 0; periodic */
    double  rho_f;         /* fluid density [kg/m^3], >= 0 (Reynolds number) */
    double  mu_f;          /* fluid dynamic viscosity [Pa s], > 0 */
    double  g[3];          /* gravitational acceleration [m/s^2] */
    double  rho_p;         /* particle material density [kg/m^3], > 0 */
    double  parcel_weight; /* droplets per parcel (paper Sec. 3.2), > 0 */
    int32_t form;          /* an st_form */
    int32_t interp;        /* 0 = trilinear (default), 1 = nearest grid point */
    int32_t drag;          /* an st_drag */
    int32_t reserved;      /* must be 0 */
    int64_t capacity;      /* maximum number of particles, >= 1 */
} st_mesh_desc;

/* Paper Sec. 2.5 (the Lagrangian solver needs the domain geometry, the mesh
 * and the Eulerian fields) and Sec. 2.2 (particles held as structure of
 * arrays per partition; here the partitions are fixed 8^3-cell chunks).
 * Creates a context on HIP device `device` and allocates, once, every
 * buffer a run of up to desc->capacity particles needs.  *out receives the
 * context.  ST_ERR_INVALID for a bad descriptor, ST_ERR_OOM when the device
 * cannot hold the buffers. */
st_status st_create_mesh(const st_mesh_desc *desc, int device, st_ctx **out);

/* Outside the paper (lifetime of a context).
 * Frees every buffer of the context (after synchronising its device). */
st_status st_destroy(st_ctx *ctx);

/* Outside the paper (error reporting).
 * Message describing the last error of this context ("" if none);
 * st_last_error(NULL) describes the last failed st_create_mesh of the
 * calling thread. */
const char *st_last_error(const st_ctx *ctx);

/* Paper Sec. 2.3 (particles are created directly on the GPU) and Sec. 3.2
 * (parcels: each represents parcel_weight droplets).
 * Adds n particles: x, up [n][3] (positions in [0,L) per axis, velocities),
 * d [n] (diameters > 0), all binary64.  Positions outside the box are
 * wrapped periodically.  New ids continue the injection order.  Host
 * arrays are validated on the host (non-finite values or d <= 0 give
 * ST_ERR_INVALID); device arrays are validated on the device and the call
 * waits for the result.  ST_ERR_CAPACITY if the count would exceed the
 * capacity (state unchanged). */
st_status st_inject(st_ctx *ctx, int64_t n, const double *x, const double *up,
                    const double *d, int on_device, void *hip_stream);

/* Outside the paper (bookkeeping).  Number of particles in the context. */
st_status st_count(const st_ctx *ctx, int64_t *n);

/* Paper Sec. 2.1 (equation of motion, drag, momentum source), Sec. 2.5
 * (semi-implicit Euler, interpolation and deposit in the containing cell)
 * and Sec. 3.3 (sub-steps); the steps numbered in the header above.
 * Advances every particle by dt with nsub sub-steps of dt/nsub, the field
 * u_cells (device memory, [3][n2][n1][n0], binary64 for ST_FORM_FP64 and
 * binary32 otherwise) held fixed (paper Sec. 3.3, sub-steps).  Each
 * sub-step adds its deposit to the context's time-integrated source.
 * tape != 0 records the step for st_backward: the field pointer is then
 * borrowed until st_backward or st_tape_clear; a checkpoint of the
 * particle state is kept every `tape` sub-steps (the value of the first
 * taped call fixes the interval; ST_ERR_INVALID in the form
 * ST_FORM_FP32).  dt must be finite and > 0, nsub >= 1. */
st_status st_step(st_ctx *ctx, const void *u_cells, double dt, int32_t nsub,
                  int32_t tape, void *hip_stream);

/* Paper Sec. 2.1 (momentum source S_u) and Sec. 2.5 (the sources are fed
 * back to the Eulerian solver).
 * Copies the time-integrated momentum source, sum over sub-steps of
 * S_u dt [kg/(m^2 s)] = -(sum of impulses J) / V_cell per cell, as binary64
 * [3][n2][n1][n0] into out.  reset != 0 zeroes the context's accumulator
 * afterwards. */
st_status st_get_sources(st_ctx *ctx, double *out, int32_t reset,
                         int on_device, void *hip_stream);

/* Outside the paper (read-out of the state for checks and output; the
 * paper's particle state is position, velocity and diameter, Sec. 2.1).
 * Copies the particle state, indexed by id, into any of the non-NULL
 * outputs: x, up [count][3] binary64 (positions in [0,L)), d [count]
 * binary64, id [count] int64 (id[i] = i once the copy is complete, a
 * check of the permutation), cell [count][3] int32 (cell per axis). */
st_status st_get_particles(st_ctx *ctx, double *x, double *up, double *d,
                           int64_t *id, int32_t *cell, int on_device,
                           void *hip_stream);

/* Outside the paper: the paper defines no adjoint.  This is the derivative
 * of the discrete step st_step computes (Sec. 2.1, Sec. 2.5), taken by
 * reversing its operations: the deposit's transpose is a gather of
 * dL/dS_int in the start-of-step cell, the interpolation's transpose a
 * scatter onto the field; the cell index and the periodic wrap are
 * piecewise constant and contribute nothing.  The differentiable form and
 * its checkpointing (every `tape` sub-steps, recomputation in between)
 * follow the workload's definition of differentiation with respect to the
 * fluid velocity field and the particle diameters.
 * Reverse-mode derivative of the taped steps.  dL_dSint (device,
 * [3][n2][n1][n0] binary64) is the derivative of a scalar loss with respect
 * to the time-integrated source accumulated by the taped steps.  Writes
 * dL/du (device, [3][n2][n1][n0] binary64; the sum over the taped steps'
 * fields, which are one tensor when every step used the same field) and
 * dL/dd (device, [count] binary64, by id; may be NULL when count is 0).
 * Checkpoints are restored and
 * the steps between them recomputed.  The tape is consumed; its checkpoint
 * buffers and the call's workspace (about tape + 1 copies of the particle
 * store, plus the adjoint records: 8 values of the state precision per
 * particle and per slot) stay allocated for the next taped run until
 * st_tape_clear or st_destroy.  Returns when the results are written and the
 * store holds the state the taped run ended in (the call synchronises
 * hip_stream); after a HIP error the store's contents are undefined.
 * ST_ERR_STATE if nothing is taped. */
st_status st_backward(st_ctx *ctx, const double *dL_dSint, double *dL_du,
                      double *dL_dd, void *hip_stream);

/* Outside the paper (see st_backward).  Drops the tape without
 * differentiating, and releases the buffers st_backward keeps. */
st_status st_tape_clear(st_ctx *ctx);

/* Outside the paper (see st_backward).  Allocates ahead of time what a taped
 * run of `substeps` sub-steps with a checkpoint every `tape` sub-steps and
 * its st_backward need (the checkpoint buffers and the backward's workspace,
 * for the particles held now), so that neither st_step nor st_backward
 * allocates during that run: for callers that time or capture it.  The
 * buffers are kept like those of a consumed tape (released by st_tape_clear
 * or st_destroy).  ST_ERR_INVALID for tape <= 0, substeps < 0 or the FP32
 * everywhere form (which is not taped), ST_ERR_STATE while a tape is
 * recorded, ST_ERR_OOM when the device memory runs out. */
st_status st_tape_reserve(st_ctx *ctx, int32_t tape, int64_t substeps);

/* Paper Sec. 2.3 (asynchronous coupling; the Eulerian and Lagrangian phases
 * at most one time step apart) and Sec. 2.5 (the lag of one step).  On one
 * GPU the Eulerian update is a synthetic field rotation on a second stream.
 * Asynchronously coupled run:
 * nsteps steps of dt in which step k uses the field
 * U^k = R_z(theta_k) U^0, rotated about z with (cos, sin) of theta_k given
 * in cs[2k], cs[2k+1] (host memory).  A second stream owned by the context
 * builds U^(k+1) while the particles step with U^k; events hold the lag at
 * exactly one step.  u0 is device memory in the form's field precision.
 * field_ms (host, may be NULL) receives the summed device time of the
 * field updates and step_ms that of the particle steps, measured with HIP
 * events on the respective streams; total_ms the wall time from the first
 * launch to the last completion (the call synchronises when any of the
 * three is non-NULL). */
st_status st_run_coupled(st_ctx *ctx, const void *u0, const double *cs,
                         int32_t nsteps, double dt, float *field_ms,
                         float *step_ms, float *total_ms, void *hip_stream);

/* Extrapolators of the extrapolator-corrector (paper Sec. 2.4). */
typedef enum {
    ST_EXTRAP_ZERO = 0,    /* no estimate: sources are applied one step late */
    ST_EXTRAP_CONST = 1,   /* the last available source */
    ST_EXTRAP_LINEAR = 2   /* linear extrapolation from the last two sources */
} st_extrapolator;

/* Paper Sec. 2.4 (extrapolator-corrector method: corrector, estimated
 * source, zero, constant and linear extrapolators).  The corrector subtracts
 * the previous extrapolation (the part of the previous estimate that stood
 * in for the then unknown source), which makes the applied sources add up
 * to the actual ones (the conservation over time the section states).
 * Extrapolator-corrector for a fluid solver that runs one step ahead of the
 * particles.  At
 * the current step only S_last, the actual time-integrated source of the
 * previous step (e.g. from st_get_sources with reset), is available.  Per
 * cell and component the call returns in `applied`
 *   (S_last - E_prev) + E_now,
 * the corrector (what the previous step's extrapolation E_prev missed) plus
 * the extrapolation E_now for the current step: 0, S_last, or
 * 2 S_last - S_prev (S_prev: the S_last of the previous call), and keeps
 * E_now and S_last for the next call.  Summed over calls, the applied
 * sources equal the actual ones plus the extrapolation still outstanding
 * (conservative over time).  S_last and applied are [3][n2][n1][n0]
 * binary64; `kind` is an st_extrapolator. */
st_status st_ec_estimate(st_ctx *ctx, int32_t kind, const double *S_last, double *applied,
                         int on_device, void *hip_stream);

/* Paper Sec. 2.4 (no source is available before the first step).  Clears
 * the extrapolator-corrector's history (E_prev = S_prev = 0). */
st_status st_ec_reset(st_ctx *ctx, void *hip_stream);

/* Outside the paper (instrumentation of the re-bin).
 * Counters of the last st_step (host memory): movers, full repacks so far,
 * particles, store slots, work items (chunk runs of the step kernel), holes
 * (slots that particles left and no arrival has taken yet; they are skipped
 * until the next full re-bin).  Any pointer may be NULL.  Synchronises the
 * stream. */
st_status st_stats(st_ctx *ctx, int64_t *last_movers, int64_t *repacks,
                   int64_t *particles, int64_t *slots, int64_t *items, int64_t *holes,
                   void *hip_stream);

/* Outside the paper (measurement; the paper reports times per step,
 * Sec. 4).
 * Device time of the step kernel (the per-particle gather, integrate,
 * deposit and relocate) measured with a pair of HIP events attached to each
 * of its launches (hipExtLaunchKernel), which take the start and end of the
 * kernel's own execution on the launch stream.  enable != 0 starts a measurement (clearing
 * earlier ones); enable == 0 stops it.  kernel_ms and launches (host, may be
 * NULL) receive the summed milliseconds and the number of launches measured
 * so far; reading them synchronises the recorded events. */
st_status st_timing(st_ctx *ctx, int32_t enable, double *kernel_ms,
                    int64_t *launches);

/* Outside the paper (measurement reference).  Copies `bytes` (a multiple of
 * 16) from src to dst (device memory, 16-byte aligned, not overlapping) with
 * the access pattern of the particle state in st_step: one 16-byte
 * non-temporal load and store per thread.  Its rate is the practical ceiling
 * of streaming traffic beside the published HBM peak.  Ordered on hip_stream;
 * ST_ERR_INVALID for bad arguments (no context, so no message). */
st_status st_stream_copy(const void *src, void *dst, int64_t bytes, void *hip_stream);

/* Paper Sec. 2.2 (particles initialised along a Hilbert curve whose
 * segments give the initial partitions).
 * Positions of new particles placed by Hilbert-curve segments.  The domain [0,L) is a lattice of 2^order voxels
 * per axis (order 1..10) visited in Hilbert-curve order (the orientation of
 * Skilling's transpose algorithm, AIP Conf. Proc. 707, 2004: the curve starts
 * in voxel (0,0,0) and ends in (2^order - 1, 0, 0)); its V = 8^order voxels are
 * cut into nseg (1..V) consecutive segments, segment s holding curve positions
 * [floor(s V / nseg), floor((s+1) V / nseg)).  Particle k (0 <= k < per_seg)
 * of segment s lies in the segment's voxel number floor(k nv / per_seg), nv its
 * voxel count, at x_a = (c_a + u_a) L_a / 2^order, c the voxel and u[3] in
 * [0,1) given by the caller.  Writes x ([n][3] binary64) for the particles of
 * segments [seg_begin, seg_end) in order, n = (seg_end - seg_begin) per_seg
 * (per_seg 1..2^31).  u and x: device memory when on_device, else host. */
st_status st_hilbert_positions(st_ctx *ctx, int32_t order, int64_t nseg, int64_t seg_begin,
                               int64_t seg_end, int64_t per_seg, const double *u, double *x,
                               int32_t on_device, void *hip_stream);

/* Paper Sec. 2.2 (initialisation by Hilbert segments) and Sec. 2.3
 * (particles created on the GPU).
 * Injects the particles that st_hilbert_positions places, with velocities up
 * ([n][3]) and diameters d ([n]); their ids continue the injection order, so
 * particle k of segment s gets id first + (s - seg_begin) per_seg + k.  Any
 * range of segments can be injected independently (the placement is global
 * and deterministic).  Errors as st_inject; host u outside [0,1) is
 * ST_ERR_INVALID. */
st_status st_inject_hilbert(st_ctx *ctx, int32_t order, int64_t nseg, int64_t seg_begin,
                            int64_t seg_end, int64_t per_seg, const double *u, const double *up,
                            const double *d, int32_t on_device, void *hip_stream);

/* Paper Sec. 2.2 (a rectangular box around the particles of each partition,
 * which identifies the Eulerian partitions it needs) and Sec. 2.3 (the boxes
 * are computed on the GPU and sent to the host).
 * Axis-aligned bounding boxes of particle partitions: partition p (0 <= p < nparts) holds the particles with id in
 * [id0 + p per_part, id0 + (p+1) per_part).  boxes ([nparts][6] binary64:
 * min x, min y, min z, max x, max y, max z, over the positions st_get_particles
 * returns; device memory when on_device) receives them; an empty partition gets
 * min = +inf and max = -inf. */
st_status st_bounding_boxes(st_ctx *ctx, int64_t id0, int64_t per_part, int64_t nparts,
                            double *boxes, int32_t on_device, void *hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * boxes as st_bounding_boxes, computed without any allocation.  The kernels
 * accumulate the bounds in a fixed device array of the library (one per GPU,
 * room for ST_NOALLOC_MAX_PARTS partitions, 3 MiB, held until the process
 * ends), which is then copied to `boxes` (device memory when on_device, else
 * host memory, and the call then synchronises the stream).  nparts above
 * ST_NOALLOC_MAX_PARTS gives ST_ERR_INVALID, as do the argument errors of
 * st_bounding_boxes.  Every call on one GPU shares that array: calls that
 * overlap on one GPU (other streams, other host threads, other contexts)
 * race, and the caller must order them. */
#define ST_NOALLOC_MAX_PARTS 65536
st_status st_bounding_boxes_noalloc(st_ctx *ctx, int64_t id0, int64_t per_part, int64_t nparts,
                                    double *boxes, int32_t on_device, void *hip_stream);

#ifdef __cplusplus
}
#endif
#endif
