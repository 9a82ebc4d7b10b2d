// Reverse mode of the taped particle steps (the paper gives no adjoint; this
// is the derivative of the discrete step the library computes).
//
// For a loss L whose derivative with respect to the time-integrated source
// is lambda = dL/dSu_int, one step of one particle (state x, u_p, d at the
// step start; u_p' the new velocity; D = tau + dt) is reversed as
//   Jbar   = -lambda[c0] / V_cell                  (deposit -> gather)
//   wbar   = ubar' + dt xbar' + m Jbar              (everything reading u_p')
//   ubar   = -m Jbar + (tau / D) wbar
//   mbar   = Jbar . (u_p' - u_p - g dt)
//   ufbar  = (dt / D) wbar                           (interpolation -> scatter)
//   taubar = wbar . (u_p + dt g - u_p') / D
//   Ubar[corner k] += w_k ufbar,   xbar = xbar' + sum_k grad w_k (U_k . ufbar)
//   dbar  += taubar 2 tau / d + mbar 3 m / d
// With Schiller-Naumann drag tau is tau_s / f, f = 1 + 0.15 Re^0.687 of the
// start-of-step slip s = u_f - u_p, Re = (rho_f / mu_f) d |s|; then
//   Rebar  = -taubar (tau / f) 0.15 0.687 Re^-0.313
//   ufbar += Rebar Re s / |s|^2,  ubar -= Rebar Re s / |s|^2
//   dbar  += (taubar / f) 2 tau_s / d + Rebar Re / d + mbar 3 m / d
// (zero slip contributes no Re term).
// The cell c0 and the periodic wrap are piecewise constant (zero derivative).
//
// Checkpoints of the particle store are kept every `tape_every` taped steps;
// each segment is recomputed from its checkpoint (deposit off), each step
// saving the state it starts from, the ids and its layout as it streams
// them, and then reversed newest first (the newest from the store itself).
// The per-particle adjoint state is kept in one record of eight values of
// the state precision per particle, indexed within a segment by the
// particle's slot in the segment's checkpoint (its anchor): the restored
// checkpoint's ids are replaced by the slot indices before the
// recomputation, so every saved step carries anchors instead of ids, and
// since particles that stay in their chunk keep their slots, each step reads
// and writes the records nearly in slot order.  Between segments the records
// of particles whose slot changed pass through an array by particle id.
// The tile sums of dL/du of a chunk that is one work item are kept per chunk
// over all the reversed steps and added to dL/du once at the end.
#include "st_internal.h"

#include <math.h>

#include <algorithm>
#include <vector>

namespace st {
namespace {

template <class T>
struct AdjArgs {
    // saved store of the step (pointers into a snapshot)
    const T *ox, *oy, *oz, *vx, *vy, *vz, *d;
    const int32_t *id;
    const int64_t *base;
    const int32_t *cnt;
    const int32_t *items;
    const int32_t *nitems;
    const T *u;              // field of the step [3][n2][n1][n0]
    const double *lamC;      // dL/dSu_int by chunk [C][3][E^3]
    T *adj;                  // adjoint records by anchor, [nrec][8]: xbar[3], ubar[3], dbar, unused
    double *Ubar;            // dL/du [3][n2][n1][n0]
    double *tacc;            // per-chunk tile sums of dL/du over the steps, [C][3][S3], or null
    int64_t nrec;            // records (the store's slots)
    Params p;
    double dt;
};

// One workgroup of 256 threads per work item, two particles per thread and
// pass (one per pass, 384-thread groups at three waves per SIMD, three per
// pass, the next pass's loads issued during the current one, and a pass's
// LDS atomics issued after all its reverses measured no faster).
constexpr int kAdjBlock = 256;
constexpr int kAdjPPT = 2;

// Field index of cell r of a chunk's tile (its cells E*c - 1 .. E*c + E per
// axis, wrapped).
template <int E>
__device__ __forceinline__ int64_t tile_cell(const Params &p, int cx, int cy, int cz, int r)
{
    constexpr int S = E + 2;
    const int k = r / (S * S), j = (r / S) % S, i = r % S;
    int gx = cx * E - 1 + i, gy = cy * E - 1 + j, gz = cz * E - 1 + k;
    gx += gx < 0 ? p.n[0] : 0;
    gx -= gx >= p.n[0] ? p.n[0] : 0;
    gy += gy < 0 ? p.n[1] : 0;
    gy -= gy >= p.n[1] ? p.n[1] : 0;
    gz += gz < 0 ? p.n[2] : 0;
    gz -= gz >= p.n[2] ? p.n[2] : 0;
    return ((int64_t)gz * p.n[1] + gy) * p.n[0] + gx;
}

// Stages the chunk's tile of the field in LDS, its loads all issued before
// the first is used.
template <class T, int E, int NTH>
__device__ __forceinline__ void stage_tile(const Params &p, const T *u, int cx, int cy, int cz,
                                           T *tile)
{
    constexpr int S3 = (E + 2) * (E + 2) * (E + 2);
    constexpr int NT = (3 * S3 + NTH - 1) / NTH;
    const int64_t ncell = (int64_t)p.n[0] * p.n[1] * p.n[2];
    T vals[NT];
#pragma unroll
    for (int k = 0; k < NT; ++k) {
        const int t = threadIdx.x + k * NTH;
        if (t < 3 * S3) {
            const int comp = t / S3;
            vals[k] = u[comp * ncell + tile_cell<E>(p, cx, cy, cz, t - comp * S3)];
        }
    }
#pragma unroll
    for (int k = 0; k < NT; ++k) {
        const int t = threadIdx.x + k * NTH;
        if (t < 3 * S3) tile[t] = vals[k];
    }
}

// A saved slot holds a particle unless its anchor is -1 (no particle at
// that slot of the checkpoint) or it is a hole (a -1 offset in binary32, a
// negated diameter in binary64).
template <class T>
__device__ __forceinline__ bool adj_live(int64_t anchor, int64_t nrec, const T (&st)[7])
{
    return anchor >= 0 && anchor < nrec && st[0] >= T(0) && st[6] > T(0);
}

// Trilinear stencil of a chunk-local position [cells]: lowest corner i0 per
// axis (-1 .. E-1, a tile index after + 1) and fractional offsets fr.
template <int E>
__device__ __forceinline__ void stencil(const double (&xi)[3], int (&i0)[3], double (&fr)[3])
{
    for (int ax = 0; ax < 3; ++ax) {
        const double sx = xi[ax] - 0.5;
        const double fl = floor(sx);
        i0[ax] = min(max((int)fl, -1), E - 1);
        fr[ax] = sx - fl;
    }
}

// The reverse of one particle's step.  st: its saved state (chunk-local
// offsets, velocity, diameter); rc: its adjoint record (xbar[3], ubar[3],
// dbar), updated in place.  Returns ufbar (the adjoint of the interpolated
// field velocity, to be scattered onto the tile) and, for trilinear, the
// stencil (i0, fr); for nearest grid point t0 is the cell's tile index.
template <class T, int E, bool TRI>
__device__ __forceinline__ void reverse_particle(const Params &p, double dt, const T *tile,
                                                 const double *lam, const T (&st)[7],
                                                 double (&rc)[7], double (&ufb)[3],
                                                 int (&i0)[3], double (&fr)[3], int &t0)
{
    constexpr int S = E + 2;
    constexpr int S3 = S * S * S;
    constexpr int E3 = E * E * E;
    const double xi[3] = {(double)st[0], (double)st[1], (double)st[2]};
    const double up[3] = {(double)st[3], (double)st[4], (double)st[5]};
    const double dp = (double)st[6];

    // interpolation at the saved position, in binary64
    int cl[3];
    for (int ax = 0; ax < 3; ++ax) cl[ax] = min(max((int)xi[ax], 0), E - 1);
    double uf[3] = {0.0, 0.0, 0.0};
    if (TRI) {
        stencil<E>(xi, i0, fr);
        t0 = ((i0[2] + 1) * S + (i0[1] + 1)) * S + (i0[0] + 1);
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int bx = k & 1, by = (k >> 1) & 1, bz = (k >> 2) & 1;
            const double w = (bx ? fr[0] : 1.0 - fr[0]) * (by ? fr[1] : 1.0 - fr[1]) *
                             (bz ? fr[2] : 1.0 - fr[2]);
            const int tc = t0 + (bz * S + by) * S + bx;
            for (int comp = 0; comp < 3; ++comp) uf[comp] += w * (double)tile[comp * S3 + tc];
        }
    } else {
        t0 = ((cl[2] + 1) * S + (cl[1] + 1)) * S + (cl[0] + 1);
        for (int comp = 0; comp < 3; ++comp) uf[comp] = (double)tile[comp * S3 + t0];
    }

    // forward quantities of the step
    const double tau_s = p.tau_coef * dp * dp;
    const double slip[3] = {uf[0] - up[0], uf[1] - up[1], uf[2] - up[2]};
    const double s2 = slip[0] * slip[0] + slip[1] * slip[1] + slip[2] * slip[2];
    const double Re = p.drag == 1 ? p.re_coef * dp * sqrt(s2) : 0.0;
    const double f = p.drag == 1 ? 1.0 + 0.15 * pow(Re, 0.687) : 1.0;
    const double tau = p.drag == 1 ? tau_s / f : tau_s;
    const double mass = p.mass_coef * dp * dp * dp;
    const double invD = 1.0 / (tau + dt);
    const double dtD = dt * invD, tauD = tau * invD;

    // reverse
    const int cell = (cl[2] * E + cl[1]) * E + cl[0];
    double ub[3];
    double mbar = 0.0, taubar = 0.0;
    for (int ax = 0; ax < 3; ++ax) {
        const double upn = (tau * up[ax] + dt * uf[ax] + tau * dt * p.g[ax]) * invD;
        const double Jbar = -lam[ax * E3 + cell] * p.inv_V;
        const double wbar = rc[3 + ax] + dt * rc[ax] + mass * Jbar;
        mbar += Jbar * (upn - up[ax] - p.g[ax] * dt);
        ufb[ax] = dtD * wbar;
        taubar += wbar * (up[ax] + dt * p.g[ax] - upn);
        ub[ax] = -mass * Jbar + tauD * wbar;
    }
    taubar *= invD;
    double Rebar = 0.0;
    if (Re > 0.0) {
        Rebar = -taubar * tau / f * (0.15 * 0.687) * pow(Re, 0.687 - 1.0);
        for (int ax = 0; ax < 3; ++ax) {
            const double sb = Rebar * Re * slip[ax] / s2;
            ufb[ax] += sb;
            ub[ax] -= sb;
        }
    }
    if (TRI) {
        // the position adjoint: the weights' gradients (d/dx of 1 - f is
        // -1/h, of f 1/h) against dot_k = U_k . ufbar at each corner k, which
        // per axis is 1/h times the bilinear interpolation, over the other
        // two axes, of the corner differences along it
        double dot[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int tc = t0 + (((k >> 2) & 1) * S + ((k >> 1) & 1)) * S + (k & 1);
            dot[k] = 0.0;
            for (int comp = 0; comp < 3; ++comp) dot[k] += (double)tile[comp * S3 + tc] * ufb[comp];
        }
        auto lerp = [](double a, double b, double t) { return a + t * (b - a); };
        rc[0] += p.inv_h[0] * lerp(lerp(dot[1] - dot[0], dot[3] - dot[2], fr[1]),
                                   lerp(dot[5] - dot[4], dot[7] - dot[6], fr[1]), fr[2]);
        rc[1] += p.inv_h[1] * lerp(lerp(dot[2] - dot[0], dot[3] - dot[1], fr[0]),
                                   lerp(dot[6] - dot[4], dot[7] - dot[5], fr[0]), fr[2]);
        rc[2] += p.inv_h[2] * lerp(lerp(dot[4] - dot[0], dot[5] - dot[1], fr[0]),
                                   lerp(dot[6] - dot[2], dot[7] - dot[3], fr[0]), fr[1]);
    }
    for (int ax = 0; ax < 3; ++ax) rc[3 + ax] = ub[ax];
    rc[6] += (2.0 * taubar * tau + Rebar * Re + 3.0 * mbar * mass) / dp;
}

// Trilinear: one workgroup per work item.  Each thread reverses up to
// kAdjPPT particles per pass, their loads issued together (saved states and anchors
// first, then the records the anchors address), and adds each particle's
// eight weighted ufbar terms to the tile's node sums in LDS: each term formed
// in the state precision from the particle's stencil offsets and ufbar
// rounded to it, the sums kept in binary64 (LDS atomic adds).  Per chunk each
// node's sum goes to dL/du with one atomic add.
template <class T, int E>
__global__ void __launch_bounds__(kAdjBlock, 2) k_adjoint_tri(AdjArgs<T> a)
{
    constexpr int S = E + 2;
    constexpr int S3 = S * S * S;
    constexpr int E3 = E * E * E;
    constexpr int PPT = kAdjPPT;
    __shared__ T tile[3 * S3];
    __shared__ double nacc[3 * S3];           // node sums, [3][S3]

    const int64_t item = blockIdx.x;
    if (item >= *a.nitems) return;
    const Params &p = a.p;
    const int64_t c = a.items[2 * item], seg = a.items[2 * item + 1];
    const int64_t s0 = a.base[c] + seg * kSeg;
    const int64_t s1 = min(s0 + (int64_t)kSeg, a.base[c] + (int64_t)a.cnt[c]);
    const int cx = (int)(c % p.nc[0]);
    const int cy = (int)((c / p.nc[0]) % p.nc[1]);
    const int cz = (int)(c / ((int64_t)p.nc[0] * p.nc[1]));
    const int64_t ncell = (int64_t)p.n[0] * p.n[1] * p.n[2];

    // a chunk that is one work item is this workgroup's alone: its node sums
    // continue those of the steps reversed before (kept per chunk), and go
    // back to them at the end; a chunk split over several items adds its
    // sums to dL/du atomically
    const bool own = a.tacc != nullptr && a.cnt[c] <= kSeg;
    double *const tacc_c = own ? a.tacc + c * 3 * S3 : nullptr;
    stage_tile<T, E, kAdjBlock>(p, a.u, cx, cy, cz, tile);
    for (int t = threadIdx.x; t < 3 * S3; t += kAdjBlock) nacc[t] = own ? tacc_c[t] : 0.0;
    __syncthreads();
    const double *lam = a.lamC + c * 3 * E3;

    // a thread takes the slots s0 + threadIdx.x + j kAdjBlock, PPT values of
    // j per pass; in binary32 the odd waves take a single one in their first
    // pass, so that the waves' loads and LDS atomics fall out of step
    const bool shift = sizeof(T) == 4 && ((threadIdx.x >> 6) & 1);
    for (int64_t j = 0, first = 1; s0 + j * kAdjBlock < s1; first = 0) {
        const int np = (first && shift) ? 1 : PPT;
        const int64_t q0 = s0 + j * kAdjBlock;
        j += np;
        int64_t an[PPT];
        T st[PPT][7];
        double rc[PPT][7];
#pragma unroll
        for (int u = 0; u < PPT; ++u) {
            const int64_t q = q0 + threadIdx.x + (int64_t)u * kAdjBlock;
            an[u] = -1;
            if (u < np && q < s1) {
                an[u] = a.id[q];
                st[u][0] = a.ox[q];
                st[u][1] = a.oy[q];
                st[u][2] = a.oz[q];
                st[u][3] = a.vx[q];
                st[u][4] = a.vy[q];
                st[u][5] = a.vz[q];
                st[u][6] = a.d[q];
            }
        }
        bool live[PPT];
#pragma unroll
        for (int u = 0; u < PPT; ++u) {
            live[u] = adj_live(an[u], a.nrec, st[u]);
            if (live[u])
                for (int k = 0; k < 7; ++k) rc[u][k] = (double)a.adj[8 * an[u] + k];
        }
#pragma unroll
        for (int u = 0; u < PPT; ++u) {
            if (!live[u]) continue;
            double ufb[3], fr[3];
            int i0[3], t0;
            reverse_particle<T, E, true>(p, a.dt, tile, lam, st[u], rc[u], ufb, i0, fr, t0);
            T *rec = a.adj + 8 * an[u];
            for (int k = 0; k < 7; ++k) rec[k] = (T)rc[u][k];
            const T f[3] = {(T)fr[0], (T)fr[1], (T)fr[2]};
            const T ub[3] = {(T)ufb[0], (T)ufb[1], (T)ufb[2]};
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int bx = k & 1, by = (k >> 1) & 1, bz = k >> 2;
                const T wk = (bx ? f[0] : T(1) - f[0]) * (by ? f[1] : T(1) - f[1]) *
                             (bz ? f[2] : T(1) - f[2]);
                const int tc = t0 + (bz * S + by) * S + bx;
#pragma unroll
                for (int comp = 0; comp < 3; ++comp)
                    atomicAdd(&nacc[comp * S3 + tc], (double)(wk * ub[comp]));
            }
        }
    }
    __syncthreads();
    if (own) {
        for (int t = threadIdx.x; t < 3 * S3; t += kAdjBlock) tacc_c[t] = nacc[t];
        return;
    }
    for (int n = threadIdx.x; n < S3; n += kAdjBlock) {
        const int64_t g = tile_cell<E>(p, cx, cy, cz, n);
        for (int comp = 0; comp < 3; ++comp) {
            const double v = nacc[comp * S3 + n];
            if (v != 0.0) atomicAdd(a.Ubar + comp * ncell + g, v);
        }
    }
}

// The per-chunk tile sums into dL/du, one atomic add per nonzero node and
// component (after the last reversed step).
template <int E>
__global__ void k_fold_tiles(const double *tacc, Params p, int64_t C, double *Ubar)
{
    constexpr int S = E + 2;
    constexpr int S3 = S * S * S;
    const int64_t ncell = (int64_t)p.n[0] * p.n[1] * p.n[2];
    for (int64_t c = blockIdx.x; c < C; c += gridDim.x) {
        const int cx = (int)(c % p.nc[0]);
        const int cy = (int)((c / p.nc[0]) % p.nc[1]);
        const int cz = (int)(c / ((int64_t)p.nc[0] * p.nc[1]));
        for (int n = threadIdx.x; n < S3; n += blockDim.x) {
            const int64_t g = tile_cell<E>(p, cx, cy, cz, n);
            for (int comp = 0; comp < 3; ++comp) {
                const double v = tacc[(c * 3 + comp) * S3 + n];
                if (v != 0.0) atomicAdd(Ubar + comp * ncell + g, v);
            }
        }
    }
}

// Nearest grid point: the reverse of each particle adds its ufbar to its
// cell of the tile with one LDS atomic per component, in the state
// precision; per chunk each tile cell's sum goes to the chunk's binary64 tile
// sums (or, for a chunk split over several items, to dL/du with one atomic).
template <class T, int E>
__global__ void __launch_bounds__(kAdjBlock) k_adjoint_ngp(AdjArgs<T> a)
{
    constexpr int S = E + 2;
    constexpr int S3 = S * S * S;
    constexpr int E3 = E * E * E;
    __shared__ T tile[3 * S3];
    __shared__ T ubt[3 * S3];

    const int64_t item = blockIdx.x;
    if (item >= *a.nitems) return;
    const Params &p = a.p;
    const int64_t c = a.items[2 * item], seg = a.items[2 * item + 1];
    const int64_t s0 = a.base[c] + seg * kSeg;
    const int64_t s1 = min(s0 + (int64_t)kSeg, a.base[c] + (int64_t)a.cnt[c]);
    const int cx = (int)(c % p.nc[0]);
    const int cy = (int)((c / p.nc[0]) % p.nc[1]);
    const int cz = (int)(c / ((int64_t)p.nc[0] * p.nc[1]));
    const int64_t ncell = (int64_t)p.n[0] * p.n[1] * p.n[2];

    stage_tile<T, E, kAdjBlock>(p, a.u, cx, cy, cz, tile);
    for (int t = threadIdx.x; t < 3 * S3; t += kAdjBlock) ubt[t] = T(0);
    __syncthreads();
    const double *lam = a.lamC + c * 3 * E3;
    for (int64_t q = s0 + threadIdx.x; q < s1; q += kAdjBlock) {
        const int64_t an = a.id[q];
        const T st[7] = {a.ox[q], a.oy[q], a.oz[q], a.vx[q], a.vy[q], a.vz[q], a.d[q]};
        if (!adj_live(an, a.nrec, st)) continue;
        double rc[7];
        for (int k = 0; k < 7; ++k) rc[k] = (double)a.adj[8 * an + k];
        double ufb[3], fr[3];
        int i0[3], t0;
        reverse_particle<T, E, false>(p, a.dt, tile, lam, st, rc, ufb, i0, fr, t0);
        for (int comp = 0; comp < 3; ++comp) atomicAdd(&ubt[comp * S3 + t0], (T)ufb[comp]);
        T *rec = a.adj + 8 * an;
        for (int k = 0; k < 7; ++k) rec[k] = (T)rc[k];
    }
    __syncthreads();
    // a chunk that is one work item adds its sums to those it keeps over the
    // steps; a chunk split over several items adds them to dL/du atomically
    const bool own = a.tacc != nullptr && a.cnt[c] <= kSeg;
    for (int t = threadIdx.x; t < 3 * S3; t += kAdjBlock) {
        const double v = (double)ubt[t];
        if (own) {
            a.tacc[c * 3 * S3 + t] += v;
        } else if (v != 0.0) {
            const int comp = t / S3;
            atomicAdd(a.Ubar + comp * ncell + tile_cell<E>(p, cx, cy, cz, t - comp * S3), v);
        }
    }
}

// dL/dSu_int from the field layout into the chunk layout
__global__ void k_lambda_to_chunks(const double *lam, Params p, double *lamC)
{
    const int64_t nx = p.n[0], ny = p.n[1], nz = p.n[2];
    const int64_t ncell = nx * ny * nz;
    const int E = p.E;
    const int64_t E3 = (int64_t)E * E * E;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < 3 * ncell;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t comp = t / ncell, r = t - comp * ncell;
        const int64_t i = r % nx, j = (r / nx) % ny, k = r / (nx * ny);
        const int64_t c = ((k / E) * p.nc[1] + (j / E)) * p.nc[0] + (i / E);
        const int64_t l = ((k % E) * E + (j % E)) * E + (i % E);
        lamC[c * 3 * E3 + comp * E3 + l] = lam[t];
    }
}

__global__ void k_zero_f64(double *p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

inline int64_t grid_of(int64_t n)
{
    const int64_t g = (n + 255) / 256;
    return g < 1 ? 1 : (g > 16384 ? 16384 : g);
}

// A checkpoint slot holds a particle when it lies in its chunk's run
// [base, base + cnt), its id is in [0, count) and it is not a hole (a hole
// keeps the id of the particle that left it; slots past the runs may hold
// stale copies of particles).
template <class T>
__device__ __forceinline__ bool ck_particle(int32_t id, int64_t count, T ox, T d)
{
    return id >= 0 && id < count && ox >= T(0) && d > T(0);
}

// The checkpoint's particles, a workgroup per chunk.  Mode bits: kAnchor
// replaces the restored store's ids by anchors (every other slot of a run
// gets -1), kToAnchor takes each particle's record from the array by id into
// the array by anchor, kToId puts it back.  With a second checkpoint (ok,
// the neighbouring segment's), only the particles that it does not hold at
// the same slot of the same chunk's run move: their records change place
// between the two segments' arrays by anchor, which are one array, so the
// others' records are already where the next segment reads them.
constexpr int kAnchor = 1, kToAnchor = 2, kToId = 4;
template <class T>
__global__ void k_checkpoint_records(const char *ck, const char *ok, SnapLayout L, int64_t slots,
                                     int64_t C, int64_t count, int32_t *store_id, T *by_id,
                                     T *rec, int mode)
{
    const T *ox = reinterpret_cast<const T *>(ck + L.state);
    const T *d = ox + 6 * slots;
    const int32_t *sid = reinterpret_cast<const int32_t *>(ck + L.id);
    const int64_t *base = reinterpret_cast<const int64_t *>(ck + L.base);
    const int32_t *cnt = reinterpret_cast<const int32_t *>(ck + L.cnt);
    const char *const oc = ok ? ok : ck;   // (not read without ok)
    const T *o_ox = reinterpret_cast<const T *>(oc + L.state);
    const T *o_d = o_ox + 6 * slots;
    const int32_t *o_sid = reinterpret_cast<const int32_t *>(oc + L.id);
    const int64_t *o_base = reinterpret_cast<const int64_t *>(oc + L.base);
    const int32_t *o_cnt = reinterpret_cast<const int32_t *>(oc + L.cnt);
    for (int64_t c = blockIdx.x; c < C; c += gridDim.x) {
        const int64_t q0 = base[c], q1 = q0 + cnt[c];
        const int64_t p0 = ok ? o_base[c] : 0, p1 = ok ? p0 + o_cnt[c] : 0;
        for (int64_t q = q0 + threadIdx.x; q < q1; q += blockDim.x) {
            const int32_t k = sid[q];
            const bool live = ck_particle(k, count, ox[q], d[q]);
            if (mode & kAnchor) store_id[q] = live ? (int32_t)q : -1;
            if (!live || !(mode & (kToAnchor | kToId))) continue;
            if (ok && q >= p0 && q < p1 && o_sid[q] == k && ck_particle(k, count, o_ox[q], o_d[q]))
                continue;   // the same slot in both
            // a record is 8 T: sizeof(T) / 2 pieces of 16 bytes
            constexpr int NV = (int)sizeof(T) / 2;
            double2 *ra = reinterpret_cast<double2 *>(rec + 8 * q);
            double2 *rb = reinterpret_cast<double2 *>(by_id + 8 * (int64_t)k);
            double2 v[NV];
            if (mode & kToAnchor) {
                for (int j = 0; j < NV; ++j) v[j] = rb[j];
                for (int j = 0; j < NV; ++j) ra[j] = v[j];
            } else {
                for (int j = 0; j < NV; ++j) v[j] = ra[j];
                for (int j = 0; j < NV; ++j) rb[j] = v[j];
            }
        }
    }
}

template <class T>
hipError_t launch_checkpoint_records(st_ctx *c, const char *ck, const char *ok, T *by_id,
                                     T *rec, int mode, hipStream_t s)
{
    const SnapLayout L = snap_layout(c->slots, c->tsize, c->C, c->max_items);
    const int64_t g = c->C < 16384 ? c->C : 16384;
    hipLaunchKernelGGL((k_checkpoint_records<T>), dim3(g > 0 ? g : 1), dim3(256), 0, s, ck, ok,
                       L, c->slots, c->C, c->count, (int32_t *)c->store[0][7], by_id, rec, mode);
    return hipGetLastError();
}

// dL/dd of every particle out of the adjoint records by id
template <class T>
__global__ void k_take_dbar(const T *adj, int64_t P, double *dd)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < P;
         i += (int64_t)gridDim.x * blockDim.x)
        dd[i] = (double)adj[8 * i + 6];
}


template <class T>
AdjArgs<T> adj_args(st_ctx *c, const char *snap, const TapeStep &ts, const double *lamC,
                    T *adj, double *Ubar, double *tacc)
{
    AdjArgs<T> a;
    if (snap) {
        const SnapLayout L = snap_layout(c->slots, c->tsize, c->C, c->max_items);
        const T *st = reinterpret_cast<const T *>(snap + L.state);
        a.ox = st;
        a.oy = st + c->slots;
        a.oz = st + 2 * c->slots;
        a.vx = st + 3 * c->slots;
        a.vy = st + 4 * c->slots;
        a.vz = st + 5 * c->slots;
        a.d = st + 6 * c->slots;
        a.id = reinterpret_cast<const int32_t *>(snap + L.id);
        a.base = reinterpret_cast<const int64_t *>(snap + L.base);
        a.cnt = reinterpret_cast<const int32_t *>(snap + L.cnt);
        a.items = reinterpret_cast<const int32_t *>(snap + L.items);
        a.nitems = reinterpret_cast<const int32_t *>(snap + L.nitems);
    } else {   // the store itself, with its layout and work items
        a.ox = (const T *)c->store[0][0];
        a.oy = (const T *)c->store[0][1];
        a.oz = (const T *)c->store[0][2];
        a.vx = (const T *)c->store[0][3];
        a.vy = (const T *)c->store[0][4];
        a.vz = (const T *)c->store[0][5];
        a.d = (const T *)c->store[0][6];
        a.id = (const int32_t *)c->store[0][7];
        a.base = c->base;
        a.cnt = c->cnt;
        a.items = c->items;
        a.nitems = c->flags + F_NITEMS;
    }
    a.u = reinterpret_cast<const T *>(ts.u);
    a.lamC = lamC;
    a.adj = adj;
    a.Ubar = Ubar;
    a.tacc = tacc;
    a.nrec = c->slots;
    a.p = c->prm;
    a.dt = ts.dt;
    return a;
}

template <class T>
hipError_t launch_adjoint_step(st_ctx *c, const AdjArgs<T> &a, hipStream_t s)
{
    const dim3 g(c->max_items), b(kAdjBlock);
    const bool ngp = c->prm.interp == 1;
    switch (c->prm.E) {
    case 2:
        if (ngp) hipLaunchKernelGGL((k_adjoint_ngp<T, 2>), g, b, 0, s, a);
        else hipLaunchKernelGGL((k_adjoint_tri<T, 2>), g, b, 0, s, a);
        break;
    case 4:
        if (ngp) hipLaunchKernelGGL((k_adjoint_ngp<T, 4>), g, b, 0, s, a);
        else hipLaunchKernelGGL((k_adjoint_tri<T, 4>), g, b, 0, s, a);
        break;
    default:
        if (ngp) hipLaunchKernelGGL((k_adjoint_ngp<T, 8>), g, b, 0, s, a);
        else hipLaunchKernelGGL((k_adjoint_tri<T, 8>), g, b, 0, s, a);
        break;
    }
    return hipGetLastError();
}

}  // namespace

namespace {

// One workspace, kept in the context for the next call: the state the
// forward run ended in, the saved states of one segment (K - 1 steps; the
// newest is the store itself), dL/dS by chunk, the adjoint records by id and
// those of the current segment by anchor, and the per-chunk tile sums of
// dL/du when they fit in a GiB (else each step adds its sums to dL/du
// atomically).
struct BwdLayout {
    size_t step_bytes, o_steps, o_lam, o_rid, o_adj, o_tacc, tbytes, bytes;
};

BwdLayout bwd_layout(const st_ctx *c, int64_t K)
{
    auto up256 = [](size_t v) { return (v + 255) & ~(size_t)255; };
    const int64_t P = c->count;
    const int64_t E3 = (int64_t)c->prm.E * c->prm.E * c->prm.E;
    const int64_t S3 = (int64_t)(c->prm.E + 2) * (c->prm.E + 2) * (c->prm.E + 2);
    const size_t rbytes = 8 * c->tsize;   // a record: eight state-precision values
    BwdLayout W;
    W.step_bytes = up256(snapshot_bytes(c));
    W.o_steps = W.step_bytes;
    W.o_lam = W.o_steps + (size_t)(K > 1 ? K - 1 : 0) * W.step_bytes;
    W.o_rid = W.o_lam + up256((size_t)c->C * 3 * E3 * 8);
    W.o_adj = W.o_rid + up256((size_t)(P > 0 ? P : 1) * rbytes);
    W.o_tacc = W.o_adj + up256((size_t)c->slots * rbytes);
    W.tbytes = (size_t)c->C * 3 * S3 * 8;
    if (W.tbytes > ((size_t)1 << 30)) W.tbytes = 0;
    W.bytes = W.o_tacc + W.tbytes;
    return W;
}

hipError_t ensure_bwd_workspace(st_ctx *c, const BwdLayout &W)
{
    if (c->bwd_ws_bytes >= W.bytes) return hipSuccess;
    (void)hipFree(c->bwd_ws);
    c->bwd_ws = nullptr;
    c->bwd_ws_bytes = 0;
    hipError_t e = hipMalloc(&c->bwd_ws, W.bytes);
    if (e != hipSuccess) return e;
    c->bwd_ws_bytes = W.bytes;
    return hipSuccess;
}

}  // namespace

hipError_t reserve_backward(st_ctx *c, int64_t K)
{
    if (K <= 0) return hipErrorInvalidValue;
    return ensure_bwd_workspace(c, bwd_layout(c, K));
}

hipError_t launch_backward(st_ctx *c, const double *lam, double *dU, double *dd, hipStream_t s)
{
    const int64_t ntape = (int64_t)c->tape.size();
    const int64_t K = c->tape_every;
    const int64_t nseg = (int64_t)c->snaps.size();
    if (ntape == 0 || K <= 0 || nseg != (ntape + K - 1) / K) return hipErrorInvalidValue;
    const int64_t P = c->count;
    const int64_t ncell = (int64_t)c->prm.n[0] * c->prm.n[1] * c->prm.n[2];

    const BwdLayout W = bwd_layout(c, K);
    hipError_t e0 = ensure_bwd_workspace(c, W);
    if (e0 != hipSuccess) return e0;
    char *ws = (char *)c->bwd_ws;
    void *final_state = ws;
    auto step_buf = [&](int64_t k) -> void * { return ws + W.o_steps + (size_t)k * W.step_bytes; };
    double *lamC = (double *)(ws + W.o_lam);
    void *rid = ws + W.o_rid;
    void *adj = ws + W.o_adj;
    double *tacc = W.tbytes ? (double *)(ws + W.o_tacc) : nullptr;
    const bool fp64 = c->form == ST_FORM_FP64;

    // an error return first drains the stream
    auto fail = [&](hipError_t err) {
        (void)hipStreamSynchronize(s);
        return err;
    };
    // keep the state the forward run ended in
    hipError_t e = launch_snapshot(c, final_state, 0, s);
    if (e != hipSuccess) return fail(e);
    hipLaunchKernelGGL(k_lambda_to_chunks, dim3(grid_of(3 * ncell)), dim3(256), 0, s, lam, c->prm,
                       lamC);
    hipLaunchKernelGGL(k_zero_f64, dim3(grid_of(3 * ncell)), dim3(256), 0, s, dU, 3 * ncell);
    if (tacc)
        hipLaunchKernelGGL(k_zero_f64, dim3(grid_of((int64_t)(W.tbytes / 8))), dim3(256), 0, s,
                           tacc, (int64_t)(W.tbytes / 8));
    hipLaunchKernelGGL(k_zero_f64, dim3(grid_of(P * (int64_t)c->tsize)), dim3(256), 0, s,
                       (double *)rid, P * (int64_t)c->tsize);
    e = hipGetLastError();
    if (e != hipSuccess) return fail(e);

    for (int64_t sg = nseg - 1; sg >= 0; --sg) {
        const int64_t k0 = sg * K, k1 = std::min(k0 + K, ntape);
        // the checkpoint, with anchors in place of its ids, and the records of
        // its particles by anchor (those the later checkpoint held at the
        // same slot are there already)
        const char *ck = (const char *)c->snaps[(size_t)sg].buf;
        const char *later = sg + 1 < nseg ? (const char *)c->snaps[(size_t)sg + 1].buf : nullptr;
        const char *earlier = sg > 0 ? (const char *)c->snaps[(size_t)sg - 1].buf : nullptr;
        e = launch_snapshot(c, c->snaps[(size_t)sg].buf, 1, s);
        if (e != hipSuccess) return fail(e);
        e = fp64 ? launch_checkpoint_records<double>(c, ck, later, (double *)rid, (double *)adj,
                                                     kAnchor | kToAnchor, s)
                 : launch_checkpoint_records<float>(c, ck, later, (float *)rid, (float *)adj,
                                                    kAnchor | kToAnchor, s);
        if (e != hipSuccess) return fail(e);
        // recompute the segment, each step saving what its reverse reads; the
        // last step's start is the store itself, reversed from there
        for (int64_t k = k0; k + 1 < k1; ++k) {
            e = launch_step(c, c->tape[(size_t)k].u, c->tape[(size_t)k].dt, 0, s, step_buf(k - k0));
            if (e != hipSuccess) return fail(e);
        }
        // and reverse it, newest step first
        for (int64_t k = k1 - 1; k >= k0; --k) {
            const char *snap = k + 1 < k1 ? (const char *)step_buf(k - k0) : nullptr;
            if (fp64)
                e = launch_adjoint_step<double>(
                    c, adj_args<double>(c, snap, c->tape[(size_t)k], lamC, (double *)adj, dU,
                                          tacc), s);
            else
                e = launch_adjoint_step<float>(
                    c, adj_args<float>(c, snap, c->tape[(size_t)k], lamC, (float *)adj, dU,
                                         tacc), s);
            if (e != hipSuccess) return fail(e);
        }
        // the records of the particles the earlier checkpoint does not hold at
        // the same slot (after the first segment, all) go to the array by id
        e = fp64 ? launch_checkpoint_records<double>(c, ck, earlier, (double *)rid, (double *)adj,
                                                     kToId, s)
                 : launch_checkpoint_records<float>(c, ck, earlier, (float *)rid, (float *)adj,
                                                    kToId, s);
        if (e != hipSuccess) return fail(e);
    }
    if (tacc) {
        const dim3 g(std::min<int64_t>(c->C, 16384));
        switch (c->prm.E) {
        case 2: hipLaunchKernelGGL(k_fold_tiles<2>, g, dim3(256), 0, s, tacc, c->prm, c->C, dU); break;
        case 4: hipLaunchKernelGGL(k_fold_tiles<4>, g, dim3(256), 0, s, tacc, c->prm, c->C, dU); break;
        default: hipLaunchKernelGGL(k_fold_tiles<8>, g, dim3(256), 0, s, tacc, c->prm, c->C, dU); break;
        }
    }
    if (fp64)
        hipLaunchKernelGGL(k_take_dbar<double>, dim3(grid_of(P)), dim3(256), 0, s,
                           (const double *)rid, P, dd);
    else
        hipLaunchKernelGGL(k_take_dbar<float>, dim3(grid_of(P)), dim3(256), 0, s,
                           (const float *)rid, P, dd);
    e = hipGetLastError();
    if (e != hipSuccess) return fail(e);
    e = launch_snapshot(c, final_state, 1, s);
    if (e != hipSuccess) return fail(e);
    // the tape's buffers are handed back when this returns: finish first
    return hipStreamSynchronize(s);
}

}  // namespace st
