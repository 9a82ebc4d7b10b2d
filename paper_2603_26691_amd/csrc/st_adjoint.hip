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
// them, and then reversed newest first.
// The per-particle adjoint state is kept by particle id, so the re-binning
// between steps needs no special treatment.
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
    int64_t grid;
    const T *u;              // field of the step [3][n2][n1][n0]
    const double *lamC;      // dL/dSu_int by chunk [C][3][E^3]
    double *adj;             // adjoint state by id, [P][8]: xbar[3], ubar[3], dbar, unused
    double *Ubar;            // dL/du [3][n2][n1][n0]
    int64_t count;
    Params p;
    double dt;
};

// One workgroup of 512 threads per work item, two per CU.
constexpr int kAdjBlock = 256;

// Block-wide exclusive scan of one value per thread (kAdjBlock threads);
// returns the prefix and the block total.
__device__ int32_t adj_block_scan(int32_t v, int32_t &total)
{
    __shared__ int32_t ws[kAdjBlock / 64];
    const int lane = __lane_id(), wave = threadIdx.x >> 6;
    int32_t incl = v;
    for (int o = 1; o < 64; o <<= 1) {
        const int32_t y = __shfl_up(incl, o);
        if (lane >= o) incl += y;
    }
    if (lane == 63) ws[wave] = incl;
    __syncthreads();
    int32_t before = 0;
    total = 0;
    for (int k = 0; k < kAdjBlock / 64; ++k) {
        if (k < wave) before += ws[k];
        total += ws[k];
    }
    __syncthreads();
    return before + incl - v;
}

// Particles per batch of the trilinear scatter (their stencil offsets and
// ufbar wait in LDS, in the state precision, ordered by stencil base): about
// 70 KB of LDS per workgroup in either form, so that two workgroups share a
// CU.
template <class T>
constexpr int adj_batch() { return sizeof(T) == 4 ? 1024 : 256; }

template <class T, int E, int INTERP>
__global__ void __launch_bounds__(kAdjBlock) k_adjoint_step(AdjArgs<T> a)
{
    constexpr int S = E + 2;
    constexpr int S3 = S * S * S;
    constexpr int E3 = E * E * E;
    constexpr int E1 = E + 1;
    constexpr int NB = E1 * E1 * E1;        // trilinear stencil bases (lowest corners)
    constexpr int B = adj_batch<T>();
    constexpr bool TRI = INTERP == 0;
    __shared__ T tile[3 * S3];
    // Nearest grid point: Ubar over the tile, summed in the state precision
    // with one atomic per particle and component.
    __shared__ T ubt[TRI ? 1 : 3 * S3];
    // Trilinear: the reverse of the gather is a scatter to 8 corners.  Instead
    // of 24 LDS atomics per particle (measured to dominate the kernel), the
    // particles of a batch are ordered by stencil base and every thread sums
    // the contributions to the tile nodes it owns, in binary64.
    __shared__ double nacc[TRI ? 3 * S3 : 1];     // node sums, [3][S3]
    __shared__ T rf[TRI ? 3 * B : 1];             // fractional offsets f
    __shared__ T ru[TRI ? 3 * B : 1];             // ufbar
    __shared__ int32_t rb[TRI ? B : 1];           // base | rank in it << 12, -1 for none
    __shared__ int32_t perm[TRI ? B : 1];         // batch entries by base
    __shared__ int32_t bstart[TRI ? NB + 1 : 1];  // first entry of each base
    __shared__ int32_t bcur[TRI ? NB : 1];        // entries per base

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
    const int ox0 = cx * E - 1, oy0 = cy * E - 1, oz0 = cz * E - 1;

    auto tile_cell = [&](int r) -> int64_t {  // field index of tile cell r
        const int k = r / (S * S), j = (r / S) % S, i = r % S;
        int gx = ox0 + i, gy = oy0 + j, gz = oz0 + k;
        gx += gx < 0 ? p.n[0] : 0;
        gx -= gx >= p.n[0] ? p.n[0] : 0;
        gy += gy < 0 ? p.n[1] : 0;
        gy -= gy >= p.n[1] ? p.n[1] : 0;
        gz += gz < 0 ? p.n[2] : 0;
        gz -= gz >= p.n[2] ? p.n[2] : 0;
        return ((int64_t)gz * p.n[1] + gy) * p.n[0] + gx;
    };
    // the tile's loads are all issued before the first is used
    {
        constexpr int NT = (3 * S3 + kAdjBlock - 1) / kAdjBlock;
        T vals[NT];
#pragma unroll
        for (int u = 0; u < NT; ++u) {
            const int t = threadIdx.x + u * kAdjBlock;
            if (t < 3 * S3) {
                const int comp = t / S3;
                vals[u] = a.u[comp * ncell + tile_cell(t - comp * S3)];
            }
        }
#pragma unroll
        for (int u = 0; u < NT; ++u) {
            const int t = threadIdx.x + u * kAdjBlock;
            if (t < 3 * S3) {
                tile[t] = vals[u];
                if (TRI) nacc[t] = 0.0;
                else ubt[t] = T(0);
            }
        }
    }
    __syncthreads();

    const double dt = a.dt;
    const double inv_V = p.inv_V;
    const double *lam = a.lamC + c * 3 * E3;
    const int64_t run = TRI ? (int64_t)B : s1 - s0;   // NGP: the whole range at once
    for (int64_t q0 = s0; q0 < s1; q0 += run) {
        const int64_t q1 = min(q0 + run, s1);
        if (TRI) {
            for (int b = threadIdx.x; b < NB; b += kAdjBlock) bcur[b] = 0;
            __syncthreads();
        }
        // a thread's particles of the batch (PPT of them) load first: ids and
        // saved states, then the adjoint records the ids address
        constexpr int PPT = TRI ? 2 : 1;
        for (int64_t qb = q0 + threadIdx.x; qb < q1; qb += (int64_t)PPT * kAdjBlock) {
        int64_t idv[PPT];
        T ls[PPT][7];
        double lr[PPT][7];
#pragma unroll
        for (int u = 0; u < PPT; ++u) {
            const int64_t q = qb + (int64_t)u * kAdjBlock;
            idv[u] = -1;
            if (q < q1) {
                idv[u] = a.id[q];
                ls[u][0] = a.ox[q];
                ls[u][1] = a.oy[q];
                ls[u][2] = a.oz[q];
                ls[u][3] = a.vx[q];
                ls[u][4] = a.vy[q];
                ls[u][5] = a.vz[q];
                ls[u][6] = a.d[q];
            }
        }
#pragma unroll
        for (int u = 0; u < PPT; ++u)
            if (idv[u] >= 0 && idv[u] < a.count && ls[u][0] >= T(0) && ls[u][6] > T(0))
                for (int k = 0; k < 7; ++k) lr[u][k] = a.adj[8 * idv[u] + k];
#pragma unroll
        for (int u = 0; u < PPT; ++u) {
            const int64_t q = qb + (int64_t)u * kAdjBlock;
            if (q >= q1) continue;
            const int jb = (int)(q - q0);   // entry in the batch
            const int64_t id = idv[u];
            // a hole: a -1 offset (binary32) or a negated diameter (binary64)
            if (id < 0 || id >= a.count || !(ls[u][0] >= T(0) && ls[u][6] > T(0))) {
                if (TRI) rb[jb] = -1;
                continue;
            }
            const double xi[3] = {(double)ls[u][0], (double)ls[u][1], (double)ls[u][2]};
            const double up[3] = {(double)ls[u][3], (double)ls[u][4], (double)ls[u][5]};
            const double dp = (double)ls[u][6];

            // interpolation stencil in binary64 at the saved position
            int cl[3], i0[3];
            double om[3][2], dom[3][2];
            for (int ax = 0; ax < 3; ++ax) {
                cl[ax] = min(max((int)xi[ax], 0), E - 1);
                if (TRI) {
                    const double s = xi[ax] - 0.5;
                    const double fl = floor(s);
                    i0[ax] = min(max((int)fl, -1), E - 1);
                    const double f = s - fl;
                    om[ax][0] = 1.0 - f;
                    om[ax][1] = f;
                    dom[ax][0] = -p.inv_h[ax];
                    dom[ax][1] = p.inv_h[ax];
                }
            }
            double uf[3] = {0.0, 0.0, 0.0};
            int tc[8];
            double w[8];
            int nk;
            if (TRI) {
                nk = 8;
                const int t0 = ((i0[2] + 1) * S + (i0[1] + 1)) * S + (i0[0] + 1);
                for (int k = 0; k < 8; ++k) {
                    const int bx = k & 1, by = (k >> 1) & 1, bz = (k >> 2) & 1;
                    tc[k] = t0 + (bz * S + by) * S + bx;
                    w[k] = om[0][bx] * om[1][by] * om[2][bz];
                }
            } else {
                nk = 1;
                tc[0] = ((cl[2] + 1) * S + (cl[1] + 1)) * S + (cl[0] + 1);
                w[0] = 1.0;
            }
            for (int k = 0; k < nk; ++k)
                for (int comp = 0; comp < 3; ++comp)
                    uf[comp] += w[k] * (double)tile[comp * S3 + tc[k]];

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
            double upn[3];
            for (int ax = 0; ax < 3; ++ax)
                upn[ax] = (tau * up[ax] + dt * uf[ax] + tau * dt * p.g[ax]) * invD;

            // reverse
            const int cell = (cl[2] * E + cl[1]) * E + cl[0];
            double xb[3], ub[3], ufb[3];
            double mbar = 0.0, taubar = 0.0;
            double *rec = a.adj + 8 * id;   // one 64-byte record per particle
            for (int ax = 0; ax < 3; ++ax) {
                xb[ax] = lr[u][ax];
                ub[ax] = lr[u][3 + ax];
            }
            for (int ax = 0; ax < 3; ++ax) {
                const double Jbar = -lam[ax * E3 + cell] * inv_V;
                const double wbar = ub[ax] + dt * xb[ax] + mass * Jbar;
                mbar += Jbar * (upn[ax] - up[ax] - p.g[ax] * dt);
                ufb[ax] = dtD * wbar;
                taubar += wbar * (up[ax] + dt * p.g[ax] - upn[ax]);
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
            for (int k = 0; k < nk; ++k) {
                double dot = 0.0;
                for (int comp = 0; comp < 3; ++comp) {
                    if (!TRI) atomicAdd(&ubt[comp * S3 + tc[k]], (T)(w[k] * ufb[comp]));
                    dot += (double)tile[comp * S3 + tc[k]] * ufb[comp];
                }
                if (TRI) {
                    const int bx = k & 1, by = (k >> 1) & 1, bz = (k >> 2) & 1;
                    xb[0] += dom[0][bx] * om[1][by] * om[2][bz] * dot;
                    xb[1] += om[0][bx] * dom[1][by] * om[2][bz] * dot;
                    xb[2] += om[0][bx] * om[1][by] * dom[2][bz] * dot;
                }
            }
            if (TRI) {
                // the scatter waits for the batch: base, offsets and ufbar
                const int b = ((i0[2] + 1) * E1 + (i0[1] + 1)) * E1 + (i0[0] + 1);
                for (int ax = 0; ax < 3; ++ax) {
                    rf[ax * B + jb] = (T)om[ax][1];
                    ru[ax * B + jb] = (T)ufb[ax];
                }
                rb[jb] = b | (atomicAdd(&bcur[b], 1) << 12);
            }
            for (int ax = 0; ax < 3; ++ax) {
                rec[ax] = xb[ax];
                rec[3 + ax] = ub[ax];
            }
            rec[6] = lr[u][6] + (2.0 * taubar * tau + Rebar * Re + 3.0 * mbar * mass) / dp;
        }
        }
        if (!TRI) break;

        // order the batch by stencil base (a counting sort in LDS) ...
        __syncthreads();
        {
            constexpr int PER = (NB + kAdjBlock - 1) / kAdjBlock;
            int32_t v[PER];
            int32_t sum = 0;
#pragma unroll
            for (int k = 0; k < PER; ++k) {
                const int b = threadIdx.x * PER + k;
                v[k] = b < NB ? bcur[b] : 0;
                sum += v[k];
            }
            int32_t total;
            int32_t ex = adj_block_scan(sum, total);
#pragma unroll
            for (int k = 0; k < PER; ++k) {
                const int b = threadIdx.x * PER + k;
                if (b < NB) bstart[b] = ex;
                ex += v[k];
            }
            if (threadIdx.x == 0) bstart[NB] = total;
        }
        __syncthreads();
        for (int jb = threadIdx.x; jb < (int)(q1 - q0); jb += kAdjBlock) {
            const int32_t w = rb[jb];
            if (w >= 0) perm[bstart[w & 4095] + (w >> 12)] = jb;
        }
        __syncthreads();
        // ... and let every node gather from the (up to 8) bases whose stencil
        // holds it: node = base + (bx, by, bz), weight prod over the axes of
        // f (offset 1) or 1 - f (offset 0)
        for (int n = threadIdx.x; n < S3; n += kAdjBlock) {   // nodes owned by this thread
            const int nx = n % S, ny = (n / S) % S, nz = n / (S * S);
            // per row (by, bz) of bases the node's x-neighbours nx - 1 (offset
            // 1) and nx (offset 0) are adjacent bases, so their entries are
            // one range [lo, hi), split at mid; all 12 bounds load first
            const int xa = max(nx - 1, 0), xl = min(nx, E);
            int lo[4], mid[4], hi[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int y = ny - (k & 1), z = nz - (k >> 1);
                const bool ok = y >= 0 && z >= 0 && y <= E && z <= E;
                const int row = (z * E1 + y) * E1;
                lo[k] = ok ? bstart[row + xa] : 0;
                hi[k] = ok ? bstart[row + xl + 1] : 0;
                mid[k] = !ok ? 0 : nx == 0 ? lo[k] : nx > E ? hi[k] : bstart[row + nx];
            }
            double sum[3] = {0.0, 0.0, 0.0};
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int by = k & 1, bz = k >> 1;
                for (int e = lo[k]; e < hi[k]; ++e) {
                    const int jb = perm[e];
                    const double fx = (double)rf[jb], fy = (double)rf[B + jb],
                                 fz = (double)rf[2 * B + jb];
                    const double wk = (e < mid[k] ? fx : 1.0 - fx) * (by ? fy : 1.0 - fy) *
                                      (bz ? fz : 1.0 - fz);
                    sum[0] += wk * (double)ru[jb];
                    sum[1] += wk * (double)ru[B + jb];
                    sum[2] += wk * (double)ru[2 * B + jb];
                }
            }
            for (int comp = 0; comp < 3; ++comp) nacc[comp * S3 + n] += sum[comp];
        }
        __syncthreads();   // the next batch overwrites the entries
    }
    if (TRI) {
        // each node's sum was last written by this thread
        for (int n = threadIdx.x; n < S3; n += kAdjBlock) {
            const int64_t g = tile_cell(n);
            for (int comp = 0; comp < 3; ++comp) {
                const double v = nacc[comp * S3 + n];
                if (v != 0.0) atomicAdd(a.Ubar + comp * ncell + g, v);
            }
        }
        return;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < 3 * S3; t += kAdjBlock) {
        const double v = (double)ubt[t];
        if (v != 0.0) {
            const int comp = t / S3;
            atomicAdd(a.Ubar + comp * ncell + tile_cell(t - comp * S3), v);
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

// dL/dd of every particle out of the adjoint records
__global__ void k_take_dbar(const double *adj, int64_t P, double *dd)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < P;
         i += (int64_t)gridDim.x * blockDim.x)
        dd[i] = adj[8 * i + 6];
}

inline int64_t grid_of(int64_t n)
{
    const int64_t g = (n + 255) / 256;
    return g < 1 ? 1 : (g > 16384 ? 16384 : g);
}

template <class T>
AdjArgs<T> adj_args(st_ctx *c, const char *snap, const TapeStep &ts, const double *lamC,
                    double *adj, double *Ubar)
{
    const SnapLayout L = snap_layout(c->slots, c->tsize, c->C, c->max_items);
    const T *st = reinterpret_cast<const T *>(snap + L.state);
    AdjArgs<T> a;
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
    a.grid = c->max_items;
    a.u = reinterpret_cast<const T *>(ts.u);
    a.lamC = lamC;
    a.adj = adj;
    a.Ubar = Ubar;
    a.count = c->count;
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
        if (ngp) hipLaunchKernelGGL((k_adjoint_step<T, 2, 1>), g, b, 0, s, a);
        else hipLaunchKernelGGL((k_adjoint_step<T, 2, 0>), g, b, 0, s, a);
        break;
    case 4:
        if (ngp) hipLaunchKernelGGL((k_adjoint_step<T, 4, 1>), g, b, 0, s, a);
        else hipLaunchKernelGGL((k_adjoint_step<T, 4, 0>), g, b, 0, s, a);
        break;
    default:
        if (ngp) hipLaunchKernelGGL((k_adjoint_step<T, 8, 1>), g, b, 0, s, a);
        else hipLaunchKernelGGL((k_adjoint_step<T, 8, 0>), g, b, 0, s, a);
        break;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_backward(st_ctx *c, const double *lam, double *dU, double *dd, hipStream_t s)
{
    const int64_t ntape = (int64_t)c->tape.size();
    const int64_t K = c->tape_every;
    const int64_t nseg = (int64_t)c->snaps.size();
    if (ntape == 0 || K <= 0 || nseg != (ntape + K - 1) / K) return hipErrorInvalidValue;
    const int64_t P = c->count;
    const int64_t ncell = (int64_t)c->prm.n[0] * c->prm.n[1] * c->prm.n[2];
    const int64_t E3 = (int64_t)c->prm.E * c->prm.E * c->prm.E;
    const size_t sbytes = snapshot_bytes(c);

    // one workspace, kept in the context for the next call: the state the
    // forward run ended in, the saved states of one segment, dL/dS by chunk
    // and the adjoint records
    auto up256 = [](size_t v) { return (v + 255) & ~(size_t)255; };
    const size_t o_steps = up256(sbytes);
    const size_t o_lam = o_steps + (size_t)K * up256(sbytes);
    const size_t o_adj = o_lam + up256((size_t)c->C * 3 * E3 * 8);
    const size_t ws_bytes = o_adj + (size_t)(P > 0 ? P : 1) * 64;
    if (c->bwd_ws_bytes < ws_bytes) {
        (void)hipFree(c->bwd_ws);
        c->bwd_ws = nullptr;
        c->bwd_ws_bytes = 0;
        hipError_t e = hipMalloc(&c->bwd_ws, ws_bytes);
        if (e != hipSuccess) return e;
        c->bwd_ws_bytes = ws_bytes;
    }
    char *ws = (char *)c->bwd_ws;
    void *final_state = ws;
    auto step_buf = [&](int64_t k) -> void * { return ws + o_steps + (size_t)k * up256(sbytes); };
    double *lamC = (double *)(ws + o_lam);
    double *adj = (double *)(ws + o_adj);

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
    hipLaunchKernelGGL(k_zero_f64, dim3(grid_of(8 * P)), dim3(256), 0, s, adj, 8 * P);
    e = hipGetLastError();
    if (e != hipSuccess) return fail(e);

    for (int64_t sg = nseg - 1; sg >= 0; --sg) {
        const int64_t k0 = sg * K, k1 = std::min(k0 + K, ntape);
        e = launch_snapshot(c, c->snaps[(size_t)sg].buf, 1, s);
        if (e != hipSuccess) return fail(e);
        // recompute the segment, each step saving what its reverse reads; the
        // last step's start is the store itself
        for (int64_t k = k0; k < k1; ++k) {
            void *save = step_buf(k - k0);
            if (k + 1 < k1)
                e = launch_step(c, c->tape[(size_t)k].u, c->tape[(size_t)k].dt, 0, s, save);
            else
                e = launch_snapshot(c, save, 0, s);
            if (e != hipSuccess) return fail(e);
        }
        // and reverse it, newest step first
        for (int64_t k = k1 - 1; k >= k0; --k) {
            const char *snap = (const char *)step_buf(k - k0);
            if (c->form == ST_FORM_FP64)
                e = launch_adjoint_step<double>(
                    c, adj_args<double>(c, snap, c->tape[(size_t)k], lamC, adj, dU), s);
            else
                e = launch_adjoint_step<float>(
                    c, adj_args<float>(c, snap, c->tape[(size_t)k], lamC, adj, dU), s);
            if (e != hipSuccess) return fail(e);
        }
    }
    hipLaunchKernelGGL(k_take_dbar, dim3(grid_of(P)), dim3(256), 0, s, (const double *)adj, P, dd);
    e = hipGetLastError();
    if (e != hipSuccess) return fail(e);
    e = launch_snapshot(c, final_state, 1, s);
    if (e != hipSuccess) return fail(e);
    // the tape's buffers are handed back when this returns: finish first
    return hipStreamSynchronize(s);
}

}  // namespace st
