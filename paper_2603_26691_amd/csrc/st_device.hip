// HIP kernels of the scaletrack library, written for CDNA4 (gfx950, wave64).
//
// One step of the particle method (paper Sec. 2.1 equations of motion and
// momentum source, Sec. 2.5 interpolation, deposit and time integration)
// is five launches:
//   step      one workgroup per work item (a run of at most kSeg slots of
//             one chunk): stage the chunk's fluid tile with a one-cell halo
//             in LDS, gather, integrate, deposit into an LDS accumulator of
//             the chunk's cells, write every particle back in place, collect
//             the chunk crossers ("movers") in LDS by direction and emit
//             them as whole records, with one atomic instruction for all of
//             a workgroup's reservations (mover list, the chunk's hole list,
//             one arrival count per neighbouring chunk), and flush the
//             accumulator with one read-modify-write (or one atomic, for
//             chunks split over several items) per cell.  A mover's slot
//             becomes a hole of its chunk (binary32: a -1 offset, written by
//             the step's own store; binary64: its diameter negated, its
//             state left in place) and goes onto the chunk's hole list; its
//             record carries its destination and its rank among the
//             destination's arrivals.  Arrivals that do not fit the
//             destination's free slots force the full re-bin;
//   arrive    one thread per mover: each arrival takes a hole of its
//             destination (the newest first) or, when there are none left,
//             the next slot past the destination's last (when a full re-bin
//             is due, nothing: the re-bin takes the movers from their
//             records);
//   counts    one thread per chunk: the new slot and hole counts; holes no
//             arrival took are skipped by every kernel until the next full
//             re-bin (forced once they exceed a sixteenth of the particles);
//   layout    work items of the next step from the counts, the reset of the
//             counters, and, when a full re-bin is due, the rooms and bases
//             of its layout (one workgroup; it also takes the counts step
//             when the mesh has few enough chunks);
//   scatter, commit
//             only when a chunk ran out of room, the mover list overflowed
//             or particles were injected: a full counting-sort re-bin into
//             the second store, copied back (decided on the device).
// (Meshes of more than kScan1Max chunks count and scan with several
// launches.)
// Device flags that decide between the two re-bins hold the tag (epoch) of
// the step that raised them, so nothing has to clear them between steps.
#include "st_internal.h"

#include <hip/hip_ext.h>

#include <math.h>

#include <algorithm>

namespace st {
namespace {

constexpr int kScan1Max = 1 << 13;  // largest scan done by one workgroup
constexpr int kScanBlock = 1024;    // elements per block of the multi-block scan

enum Gate { G_ALWAYS = 0, G_FULL = 1, G_MOVERS = 2 };

__device__ __forceinline__ bool full_rebin(const int32_t *flags, int32_t epoch)
{
    return flags[F_OVERFLOW] == epoch || flags[F_FORCE] == epoch;
}

__device__ __forceinline__ bool gate_open(const int32_t *flags, int gate, int32_t epoch)
{
    if (gate == G_ALWAYS) return true;
    return (gate == G_FULL) == full_rebin(flags, epoch);
}

// movers of the step tagged `epoch` are counted in one of two slots
__host__ __device__ __forceinline__ int nmov_slot(int32_t epoch)
{
    return (epoch & 1) ? F_NMOV_ODD : F_NMOV;
}

__device__ __forceinline__ int64_t wrapi(int64_t i, int64_t n)
{
    int64_t r = i % n;
    return r < 0 ? r + n : r;
}

__device__ __forceinline__ uint64_t lanes_below_mask() { return (1ull << __lane_id()) - 1ull; }

template <class V>
__device__ __forceinline__ V wave_incl_scan(V x)
{
    const int lane = __lane_id();
    for (int o = 1; o < 64; o <<= 1) {
        const V y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    return x;
}

// Block-wide exclusive scan of one value per thread (any multiple of 64
// threads up to 1024); returns the prefix and the block total.
template <class V>
__device__ V block_excl_scan(V v, V &total)
{
    __shared__ V ws[16];
    const int lane = __lane_id(), wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const V incl = wave_incl_scan(v);
    if (lane == 63) ws[wave] = incl;
    __syncthreads();
    if (wave == 0) {
        V w = lane < nw ? ws[lane] : V(0);
        w = wave_incl_scan(w);
        if (lane < nw) ws[lane] = w;
    }
    __syncthreads();
    total = ws[nw - 1];
    const V ex = (wave ? ws[wave - 1] : V(0)) + incl - v;
    __syncthreads();
    return ex;
}

// ---------------------------------------------------------------------------
// exclusive scans of f(i), i < n: out[i] = sum_{j<i} f(j), out[n] = total
// ---------------------------------------------------------------------------

// whole scan in one workgroup of 1024 threads, 4096 elements per round
template <class TO, class F>
__device__ void block_scan_all(const F &f, int64_t n, TO *out)
{
    TO carry = 0;
    for (int64_t r0 = 0; r0 < n; r0 += 4096) {
        TO v[4];
        TO s = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int64_t i = r0 + 4 * (int64_t)threadIdx.x + k;
            v[k] = i < n ? f(i) : TO(0);
            s += v[k];
        }
        TO total;
        TO ex = carry + block_excl_scan<TO>(s, total);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int64_t i = r0 + 4 * (int64_t)threadIdx.x + k;
            if (i < n) out[i] = ex;
            ex += v[k];
        }
        carry += total;
    }
    if (threadIdx.x == 0) out[n] = carry;
}

template <class TO, class F>
__global__ void __launch_bounds__(1024) k_scan1(F f, int64_t n, TO *out, const int32_t *flags,
                                                int gate, int32_t epoch)
{
    if (!gate_open(flags, gate, epoch)) return;
    block_scan_all<TO>(f, n, out);
}

template <class TO, class F>
__global__ void __launch_bounds__(256) k_scan_partials(F f, int64_t n, TO *part,
                                                       const int32_t *flags, int gate,
                                                       int32_t epoch)
{
    if (!gate_open(flags, gate, epoch)) return;
    const int64_t b0 = (int64_t)blockIdx.x * kScanBlock;
    TO s = 0;
    for (int k = 0; k < kScanBlock / 256; ++k) {
        const int64_t i = b0 + k * 256 + threadIdx.x;
        if (i < n) s += f(i);
    }
    TO tot;
    block_excl_scan<TO>(s, tot);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

template <class TO>
__global__ void __launch_bounds__(1024) k_scan_spine(TO *part, int64_t nb, const int32_t *flags,
                                                     int gate, int32_t epoch)
{
    if (!gate_open(flags, gate, epoch)) return;
    struct Id {
        const TO *p;
        __device__ TO operator()(int64_t i) const { return p[i]; }
    };
    // in place: the spine is short (n / 1024 entries)
    TO carry = 0;
    for (int64_t r0 = 0; r0 < nb; r0 += 1024) {
        const int64_t i = r0 + threadIdx.x;
        const TO v = i < nb ? part[i] : TO(0);
        TO total;
        const TO ex = block_excl_scan<TO>(v, total);
        if (i < nb) part[i] = carry + ex;
        carry += total;
    }
}

template <class TO, class F>
__global__ void __launch_bounds__(256) k_scan_final(F f, int64_t n, const TO *part, TO *out,
                                                    const int32_t *flags, int gate, int32_t epoch)
{
    if (!gate_open(flags, gate, epoch)) return;
    const int64_t b0 = (int64_t)blockIdx.x * kScanBlock;
    constexpr int K = kScanBlock / 256;
    TO v[K];
    TO s = 0;
    for (int k = 0; k < K; ++k) {
        const int64_t i = b0 + (int64_t)threadIdx.x * K + k;
        v[k] = i < n ? f(i) : TO(0);
        s += v[k];
    }
    TO tot;
    TO ex = block_excl_scan<TO>(s, tot) + part[blockIdx.x];
    for (int k = 0; k < K; ++k) {
        const int64_t i = b0 + (int64_t)threadIdx.x * K + k;
        if (i < n) out[i] = ex;
        ex += v[k];
        if (i == n - 1) out[n] = ex;
    }
}

// multi-block scan (three launches), for n > kScan1Max
template <class TO, class F>
hipError_t scan_multi(F f, int64_t n, TO *out, TO *part, const int32_t *flags, int gate,
                      int32_t epoch, hipStream_t s)
{
    const int64_t nb = (n + kScanBlock - 1) / kScanBlock;
    hipLaunchKernelGGL((k_scan_partials<TO, F>), dim3(nb), dim3(256), 0, s, f, n, part, flags,
                       gate, epoch);
    hipLaunchKernelGGL((k_scan_spine<TO>), dim3(1), dim3(1024), 0, s, part, nb, flags, gate,
                       epoch);
    hipLaunchKernelGGL((k_scan_final<TO, F>), dim3(nb), dim3(256), 0, s, f, n, part, out, flags,
                       gate, epoch);
    return hipGetLastError();
}

template <class TO, class F>
hipError_t scan(F f, int64_t n, TO *out, TO *part, const int32_t *flags, int gate, int32_t epoch,
                hipStream_t s)
{
    if (n <= kScan1Max) {
        hipLaunchKernelGGL((k_scan1<TO, F>), dim3(1), dim3(1024), 0, s, f, n, out, flags, gate,
                           epoch);
        return hipGetLastError();
    }
    return scan_multi<TO>(f, n, out, part, flags, gate, epoch, s);
}

// work items per chunk
struct Segments {
    const int32_t *cnt;
    __device__ int32_t operator()(int64_t i) const { return (cnt[i] + kSeg - 1) / kSeg; }
};

// Share of the spare slots a chunk asks for in a re-binned layout: the
// largest count among the chunk and its six face neighbours (periodic), plus
// kSlackMin.  What a chunk can gain before the next re-bin is bounded by what
// its neighbours can send, so a sparse chunk at the edge of a dense region
// gets room for the arrivals from the dense side.
struct RoomWeight {
    const int32_t *cnt;
    int32_t nc[3];
    __device__ int64_t operator()(int64_t i) const
    {
        const int64_t x = i % nc[0], y = (i / nc[0]) % nc[1], z = i / ((int64_t)nc[0] * nc[1]);
        const int64_t sx = 1, sy = nc[0], sz = (int64_t)nc[0] * nc[1];
        const int64_t nb[6] = {
            i + (x == nc[0] - 1 ? -(nc[0] - 1) * sx : sx), i + (x == 0 ? (nc[0] - 1) * sx : -sx),
            i + (y == nc[1] - 1 ? -(nc[1] - 1) * sy : sy), i + (y == 0 ? (nc[1] - 1) * sy : -sy),
            i + (z == nc[2] - 1 ? -(nc[2] - 1) * sz : sz), i + (z == 0 ? (nc[2] - 1) * sz : -sz)};
        int32_t m = cnt[i];
#pragma unroll
        for (int k = 0; k < 6; ++k) m = max(m, cnt[nb[k]]);
        return (int64_t)m + kSlackMin;
    }
};

// rooms of a re-binned layout: the spare slots are shared out in proportion
// to the chunks' weights (denom = their sum), rounded down to whole groups of
// kAlign slots, on top of the count rounded up to kAlign; also records the
// room
struct Rooms {
    RoomWeight w;
    int64_t spare, denom;
    int32_t *nroom;
    __device__ int64_t operator()(int64_t i) const
    {
        const int64_t n = w.cnt[i];
        const int64_t extra = denom > 0 ? spare * w(i) / denom : 0;
        const int64_t r = (n + kAlign - 1) / kAlign * kAlign + extra / kAlign * kAlign;
        nroom[i] = (int32_t)r;
        return r;
    }
};

// the same, with the sum of the weights read from device memory (several
// workgroups; written by k_room_denom)
struct RoomsDev {
    Rooms r;
    const int64_t *denom;
    __device__ int64_t operator()(int64_t i) const
    {
        Rooms q = r;
        q.denom = *denom;
        return q(i);
    }
};

// sum of f(i), i < n, over one workgroup of 1024 threads (every thread gets it)
template <class F>
__device__ int64_t block_sum_all(const F &f, int64_t n)
{
    int64_t s = 0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) s += f(i);
    int64_t tot;
    block_excl_scan<int64_t>(s, tot);
    return tot;
}

// ---------------------------------------------------------------------------
// chunks and re-basing of chunk-local offsets
// ---------------------------------------------------------------------------
__device__ __forceinline__ int64_t chunk_index(const Params &p, int64_t cx, int64_t cy,
                                               int64_t cz)
{
    return (cz * p.nc[1] + cy) * p.nc[0] + cx;
}

// An offset that left [0, E) moves to the chunk k steps away along the axis
// and is re-based onto it; a rounding that lands exactly on E belongs to the
// next chunk at offset 0.  Returns k.
template <class T>
__device__ __forceinline__ int rebase(T &xi, T fe, T inv_e)
{
    T kf = floor(xi * inv_e);
    int k = (int)kf;
    xi = xi - kf * fe;
    if (xi < T(0)) { xi += fe; --k; }
    if (xi >= fe) { xi -= fe; ++k; }
    return k;
}

template <class T>
__device__ __forceinline__ int64_t chunk_after(const Params &p, int64_t c, T &ox, T &oy, T &oz)
{
    const T fe = T(p.E), inv_e = T(1) / T(p.E);  // E is a power of two: exact
    int kx = rebase(ox, fe, inv_e), ky = rebase(oy, fe, inv_e), kz = rebase(oz, fe, inv_e);
    if ((kx | ky | kz) == 0) return c;
    const int64_t cx = c % p.nc[0];
    const int64_t cy = (c / p.nc[0]) % p.nc[1];
    const int64_t cz = c / ((int64_t)p.nc[0] * p.nc[1]);
    return chunk_index(p, wrapi(cx + kx, p.nc[0]), wrapi(cy + ky, p.nc[1]),
                       wrapi(cz + kz, p.nc[2]));
}

// FP32-everywhere form: the cell of a binary32 coordinate in metres along one
// axis, from the rounded binary32 product x n / L (a rounding that reaches n
// stays in the last cell).  Every kernel takes a particle's cell and chunk
// from this one product, so they agree on them.
__device__ __forceinline__ float gprod(float x, float inv_h) { return __fmul_rn(x, inv_h); }
__device__ __forceinline__ int gcell(float x, float inv_h, int n)
{
    const int c = (int)floorf(gprod(x, inv_h));
    return min(max(c, 0), n - 1);
}

// The chunk of a stored position: chunk-local offsets re-based from chunk c
// (left re-based), or binary32 coordinates in metres (left as they are).
template <class T>
__device__ __forceinline__ int64_t chunk_of_stored(const Params &p, int64_t c, T &x, T &y, T &z)
{
    if (p.global)
        return chunk_index(p, gcell((float)x, p.inv_hf[0], p.n[0]) / p.E,
                           gcell((float)y, p.inv_hf[1], p.n[1]) / p.E,
                           gcell((float)z, p.inv_hf[2], p.n[2]) / p.E);
    return chunk_after(p, c, x, y, z);
}

// ---------------------------------------------------------------------------
// work items of the next step, and the reset of the per-step counters
// ---------------------------------------------------------------------------
struct ItemArgs {
    int64_t C;
    int32_t *noff;       // [C+1] exclusive scan of the items per chunk
    int32_t *items;
    int32_t *out_cnt, *in_cnt, *new_cnt, *cursor;
    int32_t *flags;
    int32_t epoch;
    int32_t dead_limit;  // more holes than this force a full re-bin at the next step
};

// chunk c's work items [o, e) (its offsets in the item list), and the reset
// of its counters
__device__ __forceinline__ void write_items_at(const ItemArgs &a, int64_t c, int32_t o, int32_t e)
{
    for (int32_t s = 0; s < e - o; ++s) {
        a.items[2 * (int64_t)(o + s)] = (int32_t)c;
        a.items[2 * (int64_t)(o + s) + 1] = s;
    }
    a.out_cnt[c] = 0;
    a.in_cnt[c] = 0;
}

__device__ __forceinline__ void write_items(const ItemArgs &a, int64_t c)
{
    write_items_at(a, c, a.noff[c], a.noff[c + 1]);
}

__device__ __forceinline__ void finish_flags_n(const ItemArgs &a, int32_t nitems)
{
    a.flags[F_NITEMS] = nitems;
    a.flags[F_LASTMOV] = a.flags[nmov_slot(a.epoch)];
    a.flags[nmov_slot(a.epoch + 1)] = 0;
    // holes are streamed like particles until a full re-bin drops them
    if (a.flags[F_DEAD] > a.dead_limit) a.flags[F_FORCE] = a.epoch + 1;
}

__device__ __forceinline__ void finish_flags(const ItemArgs &a)
{
    finish_flags_n(a, a.noff[a.C]);
}

// one workgroup: scan, items and reset (C <= kScan1Max)
__global__ void __launch_bounds__(1024) k_items1(Segments f, ItemArgs a)
{
    block_scan_all<int32_t>(f, a.C, a.noff);
    __syncthreads();
    for (int64_t c = threadIdx.x; c < a.C; c += blockDim.x) write_items(a, c);
    if (threadIdx.x == 0) finish_flags(a);
}

__global__ void k_items(ItemArgs a)
{
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < a.C;
         c += (int64_t)gridDim.x * blockDim.x)
        write_items(a, c);
    if (blockIdx.x == 0 && threadIdx.x == 0) finish_flags(a);
}

// After the arrivals: chunk c's new slot and hole counts.  With h holes
// (older ones plus the step's departures) and `in` arrivals, the arrivals
// took the top min(h, in) holes and the rest of them extended the chunk;
// holes no arrival took stay listed (and marked: a -1 offset or a negated
// diameter).  Returns the chunk's holes.
// chunk c's slot count after the arrivals (as count_chunk_from sets it)
__device__ __forceinline__ int32_t chunk_count_after(int32_t out, int32_t in, int32_t nd,
                                                     int32_t cnt)
{
    const int32_t h = nd + out;
    return in >= h ? cnt + in - h : cnt;
}

template <class T>
__device__ __forceinline__ int32_t count_chunk_from(const View<T> &V, int32_t out, int32_t in,
                                                    int32_t nd, int32_t cnt, int64_t c)
{
    const int32_t h = nd + out;
    if (out == 0 && in == 0) return nd;
    if (in >= h) {
        V.cnt[c] = cnt + in - h;
        V.ndead[c] = 0;
        return 0;
    }
    V.ndead[c] = h - in;
    return h - in;
}

template <class T>
__device__ __forceinline__ int32_t count_chunk(const View<T> &V, const int32_t *out_cnt,
                                               const int32_t *in_cnt, int64_t c)
{
    return count_chunk_from(V, out_cnt[c], in_cnt[c], V.ndead[c], V.cnt[c], c);
}

// one workgroup, after the arrivals or the re-keyed count (C <= kScan1Max).
// After the arrivals: the chunks' new counts (one wave per chunk), the work
// items of the next step and the reset of the counters.  When a full re-bin
// is due: the rooms and bases of its layout and the item offsets from the
// re-keyed counts; the scatter still walks the current items, so the commit
// writes the new ones.
template <class T>
__global__ void __launch_bounds__(1024) k_layout1(Rooms rooms, int64_t *nbase,
                                                  Segments rekeyed, ItemArgs a, View<T> V,
                                                  const int32_t *flags)
{
    if (full_rebin(flags, a.epoch)) {
        rooms.denom = block_sum_all(rooms.w, a.C);
        block_scan_all<int64_t>(rooms, a.C, nbase);
        __syncthreads();
        block_scan_all<int32_t>(rekeyed, a.C, a.noff);
        return;
    }
    // a thread's chunks c = k 1024 + threadIdx.x (at most kScan1Max / 1024):
    // every load is issued before the first store, so that the latencies
    // overlap, and the new counts, item offsets and totals stay in registers
    constexpr int PT = kScan1Max / 1024;
    int32_t out[PT], in[PT], nd[PT], cn[PT];
#pragma unroll
    for (int k = 0; k < PT; ++k) {
        const int64_t c = k * 1024 + threadIdx.x;
        out[k] = in[k] = nd[k] = cn[k] = 0;
        if (c < a.C) {
            out[k] = a.out_cnt[c];
            in[k] = a.in_cnt[c];
            nd[k] = V.ndead[c];
            cn[k] = V.cnt[c];
        }
    }
    int32_t dead = 0, nseg[PT];
#pragma unroll
    for (int k = 0; k < PT; ++k) {
        const int64_t c = k * 1024 + threadIdx.x;
        nseg[k] = 0;
        if (c < a.C) {
            dead += count_chunk_from(V, out[k], in[k], nd[k], cn[k], c);
            nseg[k] = (chunk_count_after(out[k], in[k], nd[k], cn[k]) + kSeg - 1) / kSeg;
        }
    }
    int32_t total;
    block_excl_scan<int32_t>(dead, total);
    if (threadIdx.x == 0) a.flags[F_DEAD] = total;
    // the item offsets in chunk order, a round of 1024 chunks at a time
    int32_t carry = 0;
#pragma unroll
    for (int k = 0; k < PT; ++k) {
        if ((int64_t)k * 1024 >= a.C) break;   // uniform
        int32_t rt;
        const int32_t o = carry + block_excl_scan<int32_t>(nseg[k], rt);
        const int64_t c = k * 1024 + threadIdx.x;
        if (c < a.C) {
            a.noff[c] = o;
            write_items_at(a, c, o, o + nseg[k]);
        }
        carry += rt;
    }
    if (threadIdx.x == 0) {
        a.noff[a.C] = carry;
        finish_flags_n(a, carry);
    }
}

__global__ void k_set_flag(int32_t *flags, int which, int32_t v) { flags[which] = v; }

// when a full re-bin is due on a mesh of more than kScan1Max chunks: the sum
// of the chunks' room weights, kScanBlock chunks per workgroup
__global__ void __launch_bounds__(256) k_room_denom(RoomWeight w, int64_t C, int64_t *denom,
                                                    const int32_t *flags, int32_t epoch)
{
    if (!full_rebin(flags, epoch)) return;
    const int64_t b0 = (int64_t)blockIdx.x * kScanBlock;
    int64_t s = 0;
    for (int k = 0; k < kScanBlock / 256; ++k) {
        const int64_t i = b0 + k * 256 + threadIdx.x;
        if (i < C) s += w(i);
    }
    int64_t tot;
    block_excl_scan<int64_t>(s, tot);
    if (threadIdx.x == 0) atomicAdd((unsigned long long *)denom, (unsigned long long)tot);
}

// ---------------------------------------------------------------------------
// the step kernel
// ---------------------------------------------------------------------------
template <class T, class A>
struct StepArgs {
    View<T> V;
    const int32_t *items;
    const int32_t *nitems;
    const T *u;              // field [3][n2][n1][n0]
    A *src;                  // [C][3][E^3]
    Movers<T> mv;
    int32_t *nmov;
    int64_t mcap;
    int32_t *out_cnt;
    int32_t *in_cnt;
    int32_t *hole;           // holes of chunk c, relative to base[c], from hole[base[c]]
    int32_t *flags;
    int32_t deposit;         // 0: move and re-bin only (tape recompute)
    int32_t epoch;           // tag of this step in the device flags
    // tape recompute: what the reverse of the step reads, saved into a
    // snapshot buffer at the store's slot indices: the state each slot
    // starts the step with, its id, and the step's layout (its work items,
    // and the first slot and slot count of every chunk that has one)
    T *sv[7];
    int32_t *sid;
    int32_t *sitems;
    int32_t *snitems;
    int64_t *sbase;
    int32_t *scnt;
    Params p;
    T dt;
    T dt_h[3];               // dt / h per axis
    T tau_coef;
    T g[3];
    T g_dt[3];               // g dt
    T mass_coef;             // w rho_p pi / 6
    T inv_V;                 // 1 / cell volume
    T re2_coef;              // (rho_f / mu_f)^2: Re^2 = re2_coef d^2 |u_f - u_p|^2
};

// reciprocal: the hardware's (1 ulp) in binary32, a division in binary64
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }

// Re^0.687 from Re^2 (no square root): 2^(0.3435 log2 Re^2) with the
// hardware's base-2 logarithm and exponential in binary32, pow in binary64.
// Re^2 = 0 gives 0 (log2 0 = -inf).
__device__ __forceinline__ float sn_re_pow(float re2)
{
    return __builtin_amdgcn_exp2f(0.3435f * __builtin_amdgcn_logf(re2));
}
__device__ __forceinline__ double sn_re_pow(double re2) { return pow(re2, 0.3435); }

// Workgroups are dispatched round-robin over the 8 XCDs.  Work items are
// dealt to the XCDs in blocks of kXcdBlock consecutive items (neighbouring
// chunks, which share halo cells through the XCD's L2), block j to XCD
// j mod 8, so that every XCD gets a share of every region of the item list
// and of its work, however uneven the chunk occupancy.  A bijection of
// [0, R), R the item count rounded up to whole rounds of 8 blocks; ids that
// map past the items exit.  Blocks of 16 items measured best (1.8 % less
// step-kernel time than 64 on 128^3; one item per block, the hardware's own
// dealing, 7 % more).
constexpr int64_t kXcdBlock = 16;
__device__ __forceinline__ int64_t xcd_remap(int64_t bid)
{
    const int64_t x = bid % 8, k = bid / 8;
    return ((k / kXcdBlock) * 8 + x) * kXcdBlock + k % kXcdBlock;
}

// G consecutive values at a G*sizeof(T)-aligned address, as one 16-byte
// access with the non-temporal hint: the particle state is streamed, read
// once and written once per step, so it should not displace what the caches
// hold (the tile, the counters, the mover lists).  Measured: 13 % less step
// kernel time on 1e7 particles, 11 % on 1.4e9.
template <class T, int G>
__device__ __forceinline__ void vld(const T *p, T (&v)[G])
{
    typedef T vec __attribute__((ext_vector_type(G)));
    const vec r =
        __builtin_nontemporal_load((const vec *)__builtin_assume_aligned(p, G * sizeof(T)));
#pragma unroll
    for (int k = 0; k < G; ++k) v[k] = r[k];
}

template <class T, int G>
__device__ __forceinline__ void vst(T *p, const T (&v)[G])
{
    typedef T vec __attribute__((ext_vector_type(G)));
    vec r;
#pragma unroll
    for (int k = 0; k < G; ++k) r[k] = v[k];
    __builtin_nontemporal_store(r, (vec *)__builtin_assume_aligned(p, G * sizeof(T)));
}

// base + byte offset: a uniform 64-bit base plus a 32-bit per-lane offset,
// which the loads and stores take in their scalar-base addressing form
template <class T>
__device__ __forceinline__ T *at_byte(T *base, uint32_t byte_off)
{
    return (T *)((char *)base + byte_off);
}
template <class T>
__device__ __forceinline__ const T *at_byte(const T *base, uint32_t byte_off)
{
    return (const T *)((const char *)base + byte_off);
}

// Slots of chunk c free for arrivals whatever the step's departures: those
// past its last slot and its holes from earlier steps.
template <class T>
__device__ __forceinline__ int32_t free_slots(const View<T> &V, int64_t c)
{
    return V.room[c] - V.cnt[c] + V.ndead[c];
}

// A slot holds a particle unless its offset is negative (binary32 forms:
// the step kernel stores -1 for a particle that left) or its diameter is not
// positive (binary64 form: the diameter of a particle that left is negated).
template <class T>
__device__ __forceinline__ bool occupied(T ox, T d)
{
    return ox >= T(0) && d > T(0);
}

// A mover not staged in LDS (more movers than the stage holds), from its
// new state in registers (un-rebased offsets, relative to chunk c): lists
// its slot q among the chunk's holes at hpos and copies the particle,
// re-based onto its destination chunk, into the mover list at m with its
// destination and its rank among the destination's arrivals.  Returns false
// when the mover list is full: the particle then stays in place (the full
// re-bin that the overflow forces takes it from there).
template <class T, class A>
__device__ __forceinline__ bool emit_mover(const StepArgs<T, A> &a, int64_t c, int64_t base,
                                           int64_t q, int64_t m, int64_t hpos, T x, T y, T z,
                                           T vx, T vy, T vz, T dd)
{
    const View<T> &V = a.V;
    const int32_t id = V.id[q];
    const int64_t cn = chunk_of_stored(a.p, c, x, y, z);
    a.hole[base + hpos] = (int32_t)(q - base);
    if (m >= a.mcap) {
        a.flags[F_OVERFLOW] = a.epoch;
        return false;
    }
    a.mv.rec[m] = MoverRec<T>{x, y, z, vx, vy, vz, dd, id};
    a.mv.dest[m] = (int32_t)cn;
    const int32_t r = atomicAdd(&a.in_cnt[cn], 1);
    a.mv.rank[m] = r;
    // arrivals must fit the destination's free slots; one that does not
    // forces the full re-bin, which places every recorded mover itself
    if (r >= free_slots(V, cn)) a.flags[F_OVERFLOW] = a.epoch;
    return true;
}

// Staged mover: its slot within the work item (below kSeg, 14 bits), its
// direction class (0..26 the neighbouring chunks, 27 farther; 5 bits) and its
// rank within that class (below kMoverStage, 9 bits).
constexpr int kSlotBits = 14, kDirBits = 5;
static_assert(kSeg <= (1 << kSlotBits) && kMoverStage <= (1 << (32 - 1 - kSlotBits - kDirBits)),
              "staged mover fields must fit one int32");
static_assert(kDirBits * 4 <= 32, "direction classes of a group must fit one uint32");

template <class T, class A, int E, int INTERP, int DRAG, bool SAVE>
__global__ void __launch_bounds__(kBlock)
     k_step(StepArgs<T, A> a)
{
    constexpr int S = E + 2;            // tile edge with the halo
    constexpr int S3 = S * S * S;
    constexpr int E3 = E * E * E;
    constexpr int G = 16 / sizeof(T);   // consecutive particles per thread
    static_assert(kAlign % G == 0, "chunk rooms must hold whole particle groups");
    __shared__ T tile[3 * S3];
    __shared__ A acc[3 * E3];
    __shared__ int32_t mstage[kMoverStage];
    // binary32 state: the staged movers' new positions and velocities (12 KB,
    // which still lets four workgroups share a CU; the binary64 form re-reads
    // them instead)
    constexpr bool kStageVals = sizeof(T) == 4;
    __shared__ T mval[kStageVals ? 6 * kMoverStage : 1];
    __shared__ int32_t mcount, mbase_sh, hbase_sh;
    __shared__ int32_t dcount[28], doff[28], dbase[27];

    // the grid covers the most items a layout can have, rounded up to whole
    // rounds of the remap
    const int64_t item = xcd_remap(blockIdx.x);
    if constexpr (SAVE)
        if (blockIdx.x == 0 && threadIdx.x == 0) *a.snitems = *a.nitems;
    if (item >= *a.nitems) return;
    const View<T> &V = a.V;
    const int64_t c = a.items[2 * item];
    const int64_t seg = a.items[2 * item + 1];
    const int64_t base = V.base[c];
    const int32_t cnt = V.cnt[c];
    if constexpr (SAVE) {
        if (threadIdx.x == 0) {
            a.sitems[2 * item] = (int32_t)c;
            a.sitems[2 * item + 1] = (int32_t)seg;
            if (seg == 0) {
                a.sbase[c] = base;
                a.scnt[c] = cnt;
            }
        }
    }
    const int32_t nd_c = V.ndead[c];   // this step's holes are listed after these
    const int64_t s0 = base + seg * kSeg;
    const int64_t s1 = min(s0 + (int64_t)kSeg, base + (int64_t)cnt);
    const bool multi = cnt > kSeg;
    const Params &p = a.p;
    const int cx = (int)(c % p.nc[0]);
    const int cy = (int)((c / p.nc[0]) % p.nc[1]);
    const int cz = (int)(c / ((int64_t)p.nc[0] * p.nc[1]));
    const int64_t ncell = (int64_t)p.n[0] * p.n[1] * p.n[2];

    // The work item's slots are read in groups of G consecutive slots through
    // uniform base pointers and 32-bit offsets (at most kSeg).  s0 is a
    // multiple of G (chunk bases and kSeg are), and a group that runs past s1
    // stays inside the chunk's room.
    const int nq = (int)(s1 - s0);
    const int ngroups = (nq + G - 1) / G;
    T *const pox = V.ox + s0, *const poy = V.oy + s0, *const poz = V.oz + s0;
    T *const pvx = V.vx + s0, *const pvy = V.vy + s0, *const pvz = V.vz + s0;
    const T *const pd = V.d + s0;
    auto load_group = [&](int gi, T (&X)[G], T (&Y)[G], T (&Z)[G], T (&UX)[G], T (&UY)[G],
                          T (&UZ)[G], T (&DD)[G]) {
        const uint32_t ob = (uint32_t)gi * G * (uint32_t)sizeof(T);
        vld<T, G>(at_byte(pox, ob), X);
        vld<T, G>(at_byte(poy, ob), Y);
        vld<T, G>(at_byte(poz, ob), Z);
        vld<T, G>(at_byte(pvx, ob), UX);
        vld<T, G>(at_byte(pvy, ob), UY);
        vld<T, G>(at_byte(pvz, ob), UZ);
        vld<T, G>(at_byte(pd, ob), DD);
    };

    // Stage the fluid tile: cells E*c - 1 .. E*c + E per axis, wrapped.  The
    // main loop is software-pipelined: a group's loads are issued before the
    // arithmetic of the previous one, and the first group's right after the
    // tile's loads, so that memory latency overlaps work.
    constexpr int NT = (3 * S3 + kBlock - 1) / kBlock;
    T vals[NT];
    {
        const int ox0 = cx * E - 1, oy0 = cy * E - 1, oz0 = cz * E - 1;
#pragma unroll
        for (int u = 0; u < NT; ++u) {
            const int t = threadIdx.x + u * kBlock;
            if (t < 3 * S3) {
                const int comp = t / S3;
                const int r = t - comp * S3;
                const int k = r / (S * S);
                const int j = (r / S) % S;
                const int i = r % S;
                int gx = ox0 + i, gy = oy0 + j, gz = oz0 + k;
                gx += gx < 0 ? p.n[0] : 0;
                gx -= gx >= p.n[0] ? p.n[0] : 0;
                gy += gy < 0 ? p.n[1] : 0;
                gy -= gy >= p.n[1] ? p.n[1] : 0;
                gz += gz < 0 ? p.n[2] : 0;
                gz -= gz >= p.n[2] ? p.n[2] : 0;
                vals[u] = a.u[comp * ncell + ((int64_t)gz * p.n[1] + gy) * p.n[0] + gx];
            }
        }
    }
    int gi = threadIdx.x;
    T X[G], Y[G], Z[G], UX[G], UY[G], UZ[G], DD[G];
    if (gi < ngroups) load_group(gi, X, Y, Z, UX, UY, UZ, DD);
#pragma unroll
    for (int u = 0; u < NT; ++u) {
        const int t = threadIdx.x + u * kBlock;
        if (t < 3 * S3) tile[t] = vals[u];
    }
    for (int t = threadIdx.x; t < 3 * E3; t += kBlock) acc[t] = A(0);
    if (threadIdx.x < 28) dcount[threadIdx.x] = 0;
    if (threadIdx.x == 0) mcount = 0;
    __syncthreads();

    const T dt = a.dt;
    const T fe = T(E), inv_e = T(1) / T(E);
    // FP32-everywhere form: positions in binary32 metres, the cell arithmetic
    // in binary32 (the chunk origin in cells is exact)
    constexpr bool GLOBAL = sizeof(A) == 4;
    const T org[3] = {T(cx * E), T(cy * E), T(cz * E)};
    for (; gi < ngroups; gi += kBlock) {
        T Xn[G], Yn[G], Zn[G], UXn[G], UYn[G], UZn[G], DDn[G];
        if (gi + kBlock < ngroups) load_group(gi + kBlock, Xn, Yn, Zn, UXn, UYn, UZn, DDn);
        const uint32_t o = (uint32_t)gi * G;
        const uint32_t ob = o * (uint32_t)sizeof(T);
        if constexpr (SAVE) {   // the group as the step finds it, with its ids
            vst<T, G>(at_byte(a.sv[0] + s0, ob), X);
            vst<T, G>(at_byte(a.sv[1] + s0, ob), Y);
            vst<T, G>(at_byte(a.sv[2] + s0, ob), Z);
            vst<T, G>(at_byte(a.sv[3] + s0, ob), UX);
            vst<T, G>(at_byte(a.sv[4] + s0, ob), UY);
            vst<T, G>(at_byte(a.sv[5] + s0, ob), UZ);
            vst<T, G>(at_byte(a.sv[6] + s0, ob), DD);
            int32_t I[G];
            vld<int32_t, G>(at_byte((const int32_t *)V.id + s0, o * 4u), I);
            vst<int32_t, G>(at_byte(a.sid + s0, o * 4u), I);
        }
        uint32_t movers = 0, dirs = 0;   // mover bits and 5-bit direction classes
#pragma unroll
        for (int k = 0; k < G; ++k) {
            // slots past the run and holes hold no particle
            const bool valid = (int)o + k < nq && occupied(X[k], DD[k]);
            T xi[3] = {X[k], Y[k], Z[k]};   // cell units from the chunk origin
            if constexpr (GLOBAL) {
                xi[0] = gprod(X[k], p.inv_hf[0]) - org[0];
                xi[1] = gprod(Y[k], p.inv_hf[1]) - org[1];
                xi[2] = gprod(Z[k], p.inv_hf[2]) - org[2];
            }
            const T up[3] = {UX[k], UY[k], UZ[k]};
            const T dp = DD[k];

            // gather the fluid velocity at the particle
            T uf[3];
            int cl[3];
            if (INTERP == 0) {
                T f[3];
                int i0[3];
                for (int ax = 0; ax < 3; ++ax) {
                    const T s = xi[ax] - T(0.5);
                    const T fl = floor(s);
                    // -1 .. E-1 for offsets in [0, E); clamped so that no
                    // state can index outside the tile
                    i0[ax] = min(max((int)fl, -1), E - 1);
                    f[ax] = s - fl;
                    cl[ax] = min(max((int)xi[ax], 0), E - 1);
                }
                const int t0 = ((i0[2] + 1) * S + (i0[1] + 1)) * S + (i0[0] + 1);
                const T wx0 = T(1) - f[0], wx1 = f[0];
                const T wy0 = T(1) - f[1], wy1 = f[1];
                const T wz0 = T(1) - f[2], wz1 = f[2];
                const T w00 = wy0 * wz0, w10 = wy1 * wz0, w01 = wy0 * wz1, w11 = wy1 * wz1;
                for (int comp = 0; comp < 3; ++comp) {
                    const T *tc = tile + comp * S3 + t0;
                    const T r00 = wx0 * tc[0] + wx1 * tc[1];
                    const T r10 = wx0 * tc[S] + wx1 * tc[S + 1];
                    const T r01 = wx0 * tc[S * S] + wx1 * tc[S * S + 1];
                    const T r11 = wx0 * tc[S * S + S] + wx1 * tc[S * S + S + 1];
                    uf[comp] = w00 * r00 + w10 * r10 + w01 * r01 + w11 * r11;
                }
            } else {
                for (int ax = 0; ax < 3; ++ax) cl[ax] = min(max((int)xi[ax], 0), E - 1);
                const int t0 = ((cl[2] + 1) * S + (cl[1] + 1)) * S + (cl[0] + 1);
                for (int comp = 0; comp < 3; ++comp) uf[comp] = tile[comp * S3 + t0];
            }

            // semi-implicit Euler, drag implicit and gravity explicit:
            //   u_p' = (tau u_p + dt u_f + tau dt g) / (tau + dt)
            // written as the velocity change, which keeps its relative
            // accuracy in binary32:  u_p' - u_p = dt (u_f - u_p + tau g) / (tau + dt)
            T tau = a.tau_coef * dp * dp;
            if (DRAG == 1) {
                // Schiller-Naumann: tau / (1 + 0.15 Re^0.687), Re from the
                // slip at the start of the step
                const T sx = uf[0] - up[0], sy = uf[1] - up[1], sz = uf[2] - up[2];
                const T re2 = a.re2_coef * (dp * dp) * (sx * sx + sy * sy + sz * sz);
                tau = tau * recip(T(1) + T(0.15) * sn_re_pow(re2));
            }
            const T rD = dt * recip(tau + dt);
            T upn[3], xn[3];
            for (int ax = 0; ax < 3; ++ax) {
                upn[ax] = up[ax] + rD * ((uf[ax] - up[ax]) + tau * a.g[ax]);
                xn[ax] = xi[ax] + upn[ax] * a.dt_h[ax];
            }

            // drag impulse J = m (u_p' - u_p - g dt) = m dt (u_f - u_p - g dt) / (tau + dt),
            // evaluated from the stored inputs (not from the rounded new
            // velocity) and summed in the accumulator precision; the fluid
            // receives -J / V in the start-of-step cell
            if (a.deposit && valid) {
                const T coef = -(a.mass_coef * dp * dp * dp) * rD * a.inv_V;
                const int cell = (cl[2] * E + cl[1]) * E + cl[0];
                for (int ax = 0; ax < 3; ++ax) {
                    const T slip = (uf[ax] - up[ax]) - a.g_dt[ax];
                    atomicAdd(&acc[ax * E3 + cell], (A)(coef * slip));
                }
            }

            // relocate: a particle whose new offset left [0, E) on some axis
            // crossed into another chunk; it keeps the un-rebased offsets
            // (relative to this chunk) until it is emitted and re-based.  A
            // particle that stays needs no re-basing.  FP32-everywhere form:
            // the new position in metres, wrapped, and its chunk from its cells
            bool mover;
            int gk[3] = {0, 0, 0};   // FP32-everywhere: chunk steps per axis
            if constexpr (GLOBAL) {
                const T xg[3] = {X[k], Y[k], Z[k]};
                for (int ax = 0; ax < 3; ++ax) {
                    T v = xg[ax] + upn[ax] * dt;
                    if (v >= p.Lf[ax]) v -= p.Lf[ax];
                    else if (v < T(0)) v += p.Lf[ax];
                    if (!(v >= T(0) && v < p.Lf[ax])) {   // moved more than a domain length
                        v = fmodf(v, p.Lf[ax]);
                        if (v < T(0)) v += p.Lf[ax];
                    }
                    if (v >= p.Lf[ax]) v = T(0);
                    xn[ax] = v;
                    const int cc = ax == 0 ? cx : ax == 1 ? cy : cz;
                    int dk = gcell(v, p.inv_hf[ax], p.n[ax]) / E - cc;
                    // the shorter way round the periodic domain
                    if (dk > 1 && dk == p.nc[ax] - 1) dk = -1;
                    if (dk < -1 && dk == 1 - p.nc[ax]) dk = 1;
                    gk[ax] = dk;
                }
                mover = (gk[0] | gk[1] | gk[2]) != 0;
            } else {
                mover = xn[0] < T(0) || xn[0] >= fe || xn[1] < T(0) || xn[1] >= fe ||
                        xn[2] < T(0) || xn[2] >= fe;
            }
            if (valid) {   // a hole keeps what it holds (binary32: the -1 offset)
                X[k] = xn[0];
                Y[k] = xn[1];
                Z[k] = xn[2];
                UX[k] = upn[0];
                UY[k] = upn[1];
                UZ[k] = upn[2];
            }
            if (valid && mover) {
                movers |= 1u << k;
                int kx = gk[0], ky = gk[1], kz = gk[2];
                if constexpr (!GLOBAL) {
                    T tx = xn[0], ty = xn[1], tz = xn[2];
                    kx = rebase(tx, fe, inv_e);
                    ky = rebase(ty, fe, inv_e);
                    kz = rebase(tz, fe, inv_e);
                }
                const int dir = (abs(kx) <= 1 && abs(ky) <= 1 && abs(kz) <= 1)
                                    ? (kx + 1) + 3 * (ky + 1) + 9 * (kz + 1) : 27;
                dirs |= (uint32_t)dir << (kDirBits * k);
            }
        }
        // stage the movers with their direction class: one reservation of
        // stage entries per wave (their ranks within the direction classes
        // are taken after the loop)
        if (__ballot(movers != 0)) {
            // prefix of the lanes' mover counts (at most G < 8) from one
            // ballot per bit; the first active lane reserves for the wave
            const int mine = __popc(movers);
            const uint64_t below = lanes_below_mask();
            int ex = 0, tot = 0;
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const uint64_t bal = __ballot((mine >> b) & 1);
                ex += __popcll(bal & below) << b;
                tot += __popcll(bal) << b;
            }
            const int first = __ffsll((long long)__ballot(1)) - 1;
            int j0 = 0;
            if (__lane_id() == first) j0 = atomicAdd(&mcount, tot);
            int j = __shfl(j0, first) + ex;
            if constexpr (kStageVals) {
                // binary32: the new state too, so that it need not be re-read
#pragma unroll
                for (int k = 0; k < G; ++k) {
                    if (!((movers >> k) & 1)) continue;
                    if (j < kMoverStage) {
                        const int dir = (dirs >> (kDirBits * k)) & ((1 << kDirBits) - 1);
                        mstage[j] = (int32_t)(o + k) | (dir << kSlotBits);
                        mval[j] = X[k];
                        mval[kMoverStage + j] = Y[k];
                        mval[2 * kMoverStage + j] = Z[k];
                        mval[3 * kMoverStage + j] = UX[k];
                        mval[4 * kMoverStage + j] = UY[k];
                        mval[5 * kMoverStage + j] = UZ[k];
                        X[k] = T(-1);   // the slot becomes a hole
                    } else {  // more movers than the LDS stage holds: emit directly
                        const int64_t m = atomicAdd(a.nmov, 1);
                        const int64_t h = atomicAdd(&a.out_cnt[c], 1);
                        if (emit_mover(a, c, base, s0 + o + k, m, nd_c + h, X[k], Y[k], Z[k],
                                       UX[k], UY[k], UZ[k], DD[k]))
                            X[k] = T(-1);
                    }
                    ++j;
                }
            } else {
                while (movers) {
                    const int k = __ffs(movers) - 1;
                    movers &= movers - 1;
                    if (j < kMoverStage) {
                        const int dir = (dirs >> (kDirBits * k)) & ((1 << kDirBits) - 1);
                        mstage[j] = (int32_t)(o + k) | (dir << kSlotBits);
                    } else {  // more movers than the LDS stage holds: emit directly
                        const int64_t m = atomicAdd(a.nmov, 1);
                        const int64_t h = atomicAdd(&a.out_cnt[c], 1);
                        // binary64: the negated diameter marks the hole
                        if (emit_mover(a, c, base, s0 + o + k, m, nd_c + h, X[k], Y[k], Z[k],
                                       UX[k], UY[k], UZ[k], DD[k]))
                            a.V.d[s0 + o + k] = -DD[k];
                    }
                    ++j;
                }
            }
        }
        // slots past s1 in the last group are dead; writing them is harmless
        vst<T, G>(at_byte(pox, ob), X);
        vst<T, G>(at_byte(poy, ob), Y);
        vst<T, G>(at_byte(poz, ob), Z);
        vst<T, G>(at_byte(pvx, ob), UX);
        vst<T, G>(at_byte(pvy, ob), UY);
        vst<T, G>(at_byte(pvz, ob), UZ);
#pragma unroll
        for (int k = 0; k < G; ++k) {
            X[k] = Xn[k];
            Y[k] = Yn[k];
            Z[k] = Zn[k];
            UX[k] = UXn[k];
            UY[k] = UYn[k];
            UZ[k] = UZn[k];
            DD[k] = DDn[k];
        }
    }
    __syncthreads();

    // Mover reservations, all issued by one wave at once: the workgroup's
    // slots in the mover list (ordered by direction class, movers farther
    // than one chunk last, so that the arrivals a destination receives from
    // this chunk sit in consecutive records), its entries in the chunk's
    // vacated-slot list, and one arrival-count reservation per neighbouring
    // destination instead of one per mover, which would serialise on the
    // counters of crowded chunks.  The movers' state is read in the same
    // round trip.
    const int nm = min(mcount, kMoverStage);
    // ranks of the staged movers within their direction classes
    if (nm > 0) {
        for (int j = threadIdx.x; j < nm; j += kBlock) {
            const int32_t w = mstage[j];
            const int dir = (w >> kSlotBits) & ((1 << kDirBits) - 1);
            mstage[j] = w | (atomicAdd(&dcount[dir], 1) << (kSlotBits + kDirBits));
        }
        __syncthreads();
    }
    // The chunk's source cells are read first (a chunk that is one work item
    // adds its sum to them; one split over several items adds atomically).
    A *const src_c = a.src + c * (3 * E3);
    constexpr int NF = (3 * E3 + kBlock - 1) / kBlock;
    A old[NF];
    const bool rmw = a.deposit && !multi;
    if (rmw) {
#pragma unroll
        for (int u = 0; u < NF; ++u) {
            const int t = threadIdx.x + u * kBlock;
            old[u] = t < 3 * E3 ? src_c[t] : A(0);
        }
    }
    constexpr int NM = kMoverStage / kBlock;   // staged movers per thread
    T mx[NM], my[NM], mz[NM], mvx[NM], mvy[NM], mvz[NM], md[NM];
    int32_t mid[NM];
#pragma unroll
    for (int u = 0; u < NM; ++u) {
        const int j = threadIdx.x + u * kBlock;
        if (j < nm) {
            const int64_t q = s0 + (mstage[j] & ((1 << kSlotBits) - 1));
            if constexpr (kStageVals) {
                mx[u] = mval[j];
                my[u] = mval[kMoverStage + j];
                mz[u] = mval[2 * kMoverStage + j];
                mvx[u] = mval[3 * kMoverStage + j];
                mvy[u] = mval[4 * kMoverStage + j];
                mvz[u] = mval[5 * kMoverStage + j];
            } else {
                mx[u] = V.ox[q];
                my[u] = V.oy[q];
                mz[u] = V.oz[q];
                mvx[u] = V.vx[q];
                mvy[u] = V.vy[q];
                mvz[u] = V.vz[q];
            }
            md[u] = V.d[q];
            mid[u] = V.id[q];
        }
    }
    if (nm > 0 && threadIdx.x < 64) {
        const int lane = threadIdx.x;
        const int n = lane < 28 ? dcount[lane] : 0;
        int incl = n;
        for (int off = 1; off < 32; off <<= 1) {
            const int v = __shfl_up(incl, off);
            if (lane >= off) incl += v;
        }
        if (lane < 28) doff[lane] = incl - n;
        // one atomic instruction for all reservations (the counters differ
        // per lane): lanes 0..26 the arrival counts of the neighbouring
        // chunks, lane 32 the mover list, lane 33 the vacated-slot list
        const bool nb = lane < 27 && n > 0;
        const int64_t dc = chunk_index(p, wrapi(cx + lane % 3 - 1, p.nc[0]),
                                       wrapi(cy + (lane / 3) % 3 - 1, p.nc[1]),
                                       wrapi(cz + (lane / 9) % 3 - 1, p.nc[2]));
        int32_t *ctr = nb ? &a.in_cnt[dc] : lane == 32 ? a.nmov : &a.out_cnt[c];
        const int add = nb ? n : nm;
        if (nb || lane == 32 || lane == 33) {
            const int32_t r = atomicAdd(ctr, add);
            if (nb) {
                dbase[lane] = r;
                // arrivals must fit the destination's free slots (a bound
                // that ignores its departures), else the full re-bin runs
                if (r + n > free_slots(V, dc)) a.flags[F_OVERFLOW] = a.epoch;
            }
            if (lane == 32) mbase_sh = r;
            if (lane == 33) hbase_sh = r;
        }
    }

    // flush the chunk's accumulated source
    if (rmw) {
#pragma unroll
        for (int u = 0; u < NF; ++u) {
            const int t = threadIdx.x + u * kBlock;
            if (t < 3 * E3) src_c[t] = old[u] + acc[t];
        }
    } else if (a.deposit) {
        for (int t = threadIdx.x; t < 3 * E3; t += kBlock) {
            const A v = acc[t];
            if (v != A(0)) atomicAdd(src_c + t, v);
        }
    }
    if (nm == 0) return;
    __syncthreads();

    // emit the staged movers into their records and the arrival lists
#pragma unroll
    for (int u = 0; u < NM; ++u) {
        const int j = threadIdx.x + u * kBlock;
        if (j >= nm) continue;
        const int32_t w = mstage[j];
        const int32_t off = w & ((1 << kSlotBits) - 1);
        const int dir = (w >> kSlotBits) & ((1 << kDirBits) - 1);
        const int rank = w >> (kSlotBits + kDirBits);
        const int64_t m = (int64_t)mbase_sh + doff[dir] + rank;
        // re-base the offsets into the destination chunk (FP32-everywhere
        // form: positions in metres stay as they are)
        T rx = mx[u], ry = my[u], rz = mz[u];
        const int64_t cfar = chunk_of_stored(p, c, rx, ry, rz);
        int64_t dest;
        int32_t r;
        if (dir < 27) {   // within the direction's reservation
            dest = chunk_index(p, wrapi(cx + dir % 3 - 1, p.nc[0]),
                               wrapi(cy + (dir / 3) % 3 - 1, p.nc[1]),
                               wrapi(cz + dir / 9 - 1, p.nc[2]));
            r = dbase[dir] + rank;
        } else {          // farther than one chunk: a reservation of its own
            dest = cfar;
            r = atomicAdd(&a.in_cnt[dest], 1);
            if (r >= free_slots(V, dest)) a.flags[F_OVERFLOW] = a.epoch;
        }
        // the slot becomes a hole of this chunk (binary32: the step stored a
        // -1 offset; binary64: the diameter is negated)
        a.hole[base + nd_c + hbase_sh + j] = (int32_t)(s0 + off - base);
        if (m < a.mcap) {
            a.mv.rec[m] = MoverRec<T>{rx, ry, rz, mvx[u], mvy[u], mvz[u], md[u], mid[u]};
            a.mv.dest[m] = (int32_t)dest;
            // a rank beyond the destination's free slots has forced the full
            // re-bin, which places every recorded mover itself
            a.mv.rank[m] = r;
            if constexpr (!kStageVals) V.d[s0 + off] = -md[u];
        } else {
            // the mover list is full: the particle stays in place (its
            // un-rebased offsets) for the full re-bin that this forces
            a.flags[F_OVERFLOW] = a.epoch;
            if constexpr (kStageVals) V.ox[s0 + off] = mx[u];
        }
    }
}


// ---------------------------------------------------------------------------
// re-bin after the step: the arrivals or the full counting sort
// ---------------------------------------------------------------------------
template <class T>
__device__ __forceinline__ void place_mover(const View<T> &V, int64_t dst, const Movers<T> &mv,
                                            int64_t m)
{
    const MoverRec<T> r = mv.rec[m];
    V.ox[dst] = r.ox;
    V.oy[dst] = r.oy;
    V.oz[dst] = r.oz;
    V.vx[dst] = r.vx;
    V.vy[dst] = r.vy;
    V.vz[dst] = r.vz;
    V.d[dst] = r.d;
    V.id[dst] = r.id;
}

template <class T>
struct RebinArgs {
    View<T> V;
    View<T> W;               // second store (target of the full re-bin)
    Movers<T> mv;
    int64_t C;
    const int32_t *out_cnt, *in_cnt;
    int32_t *hole;
    const int32_t *items, *nitems;
    Params p;
    int64_t npend;           // staged injected particles (full re-bin only)
    int64_t mcap;            // mover list capacity
    int32_t *new_cnt, *cursor;
    const int64_t *nbase;
    const int32_t *nroom;
    int64_t *room_denom;     // sum of the room weights (zeroed by the count)
    int64_t slots;
    int32_t *flags;
    int32_t epoch;
};

constexpr int kArriveBlock = 256;   // threads per workgroup of the arrivals

// One thread per mover of the step: its arrival of rank r in chunk c takes
// the hole r places from the top of the chunk's hole list (the step's own
// departures first, then the older holes), or, past the holes, the slot
// r - holes past the chunk's last.  Counts are those of the step's start
// (the counts pass runs after this one).
template <class T>
__device__ void arrive(const RebinArgs<T> &a)
{
    const View<T> &V = a.V;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    // a thread's first destination and rank are read together with the
    // count (the list's entries below its capacity can all be read), the
    // next ones while the current mover is placed; a record is read beside
    // its destination's counts
    int32_t c = 0, r = 0;
    if (m < a.mcap) {
        c = a.mv.dest[m];
        r = a.mv.rank[m];
    }
    const int64_t nm = a.flags[nmov_slot(a.epoch)];
    if (blockIdx.x == 0 && threadIdx.x == 0) a.flags[F_DEAD] = 0;   // summed by the counts
    for (; m < nm; m += stride) {
        const MoverRec<T> cur = a.mv.rec[m];
        const int64_t base = V.base[c];
        const int32_t h = V.ndead[c] + a.out_cnt[c];
        const int64_t slot = r < h ? base + a.hole[base + h - 1 - r]
                                   : base + V.cnt[c] + (r - h);
        if (m + stride < nm && m + stride < a.mcap) {
            c = a.mv.dest[m + stride];
            r = a.mv.rank[m + stride];
        }
        V.ox[slot] = cur.ox;
        V.oy[slot] = cur.oy;
        V.oz[slot] = cur.oz;
        V.vx[slot] = cur.vx;
        V.vy[slot] = cur.vy;
        V.vz[slot] = cur.vz;
        V.d[slot] = cur.d;
        V.id[slot] = cur.id;
    }
}

// Records the full re-bin places: the staged injections, or the movers the
// step recorded (all of them unless the mover list overflowed; those it
// could not record stayed in place).
template <class T>
__device__ __forceinline__ int64_t records(const RebinArgs<T> &a)
{
    const int64_t nm = a.flags[nmov_slot(a.epoch)];
    return a.npend + (nm < a.mcap ? nm : a.mcap);
}

// Full re-bin, first pass: particles per destination chunk, from the
// occupied slots (holes skipped) and the records.
template <class T>
__device__ void rekey_count(const RebinArgs<T> &a)
{
    const View<T> &V = a.V;
    if (blockIdx.x == 0 && threadIdx.x == 0) *a.room_denom = 0;
    const int64_t ni = *a.nitems;
    for (int64_t it = blockIdx.x; it < ni; it += gridDim.x) {
        const int64_t c = a.items[2 * it], seg = a.items[2 * it + 1];
        const int64_t s0 = V.base[c] + seg * kSeg;
        const int64_t s1 = min(s0 + (int64_t)kSeg, V.base[c] + (int64_t)V.cnt[c]);
        for (int64_t q = s0 + threadIdx.x; q < s1; q += blockDim.x) {
            T x = V.ox[q], y = V.oy[q], z = V.oz[q];
            const bool live = occupied(x, V.d[q]);
            const int64_t cn = live ? chunk_of_stored(a.p, c, x, y, z) : -1;
            // one atomic per wave for the lanes that stay in chunk c
            const uint64_t stay = __ballot(cn == c);
            if (cn == c) {
                if (__lane_id() == __ffsll((unsigned long long)stay) - 1)
                    atomicAdd(&a.new_cnt[c], __popcll(stay));
            } else if (live) {
                atomicAdd(&a.new_cnt[cn], 1);
            }
        }
    }
    const int64_t nr = records(a);
    for (int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; m < nr;
         m += (int64_t)gridDim.x * blockDim.x)
        atomicAdd(&a.new_cnt[a.mv.dest[m]], 1);
}

template <class T>
__global__ void __launch_bounds__(kArriveBlock) k_arrive_or_count(RebinArgs<T> a)
{
    if (full_rebin(a.flags, a.epoch)) rekey_count(a);
    else arrive(a);
}

template <class T>
__global__ void __launch_bounds__(256) k_counts(View<T> V, const int32_t *out_cnt,
                                                const int32_t *in_cnt, int64_t C, int32_t *flags,
                                                int32_t epoch)
{
    if (full_rebin(flags, epoch)) return;
    int32_t dead = 0;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < C;
         c += (int64_t)gridDim.x * blockDim.x)
        dead += count_chunk(V, out_cnt, in_cnt, c);
    int32_t total;
    block_excl_scan<int32_t>(dead, total);
    if (threadIdx.x == 0 && total) atomicAdd(&flags[F_DEAD], total);
}

// Full re-bin, second pass: scatter into the second store.
template <class T>
__global__ void __launch_bounds__(256) k_rekey_scatter(RebinArgs<T> a)
{
    if (!full_rebin(a.flags, a.epoch)) return;
    const View<T> &V = a.V;
    const View<T> &W = a.W;
    const int64_t ni = *a.nitems;
    for (int64_t it = blockIdx.x; it < ni; it += gridDim.x) {
        const int64_t c = a.items[2 * it], seg = a.items[2 * it + 1];
        const int64_t s0 = V.base[c] + seg * kSeg;
        const int64_t s1 = min(s0 + (int64_t)kSeg, V.base[c] + (int64_t)V.cnt[c]);
        for (int64_t q = s0 + threadIdx.x; q < s1; q += blockDim.x) {
            T x = V.ox[q], y = V.oy[q], z = V.oz[q];
            const T dd = V.d[q];
            const bool live = occupied(x, dd);      // holes are dropped
            const int64_t cn = live ? chunk_of_stored(a.p, c, x, y, z) : -1;
            int64_t dst = -1;
            const uint64_t stay = __ballot(cn == c);
            if (cn == c) {
                const int leader = __ffsll((unsigned long long)stay) - 1;
                int32_t b = 0;
                if (__lane_id() == leader) b = atomicAdd(&a.cursor[c], __popcll(stay));
                b = __shfl(b, leader, 64);
                dst = a.nbase[c] + b + __popcll(stay & lanes_below_mask());
            } else if (live) {
                dst = a.nbase[cn] + atomicAdd(&a.cursor[cn], 1);
            }
            if (!live) continue;
            W.ox[dst] = x;
            W.oy[dst] = y;
            W.oz[dst] = z;
            W.vx[dst] = V.vx[q];
            W.vy[dst] = V.vy[q];
            W.vz[dst] = V.vz[q];
            W.d[dst] = dd;
            W.id[dst] = V.id[q];
        }
    }
    const int64_t nr = records(a);
    for (int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; m < nr;
         m += (int64_t)gridDim.x * blockDim.x) {
        const int64_t cn = a.mv.dest[m];
        const int64_t dst = a.nbase[cn] + atomicAdd(&a.cursor[cn], 1);
        place_mover(W, dst, a.mv, m);
    }
}

// Full re-bin, last pass: the second store and the new layout become the store.
template <class T>
__global__ void k_rekey_commit(RebinArgs<T> a, ItemArgs ia, int items_here)
{
    if (!full_rebin(a.flags, a.epoch)) return;
    const View<T> &V = a.V;
    const View<T> &W = a.W;
    const int64_t g0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t gs = (int64_t)gridDim.x * blockDim.x;
    for (int64_t q = g0; q < a.slots; q += gs) {
        V.ox[q] = W.ox[q];
        V.oy[q] = W.oy[q];
        V.oz[q] = W.oz[q];
        V.vx[q] = W.vx[q];
        V.vy[q] = W.vy[q];
        V.vz[q] = W.vz[q];
        V.d[q] = W.d[q];
        V.id[q] = W.id[q];
    }
    for (int64_t c = g0; c < a.C; c += gs) {
        V.cnt[c] = a.new_cnt[c];
        V.ndead[c] = 0;
        V.base[c] = a.nbase[c];
        V.room[c] = a.nroom[c];
        a.new_cnt[c] = 0;   // ready for the next full re-bin
        a.cursor[c] = 0;
        if (items_here) write_items(ia, c);
    }
    if (g0 == 0) {
        a.flags[F_DEAD] = 0;
        if (items_here) finish_flags(ia);
        a.flags[F_REPACKS] += 1;
    }
}

// ---------------------------------------------------------------------------
// inject: binary64 global positions -> chunk + chunk-local offsets, staged
// ---------------------------------------------------------------------------
template <class T>
__global__ void k_stage(int64_t n, const double *x, const double *up, const double *d,
                        int64_t at, int64_t id0, Params p, Movers<T> mv, int32_t *flags)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        bool ok = true;
        int64_t ch[3];
        T loc[3];
        for (int a = 0; a < 3; ++a) {
            double xa = x[3 * i + a];
            if (!isfinite(xa)) { ok = false; xa = 0.0; }
            // periodic image in [0, L)
            xa = xa - floor(xa / p.L[a]) * p.L[a];
            if (xa >= p.L[a] || xa < 0.0) xa = 0.0;
            if (p.global) {   // binary32 metres; its cell from the binary32 product
                float xf = (float)xa;
                if (xf >= p.Lf[a]) xf = 0.f;
                ch[a] = gcell(xf, p.inv_hf[a], p.n[a]) / p.E;
                loc[a] = (T)xf;
                continue;
            }
            double g = xa / p.h[a];                  // cell units
            int64_t ci = (int64_t)floor(g);
            if (ci >= p.n[a]) { g -= p.n[a]; ci -= p.n[a]; }
            if (ci < 0) { g += p.n[a]; ci += p.n[a]; }
            ch[a] = ci / p.E;
            T o = (T)(g - (double)(ch[a] * p.E));   // exact before the rounding to T
            const int k = rebase(o, T(p.E), T(1) / T(p.E));
            ch[a] = wrapi(ch[a] + k, p.nc[a]);
            loc[a] = o;
        }
        const double v[3] = {up[3 * i], up[3 * i + 1], up[3 * i + 2]};
        const double dd = d[i];
        for (int a = 0; a < 3; ++a)
            if (!isfinite(v[a])) ok = false;
        if (!isfinite(dd) || !(dd > 0.0)) ok = false;
        const int64_t m = at + i;
        mv.rec[m] = MoverRec<T>{loc[0], loc[1], loc[2], (T)v[0], (T)v[1], (T)v[2], (T)dd,
                                (int32_t)(id0 + i)};
        mv.dest[m] = (int32_t)chunk_index(p, ch[0], ch[1], ch[2]);
        if (!ok) flags[F_BADINPUT] = 1;
    }
}

// ---------------------------------------------------------------------------
// outputs
// ---------------------------------------------------------------------------
template <class T>
__global__ void __launch_bounds__(256) k_get_particles(View<T> V, const int32_t *items,
                                                       const int32_t *nitems, Params p,
                                                       int64_t count, double *x, double *up,
                                                       double *d, int64_t *id, int32_t *cell)
{
    const int64_t ni = *nitems;
    for (int64_t it = blockIdx.x; it < ni; it += gridDim.x) {
        const int64_t c = items[2 * it], seg = items[2 * it + 1];
        const int64_t cc[3] = {c % p.nc[0], (c / p.nc[0]) % p.nc[1],
                               c / ((int64_t)p.nc[0] * p.nc[1])};
        const int64_t s0 = V.base[c] + seg * kSeg;
        const int64_t s1 = min(s0 + (int64_t)kSeg, V.base[c] + (int64_t)V.cnt[c]);
        for (int64_t q = s0 + threadIdx.x; q < s1; q += blockDim.x) {
            if (!occupied(V.ox[q], V.d[q])) continue;   // a hole
            const int64_t k = V.id[q];
            if (k < 0 || k >= count) continue;  // never in a consistent store
            const T o[3] = {V.ox[q], V.oy[q], V.oz[q]};
            const T v[3] = {V.vx[q], V.vy[q], V.vz[q]};
            for (int a = 0; a < 3; ++a) {
                const double org = (double)(cc[a] * p.E);
                if (p.global) {   // binary32 metres
                    if (x) x[3 * k + a] = (double)o[a];
                    if (cell) cell[3 * k + a] = gcell((float)o[a], p.inv_hf[a], p.n[a]);
                } else {
                    if (x) x[3 * k + a] = (org + (double)o[a]) * p.h[a];
                    if (cell)
                        cell[3 * k + a] = (int32_t)(cc[a] * p.E + min(max((int)o[a], 0), p.E - 1));
                }
                if (up) up[3 * k + a] = (double)v[a];
            }
            if (d) d[k] = (double)V.d[q];
            if (id) id[k] = k;
        }
    }
}

template <class A>
__global__ void k_get_sources(A *src, Params p, double *out, int reset)
{
    const int64_t nx = p.n[0], ny = p.n[1], nz = p.n[2];
    const int64_t ncell = nx * ny * nz;
    const int E = p.E;
    const int64_t E3 = (int64_t)E * E * E;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < 3 * ncell;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t comp = t / ncell;
        const int64_t r = t - comp * ncell;
        const int64_t i = r % nx, j = (r / nx) % ny, k = r / (nx * ny);
        const int64_t c = ((k / E) * p.nc[1] + (j / E)) * p.nc[0] + (i / E);
        const int64_t l = ((k % E) * E + (j % E)) * E + (i % E);
        A *s = src + c * 3 * E3 + comp * E3 + l;
        out[t] = (double)*s;
        if (reset) *s = A(0);
    }
}

template <class A>
__global__ void k_fill_acc(A *p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = A(0);
}

__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_fill_i64(int64_t *p, int64_t n, int64_t v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// synthetic fluid update: U^k = R_z(theta_k) U^0, rounded once to T
template <class T>
__global__ void k_rotate(const T *u0, T *u, int64_t ncell, double cs, double sn)
{
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < ncell;
         q += (int64_t)gridDim.x * blockDim.x) {
        const double ux = (double)u0[q], uy = (double)u0[ncell + q];
        u[q] = (T)(cs * ux - sn * uy);
        u[ncell + q] = (T)(sn * ux + cs * uy);
        u[2 * ncell + q] = u0[2 * ncell + q];
    }
}

// checkpoint copy of the store (all slots), its hole lists and its layout
template <class T>
__global__ void k_snapshot(View<T> V, int32_t *hole, int64_t slots, int64_t C, char *buf,
                           SnapLayout L, int32_t *items, const int32_t *nitems, int64_t max_items,
                           int restore)
{
    T *arr[7] = {V.ox, V.oy, V.oz, V.vx, V.vy, V.vz, V.d};
    T *sT = reinterpret_cast<T *>(buf + L.state);
    int32_t *sid = reinterpret_cast<int32_t *>(buf + L.id);
    int32_t *shole = reinterpret_cast<int32_t *>(buf + L.hole);
    int64_t *sbase = reinterpret_cast<int64_t *>(buf + L.base);
    int32_t *sroom = reinterpret_cast<int32_t *>(buf + L.room);
    int32_t *scnt = reinterpret_cast<int32_t *>(buf + L.cnt);
    int32_t *sndead = reinterpret_cast<int32_t *>(buf + L.ndead);
    int32_t *sitems = reinterpret_cast<int32_t *>(buf + L.items);
    int32_t *snitems = reinterpret_cast<int32_t *>(buf + L.nitems);
    const int64_t g0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (!restore) {  // the work items of this layout travel with it
        const int64_t ni = *nitems;
        for (int64_t k = g0; k < 2 * ni; k += (int64_t)gridDim.x * blockDim.x)
            sitems[k] = items[k];
        if (g0 == 0) *snitems = (int32_t)ni;
    }
    (void)max_items;
    const int64_t gs = (int64_t)gridDim.x * blockDim.x;
    for (int64_t q = g0; q < slots; q += gs) {
        if (restore) {
            for (int a = 0; a < 7; ++a) arr[a][q] = sT[a * slots + q];
            V.id[q] = sid[q];
            hole[q] = shole[q];
        } else {
            for (int a = 0; a < 7; ++a) sT[a * slots + q] = arr[a][q];
            sid[q] = V.id[q];
            shole[q] = hole[q];
        }
    }
    for (int64_t c = g0; c < C; c += gs) {
        if (restore) {
            V.base[c] = sbase[c];
            V.room[c] = sroom[c];
            V.cnt[c] = scnt[c];
            V.ndead[c] = sndead[c];
        } else {
            sbase[c] = V.base[c];
            sroom[c] = V.room[c];
            scnt[c] = V.cnt[c];
            sndead[c] = V.ndead[c];
        }
    }
}

// ---------------------------------------------------------------------------
// host-side helpers
// ---------------------------------------------------------------------------
inline int64_t grid_for(int64_t n, int64_t cap = 8192)
{
    int64_t g = (n + 255) / 256;
    if (g < 1) g = 1;
    return g > cap ? cap : g;
}

template <class T>
View<T> view_of(st_ctx *c, int b)
{
    View<T> v;
    v.ox = (T *)c->store[b][0];
    v.oy = (T *)c->store[b][1];
    v.oz = (T *)c->store[b][2];
    v.vx = (T *)c->store[b][3];
    v.vy = (T *)c->store[b][4];
    v.vz = (T *)c->store[b][5];
    v.d = (T *)c->store[b][6];
    v.id = (int32_t *)c->store[b][7];
    v.base = c->base;
    v.room = c->room;
    v.cnt = c->cnt;
    v.ndead = c->ndead;
    return v;
}

template <class T>
Movers<T> movers_of(st_ctx *c)
{
    Movers<T> m;
    m.rec = (MoverRec<T> *)c->mov[0];
    m.dest = (int32_t *)c->mov[1];
    m.rank = (int32_t *)c->mov[2];
    return m;
}

// more holes than this force a full re-bin (a sixteenth of the particles)
inline int32_t dead_limit(const st_ctx *c)
{
    const int64_t v = c->count / 16 + 1024;
    return (int32_t)(v < 0x7fffffff ? v : 0x7fffffff);
}

template <class F>
hipError_t dispatch(st_ctx *c, F &&f)
{
    switch (c->form) {
    case ST_FORM_FP64: return f(double(0), double(0));
    case ST_FORM_FP32_LOCAL: return f(float(0), double(0));
    default: return f(float(0), float(0));
    }
}

// ev[0], ev[1] (when not null) take the start and end of the kernel's own
// execution (not of the commands around it)
template <class T, class A, int E, int I, int D>
hipError_t launch_step_t(st_ctx *c, const StepArgs<T, A> &a, hipStream_t s, hipEvent_t *ev)
{
    const int64_t round = 8 * kXcdBlock;
    const int64_t grid = (c->max_items + round - 1) / round * round;
    if constexpr (sizeof(A) == 8) {   // only the forms that tape save
        if (a.sv[0]) {
            hipLaunchKernelGGL((k_step<T, A, E, I, D, true>), dim3(grid), dim3(kBlock), 0, s, a);
            return hipGetLastError();
        }
    }
    if (ev[0])
        hipExtLaunchKernelGGL((k_step<T, A, E, I, D, false>), dim3(grid), dim3(kBlock), 0, s,
                              ev[0], ev[1], 0, a);
    else
        hipLaunchKernelGGL((k_step<T, A, E, I, D, false>), dim3(grid), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

template <class T, class A, int E, int I>
hipError_t launch_step_d(st_ctx *c, const StepArgs<T, A> &a, hipStream_t s, hipEvent_t *ev)
{
    return c->prm.drag == 1 ? launch_step_t<T, A, E, I, 1>(c, a, s, ev)
                            : launch_step_t<T, A, E, I, 0>(c, a, s, ev);
}

template <class T, class A, int E>
hipError_t launch_step_e(st_ctx *c, const StepArgs<T, A> &a, hipStream_t s, hipEvent_t *ev)
{
    return c->prm.interp == 1 ? launch_step_d<T, A, E, 1>(c, a, s, ev)
                              : launch_step_d<T, A, E, 0>(c, a, s, ev);
}

template <class T>
RebinArgs<T> rebin_args(st_ctx *c, int64_t npend)
{
    RebinArgs<T> a;
    a.V = view_of<T>(c, 0);
    a.W = view_of<T>(c, 1);
    a.mv = movers_of<T>(c);
    a.C = c->C;
    a.out_cnt = c->out_cnt;
    a.in_cnt = c->in_cnt;
    a.hole = c->hole;
    a.items = c->items;
    a.nitems = c->flags + F_NITEMS;
    a.p = c->prm;
    a.npend = npend;
    a.mcap = c->mcap;
    a.new_cnt = c->new_cnt;
    a.cursor = c->cursor;
    a.nbase = c->nbase;
    a.nroom = c->nroom;
    a.room_denom = c->room_denom;
    a.slots = c->slots;
    a.flags = c->flags;
    a.epoch = c->epoch;
    return a;
}

// everything after the step kernel: arrivals or full re-bin, then the items
template <class T>
hipError_t launch_rebin(st_ctx *c, int64_t npend, hipStream_t s)
{
    const RebinArgs<T> a = rebin_args<T>(c, npend);
    const int64_t C = c->C;
    // a thread per mover for the arrivals (at most mcap of them); the count
    // (rare) strides over the items
    int64_t g = std::max<int64_t>((c->mcap + kArriveBlock - 1) / kArriveBlock, c->max_items);
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL((k_arrive_or_count<T>), dim3(g), dim3(kArriveBlock), 0, s, a);
    const int64_t total = c->count + npend;
    const RoomWeight rw{c->new_cnt, {c->prm.nc[0], c->prm.nc[1], c->prm.nc[2]}};
    const Rooms rooms{rw, c->slots - total - (int64_t)kAlign * C, 0, c->nroom};
    // the full re-bin launches run every step and usually exit at their gate:
    // grids of at most 2048 workgroups (strided loops) keep that cheap
    const int64_t gs = c->max_items < 2048 ? c->max_items : 2048;
    ItemArgs ia{C, c->nseg, c->items, c->out_cnt, c->in_cnt, c->new_cnt, c->cursor, c->flags,
                c->epoch, dead_limit(c)};
    if (C <= kScan1Max) {
        // counts, rooms (when due) and the next items in one workgroup
        hipLaunchKernelGGL((k_layout1<T>), dim3(1), dim3(1024), 0, s, rooms, c->nbase,
                           Segments{c->new_cnt}, ia, a.V, c->flags);
        hipLaunchKernelGGL((k_rekey_scatter<T>), dim3(gs), dim3(256), 0, s, a);
        hipLaunchKernelGGL((k_rekey_commit<T>), dim3(grid_for(c->slots, 2048)), dim3(256), 0, s,
                           a, ia, 1);
        return hipGetLastError();
    }
    hipLaunchKernelGGL((k_counts<T>), dim3(grid_for(C)), dim3(256), 0, s, a.V, c->out_cnt,
                       c->in_cnt, C, c->flags, c->epoch);
    hipLaunchKernelGGL(k_room_denom, dim3((C + kScanBlock - 1) / kScanBlock), dim3(256), 0, s, rw,
                       C, c->room_denom, c->flags, c->epoch);
    hipError_t e = scan<int64_t>(RoomsDev{rooms, c->room_denom}, C, c->nbase, c->scan_tmp,
                                 c->flags, G_FULL, c->epoch, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_rekey_scatter<T>), dim3(gs), dim3(256), 0, s, a);
    hipLaunchKernelGGL((k_rekey_commit<T>), dim3(grid_for(c->slots, 2048)), dim3(256), 0, s, a,
                       ia, 0);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_items(c, s);
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_items(st_ctx *c, hipStream_t s)
{
    ItemArgs a{c->C, c->nseg, c->items, c->out_cnt, c->in_cnt, c->new_cnt, c->cursor, c->flags,
               c->epoch, dead_limit(c)};
    if (c->C <= kScan1Max) {
        hipLaunchKernelGGL(k_items1, dim3(1), dim3(1024), 0, s, Segments{c->cnt}, a);
        return hipGetLastError();
    }
    hipError_t e = scan_multi<int32_t>(Segments{c->cnt}, c->C, c->nseg, (int32_t *)c->scan_tmp,
                                       c->flags, G_ALWAYS, c->epoch, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_items, dim3(grid_for(c->C)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_init(st_ctx *c, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(c->C)), dim3(256), 0, s, c->cnt, c->C, 0);
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(c->C)), dim3(256), 0, s, c->room, c->C, 0);
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(c->C)), dim3(256), 0, s, c->ndead, c->C, 0);
    hipLaunchKernelGGL(k_fill_i64, dim3(grid_for(c->C + 1)), dim3(256), 0, s, c->base, c->C + 1,
                       (int64_t)0);
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(256), 0, s, c->flags, (int64_t)F_COUNT, 0);
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(c->C)), dim3(256), 0, s, c->new_cnt, c->C, 0);
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(c->C)), dim3(256), 0, s, c->cursor, c->C, 0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_items(c, s);
}

hipError_t launch_step(st_ctx *c, const void *u, double dt, int deposit, hipStream_t s,
                       void *save)
{
    c->epoch += 1;
    return dispatch(c, [&](auto t, auto acc) -> hipError_t {
        using T = decltype(t);
        using A = decltype(acc);
        StepArgs<T, A> a;
        a.V = view_of<T>(c, 0);
        for (int k = 0; k < 7; ++k) a.sv[k] = nullptr;
        if (save) {
            const SnapLayout L = snap_layout(c->slots, c->tsize, c->C, c->max_items);
            char *b = (char *)save;
            for (int k = 0; k < 7; ++k) a.sv[k] = (T *)(b + L.state) + k * c->slots;
            a.sid = (int32_t *)(b + L.id);
            a.sitems = (int32_t *)(b + L.items);
            a.snitems = (int32_t *)(b + L.nitems);
            a.sbase = (int64_t *)(b + L.base);
            a.scnt = (int32_t *)(b + L.cnt);
        }
        a.items = c->items;
        a.nitems = c->flags + F_NITEMS;
        a.u = (const T *)u;
        a.src = (A *)c->src;
        a.mv = movers_of<T>(c);
        a.nmov = c->flags + nmov_slot(c->epoch);
        a.mcap = c->mcap;
        a.out_cnt = c->out_cnt;
        a.in_cnt = c->in_cnt;
        a.hole = c->hole;
        a.flags = c->flags;
        a.deposit = deposit;
        a.epoch = c->epoch;
        a.p = c->prm;
        a.dt = (T)dt;
        for (int ax = 0; ax < 3; ++ax) {
            a.dt_h[ax] = (T)(dt / c->prm.h[ax]);
            a.g[ax] = (T)c->prm.g[ax];
        }
        a.tau_coef = (T)c->prm.tau_coef;
        for (int ax = 0; ax < 3; ++ax) a.g_dt[ax] = (T)(c->prm.g[ax] * dt);
        a.mass_coef = (T)c->prm.mass_coef;
        a.inv_V = (T)c->prm.inv_V;
        a.re2_coef = (T)(c->prm.re_coef * c->prm.re_coef);
        hipEvent_t ev[2] = {nullptr, nullptr};
        if (c->timing) {
            for (int k = 0; k < 2; ++k) {
                hipError_t ee = hipEventCreate(&ev[k]);
                if (ee != hipSuccess) return ee;
                c->tev.push_back(ev[k]);
            }
        }
        hipError_t r;
        switch (c->prm.E) {
        case 2: r = launch_step_e<T, A, 2>(c, a, s, ev); break;
        case 4: r = launch_step_e<T, A, 4>(c, a, s, ev); break;
        default: r = launch_step_e<T, A, 8>(c, a, s, ev); break;
        }
        if (r != hipSuccess) return r;

        return launch_rebin<T>(c, 0, s);
    });
}

hipError_t launch_flush_pending(st_ctx *c, hipStream_t s)
{
    c->epoch += 1;
    hipLaunchKernelGGL(k_set_flag, dim3(1), dim3(1), 0, s, c->flags, (int)F_FORCE, c->epoch);
    return dispatch(c, [&](auto t, auto) -> hipError_t {
        using T = decltype(t);
        return launch_rebin<T>(c, c->pending, s);
    });
}

hipError_t launch_stage_inject(st_ctx *c, int64_t n, const double *x, const double *up,
                               const double *d, int64_t at, hipStream_t s)
{
    return dispatch(c, [&](auto t, auto) -> hipError_t {
        using T = decltype(t);
        hipLaunchKernelGGL((k_stage<T>), dim3(grid_for(n)), dim3(256), 0, s, n, x, up, d, at,
                           c->next_id, c->prm, movers_of<T>(c), c->flags);
        return hipGetLastError();
    });
}

hipError_t launch_get_particles(st_ctx *c, double *x, double *up, double *d, int64_t *id,
                                int32_t *cell, hipStream_t s)
{
    return dispatch(c, [&](auto t, auto) -> hipError_t {
        using T = decltype(t);
        const int64_t gi = c->max_items < 65536 ? c->max_items : 65536;
        hipLaunchKernelGGL((k_get_particles<T>), dim3(gi), dim3(256), 0, s, view_of<T>(c, 0),
                           c->items, c->flags + F_NITEMS, c->prm, c->count, x, up, d, id, cell);
        return hipGetLastError();
    });
}

hipError_t launch_get_sources(st_ctx *c, double *out, int reset, hipStream_t s)
{
    return dispatch(c, [&](auto, auto acc) -> hipError_t {
        using A = decltype(acc);
        const int64_t n = 3 * (int64_t)c->prm.n[0] * c->prm.n[1] * c->prm.n[2];
        hipLaunchKernelGGL((k_get_sources<A>), dim3(grid_for(n, 16384)), dim3(256), 0, s,
                           (A *)c->src, c->prm, out, reset);
        return hipGetLastError();
    });
}

hipError_t launch_zero_sources(st_ctx *c, hipStream_t s)
{
    return dispatch(c, [&](auto, auto acc) -> hipError_t {
        using A = decltype(acc);
        const int64_t n = 3 * (int64_t)c->prm.n[0] * c->prm.n[1] * c->prm.n[2];
        hipLaunchKernelGGL((k_fill_acc<A>), dim3(grid_for(n, 16384)), dim3(256), 0, s,
                           (A *)c->src, n);
        return hipGetLastError();
    });
}

hipError_t launch_zero_i32(int32_t *p, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n)), dim3(256), 0, s, p, n, 0);
    return hipGetLastError();
}

hipError_t launch_rotate_field(st_ctx *c, const void *u0, void *out, double cs, double sn,
                               hipStream_t s)
{
    return dispatch(c, [&](auto t, auto) -> hipError_t {
        using T = decltype(t);
        const int64_t ncell = (int64_t)c->prm.n[0] * c->prm.n[1] * c->prm.n[2];
        hipLaunchKernelGGL((k_rotate<T>), dim3(grid_for(ncell, 16384)), dim3(256), 0, s,
                           (const T *)u0, (T *)out, ncell, cs, sn);
        return hipGetLastError();
    });
}

// streaming reference: a plain copy with the particle state's access pattern
// (one 16-byte non-temporal load and store per thread)
typedef float f32x4 __attribute__((ext_vector_type(4)));
__global__ void __launch_bounds__(1024) k_stream_copy(const f32x4 *src, f32x4 *dst, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

hipError_t launch_stream_copy(const void *src, void *dst, int64_t bytes, hipStream_t s)
{
    const int64_t n = bytes / 16;
    int64_t g = (n + 1023) / 1024;
    if (g < 1) g = 1;
    if (g > (1 << 20)) g = 1 << 20;
    hipLaunchKernelGGL(k_stream_copy, dim3(g), dim3(1024), 0, s, (const f32x4 *)src,
                       (f32x4 *)dst, n);
    return hipGetLastError();
}

// extrapolator-corrector, elementwise over cells and components
__global__ void k_ec(int64_t n, int kind, const double *S_last, double *S_prev, double *E_prev,
                     double *applied)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double s = S_last[i];
        const double corrector = s - E_prev[i];
        double e = 0.0;
        if (kind == 1) e = s;
        if (kind == 2) e = 2.0 * s - S_prev[i];
        applied[i] = corrector + e;
        E_prev[i] = e;
        S_prev[i] = s;
    }
}

__global__ void k_zero_f64(double *p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

hipError_t launch_ec(st_ctx *c, int kind, const double *S_last, double *applied, hipStream_t s)
{
    const int64_t n = 3 * (int64_t)c->prm.n[0] * c->prm.n[1] * c->prm.n[2];
    hipLaunchKernelGGL(k_ec, dim3(grid_for(n, 16384)), dim3(256), 0, s, n, kind, S_last,
                       c->ec_prev, c->ec_ext, applied);
    return hipGetLastError();
}

hipError_t launch_zero_f64(double *p, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_f64, dim3(grid_for(n, 16384)), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

size_t snapshot_bytes(const st_ctx *c)
{
    return snap_layout(c->slots, c->tsize, c->C, c->max_items).bytes;
}

// Saves the store, its layout and its work items into dst, or (restore)
// puts a saved store and layout back and rebuilds the work items.
hipError_t launch_snapshot(st_ctx *c, void *dst, int restore, hipStream_t s)
{
    const SnapLayout L = snap_layout(c->slots, c->tsize, c->C, c->max_items);
    hipError_t e = dispatch(c, [&](auto t, auto) -> hipError_t {
        using T = decltype(t);
        hipLaunchKernelGGL((k_snapshot<T>), dim3(grid_for(c->slots, 16384)), dim3(256), 0, s,
                           view_of<T>(c, 0), c->hole, c->slots, c->C, (char *)dst, L, c->items,
                           c->flags + F_NITEMS, c->max_items, restore);
        return hipGetLastError();
    });
    if (e != hipSuccess || !restore) return e;
    return launch_items(c, s);
}

}  // namespace st
