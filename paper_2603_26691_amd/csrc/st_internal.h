// Internal declarations of the scaletrack HIP library (not part of the ABI).
//
// Particle store: structure of arrays, kept sorted by chunk (a cube of
// E^3 cells, E = chunk_edge).  Chunk c owns the slot range
// [base[c], base[c] + room[c]); its particles sit in the first cnt[c] slots
// of that range, among ndead[c] holes: slots a particle left (a -1 offset in
// binary32, a negative diameter in binary64), listed (relative to base[c])
// at hole[base[c] .. base[c] + ndead[c]).  Arrivals fill holes first.
// Positions are stored as chunk-local offsets in cell units, xi in [0, E)
// per axis; the chunk origin is exact (the chunk index times E cells).  The
// FP32-everywhere form stores binary32 coordinates in metres instead, and
// takes the cell from their binary32 product with n / L.  Kernels get the
// store's pointers as arguments (so
// every access is a global-memory instruction); a full re-bin scatters into
// a second store and copies back.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "st.h"

namespace st {

constexpr int kBlock = 256;       // threads per workgroup of the step kernels
constexpr int kSeg = 16384;       // max particles per step work item
constexpr int kSlackMin = 32;     // spare-slot weight per chunk in the room formula
constexpr int kMoverStage = 512;  // movers per workgroup staged in LDS
constexpr int kAlign = 4;         // chunk rooms are whole multiples of this
// The state arrays are streamed together at equal slot indices; array k of
// store b starts (8 b + k) kStagger bytes into its allocation, so that equal
// indices of different arrays do not fall on the same HBM channels (aligned
// starts measured 14 % slower on the 1.4e9-particle plume workload; staggers
// of 1 KiB to 17 KiB all remove it, 256 B does not).
constexpr size_t kStagger = 4096 + 256;
// partitions st_bounding_boxes_noalloc can take (its fixed device scratch)
constexpr int64_t kNoAllocMaxParts = 65536;

template <class T>
struct View {
    T *ox, *oy, *oz;   // chunk-local offsets [cells] (FP32-everywhere form: metres)
    T *vx, *vy, *vz;   // velocity [m/s]
    T *d;              // diameter [m]; binary64: -d marks a hole (the state
                       // of the particle that left it is still in place)
    int32_t *id;       // particle id
    int64_t *base;     // [C] first slot of the chunk
    int32_t *room;     // [C] slots owned by the chunk
    int32_t *cnt;      // [C] slots in use: particles and holes
    int32_t *ndead;    // [C] holes among them
};

// One particle in flight between chunks (also the staging area of
// st_inject), kept together so that moving it reads and writes whole
// 16-byte vectors: 32 bytes in binary32, 64 in binary64.
template <class T>
struct alignas(16) MoverRec {
    T ox, oy, oz, vx, vy, vz, d;
    int32_t id;
};
static_assert(sizeof(MoverRec<float>) == 32, "binary32 mover record is 32 bytes");
static_assert(sizeof(MoverRec<double>) == 64, "binary64 mover record is 64 bytes");

template <class T>
struct Movers {
    MoverRec<T> *rec;
    int32_t *dest;     // destination chunk
    int32_t *rank;     // rank among the destination's arrivals of the step
};

// Scalars of the mesh and material used by the kernels.
struct Params {
    int32_t n[3];          // cells per axis
    int32_t nc[3];         // chunks per axis
    int32_t E;             // chunk edge
    int32_t interp;        // 0 trilinear, 1 nearest grid point
    int32_t drag;          // 0 Stokes, 1 Schiller-Naumann
    int32_t pad_;
    int64_t C;             // chunks
    double L[3];           // domain extent
    double h[3];           // cell widths
    double inv_h[3];
    double inv_V;          // 1 / cell volume
    double g[3];
    double tau_coef;       // rho_p / (18 mu_f): tau = tau_coef d^2
    double mass_coef;      // w rho_p pi / 6:    m = mass_coef d^3
    double re_coef;        // rho_f / mu_f:      Re = re_coef d |u_f - u_p|
    // FP32-everywhere form: positions are stored as binary32 coordinates in
    // metres (global != 0); its cell arithmetic in binary32
    float inv_hf[3];       // binary32 n / L per axis
    float Lf[3];           // binary32 L per axis
    int32_t global;
    int32_t pad2_;
};

// Flags and counters on the device (one int32 each).  F_OVERFLOW and
// F_FORCE hold the tag (epoch) of the step or flush that raised them; the
// movers of a step are counted in F_NMOV or F_NMOV_ODD by the tag's parity.
// F_DEAD counts the holes of the store after the last arrivals.
enum DevFlag { F_OVERFLOW = 0, F_NMOV = 1, F_NITEMS = 2, F_FORCE = 3, F_BADINPUT = 4,
               F_REPACKS = 5, F_LASTMOV = 6, F_NMOV_ODD = 7, F_DEAD = 8, F_COUNT = 9 };

struct TapeStep {
    const void *u;     // field of the step (borrowed)
    double dt;         // sub-step length
};

struct Snapshot {      // particle store and layout at a checkpoint
    void *buf = nullptr;
    size_t bytes = 0;
};

// Byte offsets inside a snapshot: the 7 state arrays ([7][slots] of the
// state scalar), ids, the hole lists, the chunk layout (base, room, cnt,
// ndead) and the work items of that layout with their count.
struct SnapLayout {
    size_t state, id, hole, base, room, cnt, ndead, items, nitems, bytes;
};

inline SnapLayout snap_layout(int64_t slots, size_t tsize, int64_t C, int64_t max_items)
{
    auto up8 = [](size_t v) { return (v + 7) & ~(size_t)7; };
    SnapLayout l;
    l.state = 0;
    l.id = 7 * (size_t)slots * tsize;
    l.hole = l.id + (size_t)slots * 4;
    l.base = up8(l.hole + (size_t)slots * 4);
    l.room = l.base + (size_t)C * 8;
    l.cnt = l.room + (size_t)C * 4;
    l.ndead = l.cnt + (size_t)C * 4;
    l.items = up8(l.ndead + (size_t)C * 4);
    l.nitems = l.items + (size_t)max_items * 8;
    l.bytes = up8(l.nitems + 4);
    return l;
}

}  // namespace st

struct st_ctx {
    st_mesh_desc desc;
    st::Params prm;
    int device = 0;
    int form = 0;
    size_t tsize = 8;          // bytes of the state scalar
    size_t asize = 8;          // bytes of the source accumulator
    int64_t C = 0;             // chunks
    int64_t cap = 0;           // particle capacity
    int64_t slots = 0;         // slots per store
    int64_t mcap = 0;          // mover / staging capacity
    int64_t max_items = 0;     // upper bound of step work items
    int64_t count = 0;         // particles in the store (host mirror)
    int64_t pending = 0;       // injected particles waiting in the staging area
    int64_t next_id = 0;
    int32_t epoch = 0;         // tag of the last step or flush launched

    // device memory
    void *store[2][8] = {};    // SoA arrays: [0] the store, [1] re-bin target
    void *store_raw[2][8] = {};  // their allocations (the arrays start past a stagger)
    int64_t *base = nullptr;   // [C+1] layout of the store
    int32_t *room = nullptr;   // [C]
    int32_t *cnt = nullptr;    // [C]
    int32_t *ndead = nullptr;  // [C]
    void *mov[3] = {};         // Movers: records, destination chunks, ranks
    int32_t *out_cnt = nullptr, *in_cnt = nullptr;
    int32_t *cursor = nullptr;     // [C] scatter cursors of the full re-bin
    int32_t *new_cnt = nullptr;    // [C]
    int64_t *nbase = nullptr;      // [C+1] first slots of the re-binned layout
    int32_t *nroom = nullptr;      // [C]   rooms of the re-binned layout
    int32_t *hole = nullptr;       // [slots] holes of chunk c from base[c]
    int32_t *items = nullptr;      // [max_items][2]
    int32_t *nseg = nullptr;       // [C+1] offsets of the work items per chunk
    int64_t *scan_tmp = nullptr;   // block partials of the scans
    int64_t *room_denom = nullptr; // [1] sum of the chunks' room weights
    int32_t *flags = nullptr;      // DevFlag counters
    void *src = nullptr;           // [C][3][E^3] accumulator (double or float)
    double *stage64 = nullptr;     // staging for host-side injects ([batch][7])

    // tape
    int tape_every = 0;
    std::vector<st::TapeStep> tape;
    std::vector<st::Snapshot> snaps;  // one per tape_every steps
    // kept from a consumed tape for the next one (released by st_tape_clear
    // and st_destroy): checkpoint buffers, and the workspace of st_backward
    // (the state at the end of the forward run, the saved states of one
    // segment, the adjoint records and dL/dS by chunk)
    std::vector<st::Snapshot> spare;
    void *bwd_ws = nullptr;
    size_t bwd_ws_bytes = 0;

    // coupled run
    void *fieldbuf[2] = {};
    hipStream_t side = nullptr;

    // extrapolator-corrector history ([3][ncell] binary64 each), allocated
    // on first use
    double *ec_prev = nullptr;     // S_last of the previous call
    double *ec_ext = nullptr;      // extrapolation made at the previous call

    // step-kernel timing (a pair of events attached to each launch)
    int timing = 0;
    std::vector<hipEvent_t> tev;   // pairs: start, stop

    std::string err;
};

namespace st {

// Kernel launchers (st_kernels.hip).  All enqueue on `s`.
hipError_t launch_init(st_ctx *c, hipStream_t s);
hipError_t launch_items(st_ctx *c, hipStream_t s);
hipError_t launch_flush_pending(st_ctx *c, hipStream_t s);
hipError_t launch_zero_sources(st_ctx *c, hipStream_t s);
hipError_t launch_zero_i32(int32_t *p, int64_t n, hipStream_t s);
// save (a snapshot buffer, or null): the step also writes there what its
// reverse reads (the state each slot starts with, ids and the layout)
hipError_t launch_step(st_ctx *c, const void *u, double dt, int deposit, hipStream_t s,
                       void *save = nullptr);
hipError_t launch_stage_inject(st_ctx *c, int64_t n, const double *x, const double *up,
                               const double *d, int64_t at, hipStream_t s);
hipError_t launch_get_particles(st_ctx *c, double *x, double *up, double *d, int64_t *id,
                                int32_t *cell, hipStream_t s);
hipError_t launch_get_sources(st_ctx *c, double *out, int reset, hipStream_t s);
hipError_t launch_rotate_field(st_ctx *c, const void *u0, void *out, double cs, double sn,
                               hipStream_t s);
hipError_t launch_snapshot(st_ctx *c, void *dst, int restore, hipStream_t s);
hipError_t launch_ec(st_ctx *c, int kind, const double *S_last, double *applied, hipStream_t s);
hipError_t launch_zero_f64(double *p, int64_t n, hipStream_t s);
size_t snapshot_bytes(const st_ctx *c);
hipError_t launch_backward(st_ctx *c, const double *lam, double *dU, double *dd, hipStream_t s);
// allocates st_backward's workspace for checkpoints every K sub-steps, if smaller
hipError_t reserve_backward(st_ctx *c, int64_t K);
hipError_t launch_hilbert_positions(int32_t order, int64_t nseg, int64_t seg_begin,
                                    int64_t per_seg, const double L[3], int64_t first, int64_t n,
                                    const double *u, double *x, hipStream_t s);
hipError_t launch_bounding_boxes(st_ctx *c, int64_t id0, int64_t per_part, int64_t nparts,
                                 double *box, hipStream_t s);
// The fixed device array of st_bounding_boxes_noalloc (st_hilbert.hip):
// noalloc_scratch_init takes this device's address of it (the device must be
// current; once per device, later calls return at once); noalloc_scratch
// returns that address, or an error if it was never taken.
hipError_t noalloc_scratch_init(int device);
hipError_t launch_stream_copy(const void *src, void *dst, int64_t bytes, hipStream_t s);
hipError_t noalloc_scratch(int device, double **ptr);

}  // namespace st
