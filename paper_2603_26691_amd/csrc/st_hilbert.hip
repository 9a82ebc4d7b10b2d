// Placement of new particles by Hilbert-curve segments, and bounding boxes of
// particle partitions (paper Sec. 2.2, initialisation and chunk bounding
// boxes).
//
// Placement: the domain is a lattice of 2^order voxels per axis, visited in
// Hilbert-curve order and cut into nseg consecutive segments; segment s holds
// curve positions [floor(s V / nseg), floor((s+1) V / nseg)), V = 8^order.
// Particle k of a segment with nv voxels lies in its voxel floor(k nv / per_seg),
// at x_a = (c_a + u_a) (L_a / 2^order) for given uniforms u in [0, 1)^3: every
// segment holds exactly per_seg particles, voxel counts differ by at most one,
// and the particles follow the curve.  The mapping is global and
// deterministic, so any range of segments can be placed independently.
//
// Bounding boxes: partition p holds the particles with id in
// [id0 + p per_part, id0 + (p+1) per_part); its box is the componentwise
// minimum and maximum of their positions (positions as st_get_particles
// returns them).
#include "st_internal.h"

#include <mutex>

// Partial results of st_bounding_boxes_noalloc (the min and max bounds of up
// to kNoAllocMaxParts boxes, as ordered integer images of binary64): a fixed
// device array, one copy per GPU, held until the process ends, so that the
// call allocates nothing.  Host code never passes this name to a kernel or a
// copy (on the host it is a stand-in, not a device address); it uses the
// per-device address that noalloc_scratch_init takes.
static __device__ __align__(256) unsigned long long scratch[st::kNoAllocMaxParts * 6];

namespace st {
namespace {

// Hilbert curve position h -> voxel: the index is split into its transpose
// (bit level l of axis i is bit 3 l + 2 - i of h), then Skilling's
// transpose-to-axes (AIP Conf. Proc. 707, 2004): Gray decode, then undo the
// reflections and exchanges from the least significant level up.
__device__ void hilbert_voxel(int order, int64_t h, int32_t c[3])
{
    uint32_t X[3] = {0u, 0u, 0u};
    for (int l = 0; l < order; ++l)
        for (int i = 0; i < 3; ++i)
            X[i] |= (uint32_t)((h >> (3 * l + 2 - i)) & 1) << l;
    const uint32_t N = 2u << (order - 1);
    uint32_t t = X[2] >> 1;
    for (int i = 2; i > 0; --i) X[i] ^= X[i - 1];
    X[0] ^= t;
    for (uint32_t Q = 2; Q != N; Q <<= 1) {
        const uint32_t P = Q - 1;
        for (int i = 2; i >= 0; --i) {
            if (X[i] & Q) {
                X[0] ^= P;
            } else {
                t = (X[0] ^ X[i]) & P;
                X[0] ^= t;
                X[i] ^= t;
            }
        }
    }
    for (int i = 0; i < 3; ++i) c[i] = (int32_t)X[i];
}

struct HilbertArgs {
    int32_t order;
    int64_t nseg, seg_begin, per_seg;
    double hv[3];        // voxel width per axis, L / 2^order
};

// positions of particles first .. first + n - 1 of the call (particle g of the
// call is particle g mod per_seg of segment seg_begin + g / per_seg)
__global__ void k_hilbert_positions(HilbertArgs a, int64_t first, int64_t n, const double *u,
                                    double *x)
{
    const int64_t V = (int64_t)1 << (3 * a.order);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t g = first + i;
        const int64_t s = a.seg_begin + g / a.per_seg, k = g % a.per_seg;
        const int64_t v0 = s * V / a.nseg, v1 = (s + 1) * V / a.nseg;
        const int64_t v = v0 + k * (v1 - v0) / a.per_seg;
        int32_t c[3];
        hilbert_voxel(a.order, v, c);
        for (int ax = 0; ax < 3; ++ax)
            x[3 * i + ax] = ((double)c[ax] + u[3 * i + ax]) * a.hv[ax];
    }
}

// ---------------------------------------------------------------------------
// bounding boxes: positions are non-negative, so their binary64 bit patterns
// order like the values and the extrema are integer atomics on the patterns
// ---------------------------------------------------------------------------
constexpr unsigned long long kPosInf = 0x7FF0000000000000ull;
constexpr unsigned long long kNegInf = 0xFFF0000000000000ull;

__global__ void k_bbox_init(unsigned long long *box, int64_t nparts)
{
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < 6 * nparts;
         t += (int64_t)gridDim.x * blockDim.x)
        box[t] = (t % 6) < 3 ? kPosInf : 0ull;
}

// an empty partition keeps min = +inf; its max becomes -inf
__global__ void k_bbox_finish(unsigned long long *box, int64_t nparts)
{
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < nparts;
         p += (int64_t)gridDim.x * blockDim.x)
        if (box[6 * p] == kPosInf)
            for (int a = 0; a < 3; ++a) box[6 * p + 3 + a] = kNegInf;
}

__device__ __forceinline__ double wave_min(double v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ double wave_max(double v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}

template <class T>
struct BoxArgs {
    View<T> V;
    const int32_t *items;
    const int32_t *nitems;
    Params p;
    int64_t id0, per_part, nparts;
    unsigned long long *box;
};

// One workgroup per work item.  When every particle of a wave that belongs
// to a partition belongs to the same one (the usual case while partitions are
// compact), the wave reduces first and one lane updates the box.
template <class T>
__global__ void __launch_bounds__(256) k_bbox(BoxArgs<T> a)
{
    const int64_t ni = *a.nitems;
    const Params &p = a.p;
    for (int64_t it = blockIdx.x; it < ni; it += gridDim.x) {
        const int64_t c = a.items[2 * it], seg = a.items[2 * it + 1];
        const int64_t cc[3] = {c % p.nc[0], (c / p.nc[0]) % p.nc[1],
                               c / ((int64_t)p.nc[0] * p.nc[1])};
        const int64_t s0 = a.V.base[c] + seg * kSeg;
        const int64_t s1 = min(s0 + (int64_t)kSeg, a.V.base[c] + (int64_t)a.V.cnt[c]);
        // every lane of the workgroup runs the same number of rounds
        for (int64_t q0 = s0; q0 < s1; q0 += blockDim.x) {
            const int64_t q = q0 + threadIdx.x;
            int64_t part = -1;
            double xg[3] = {0.0, 0.0, 0.0};
            // a hole has a -1 offset (binary32) or a negated diameter (binary64)
            if (q < s1 && a.V.ox[q] >= T(0) && a.V.d[q] > T(0)) {
                const int64_t id = a.V.id[q];
                if (id >= a.id0 && (id - a.id0) / a.per_part < a.nparts) {
                    part = (id - a.id0) / a.per_part;
                    const T o[3] = {a.V.ox[q], a.V.oy[q], a.V.oz[q]};
                    for (int ax = 0; ax < 3; ++ax)   // binary32 metres in the FP32-everywhere form
                        xg[ax] = p.global ? (double)o[ax]
                                          : ((double)(cc[ax] * p.E) + (double)o[ax]) * p.h[ax];
                }
            }
            const uint64_t has = __ballot(part >= 0);
            if (has == 0) continue;
            const int lead = __ffsll((unsigned long long)has) - 1;
            const int64_t p0 = __shfl(part, lead);
            if (__ballot(part >= 0 && part != p0) == 0) {
                double lo[3], hi[3];
                for (int ax = 0; ax < 3; ++ax) {
                    lo[ax] = wave_min(part >= 0 ? xg[ax] : INFINITY);
                    hi[ax] = wave_max(part >= 0 ? xg[ax] : 0.0);
                }
                if (__lane_id() == lead)
                    for (int ax = 0; ax < 3; ++ax) {
                        atomicMin(a.box + 6 * p0 + ax, (unsigned long long)__double_as_longlong(lo[ax]));
                        atomicMax(a.box + 6 * p0 + 3 + ax,
                                  (unsigned long long)__double_as_longlong(hi[ax]));
                    }
            } else if (part >= 0) {
                for (int ax = 0; ax < 3; ++ax) {
                    const unsigned long long b = (unsigned long long)__double_as_longlong(xg[ax]);
                    atomicMin(a.box + 6 * part + ax, b);
                    atomicMax(a.box + 6 * part + 3 + ax, b);
                }
            }
        }
    }
}

template <class T>
View<T> store_view(st_ctx *c)
{
    View<T> v;
    v.ox = (T *)c->store[0][0];
    v.oy = (T *)c->store[0][1];
    v.oz = (T *)c->store[0][2];
    v.vx = (T *)c->store[0][3];
    v.vy = (T *)c->store[0][4];
    v.vz = (T *)c->store[0][5];
    v.d = (T *)c->store[0][6];
    v.id = (int32_t *)c->store[0][7];
    v.base = c->base;
    v.room = c->room;
    v.cnt = c->cnt;
    v.ndead = c->ndead;
    return v;
}

inline int64_t blocks_for(int64_t n, int64_t cap = 8192)
{
    const int64_t b = (n + 255) / 256;
    return b < 1 ? 1 : (b > cap ? cap : b);
}

}  // namespace

hipError_t launch_hilbert_positions(int32_t order, int64_t nseg, int64_t seg_begin,
                                    int64_t per_seg, const double L[3], int64_t first, int64_t n,
                                    const double *u, double *x, hipStream_t s)
{
    HilbertArgs a;
    a.order = order;
    a.nseg = nseg;
    a.seg_begin = seg_begin;
    a.per_seg = per_seg;
    for (int ax = 0; ax < 3; ++ax) a.hv[ax] = L[ax] / (double)((int64_t)1 << order);
    hipLaunchKernelGGL(k_hilbert_positions, dim3(blocks_for(n)), dim3(256), 0, s, a, first, n, u,
                       x);
    return hipGetLastError();
}

hipError_t launch_bounding_boxes(st_ctx *c, int64_t id0, int64_t per_part, int64_t nparts,
                                 double *box, hipStream_t s)
{
    unsigned long long *b = (unsigned long long *)box;
    hipLaunchKernelGGL(k_bbox_init, dim3(blocks_for(6 * nparts)), dim3(256), 0, s, b, nparts);
    const int64_t gi = c->max_items < 65536 ? c->max_items : 65536;
    auto run = [&](auto t) {
        using T = decltype(t);
        BoxArgs<T> a{store_view<T>(c), c->items, c->flags + F_NITEMS, c->prm, id0, per_part,
                     nparts, b};
        hipLaunchKernelGGL((k_bbox<T>), dim3(gi), dim3(256), 0, s, a);
    };
    if (c->form == ST_FORM_FP64) run(double(0));
    else run(float(0));
    hipLaunchKernelGGL(k_bbox_finish, dim3(blocks_for(nparts)), dim3(256), 0, s, b, nparts);
    return hipGetLastError();
}

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t noalloc_scratch_init(int device)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return hipSuccess;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = static_cast<double *>(p);
    return hipSuccess;
}

hipError_t noalloc_scratch(int device, double **ptr)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    *ptr = g_scratch_ptr[device];
    return *ptr ? hipSuccess : hipErrorNotInitialized;
}

}  // namespace st
