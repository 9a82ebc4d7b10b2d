// C ABI of the scaletrack library: argument validation, buffer ownership and
// the order of kernel launches.  Every entry point returns an st_status and
// catches everything; nothing throws or aborts across the boundary.
#include <hip/hip_runtime.h>

#include <math.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <string>
#include <vector>

#include "st_internal.h"

namespace {

constexpr double kPi = 3.14159265358979323846;

// message of the last failed st_create_mesh on this thread (no context yet)
thread_local std::string g_create_err;

st_status fail(st_ctx *c, st_status s, const std::string &msg)
{
    if (c) c->err = msg;
    return s;
}

st_status dev_fail(st_ctx *c, hipError_t e, const char *what)
{
    return fail(c, ST_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define ST_HIP(call)                                        \
    do {                                                    \
        hipError_t e_ = (call);                             \
        if (e_ != hipSuccess) return dev_fail(c, e_, #call); \
    } while (0)

template <class P>
hipError_t dalloc(P **p, size_t bytes, size_t &total)
{
    total += bytes;
    return hipMalloc((void **)p, bytes ? bytes : 8);
}

void free_all(st_ctx *c)
{
    for (int b = 0; b < 2; ++b)
        for (int k = 0; k < 8; ++k) (void)hipFree(c->store_raw[b][k]);
    for (int k = 0; k < 3; ++k) (void)hipFree(c->mov[k]);
    void *singles[] = {c->base, c->room, c->cnt, c->ndead, c->out_cnt, c->in_cnt, c->cursor,
                       c->new_cnt, c->nbase, c->nroom, c->hole, c->items, c->nseg,
                       c->scan_tmp, c->room_denom, c->flags, c->src, c->stage64, c->fieldbuf[0],
                       c->fieldbuf[1], c->ec_prev, c->ec_ext};
    for (void *p : singles) (void)hipFree(p);
    for (auto &sn : c->snaps) (void)hipFree(sn.buf);
    c->snaps.clear();
    for (auto &sn : c->spare) (void)hipFree(sn.buf);
    c->spare.clear();
    (void)hipFree(c->bwd_ws);
    c->bwd_ws = nullptr;
    c->bwd_ws_bytes = 0;
    for (hipEvent_t e : c->tev) (void)hipEventDestroy(e);
    c->tev.clear();
    if (c->side) (void)hipStreamDestroy(c->side);
}

st_status ensure_flushed(st_ctx *c, hipStream_t s)
{
    if (c->pending == 0) return ST_OK;
    ST_HIP(st::launch_flush_pending(c, s));
    c->count += c->pending;
    c->pending = 0;
    return ST_OK;
}

bool finite3(const double *v)
{
    return isfinite(v[0]) && isfinite(v[1]) && isfinite(v[2]);
}

}  // namespace

extern "C" {

st_status st_create_mesh(const st_mesh_desc *desc, int device, st_ctx **out)
{
    if (!desc || !out) return ST_ERR_INVALID;
    *out = nullptr;
    st_ctx *c = nullptr;
    try {
        c = new st_ctx();
    } catch (...) {
        return ST_ERR_OOM;
    }
    auto bad = [&](const std::string &m) {
        delete c;
        g_create_err = "st_create_mesh: " + m;
        return ST_ERR_INVALID;
    };
    const st_mesh_desc &d = *desc;
    const int E = d.chunk_edge;
    if (!(E == 2 || E == 4 || E == 8)) return bad("chunk_edge must be 2, 4 or 8");
    for (int a = 0; a < 3; ++a) {
        if (d.n[a] < E || d.n[a] % E != 0) return bad("n must be a positive multiple of chunk_edge");
        if (!(isfinite(d.L[a]) && d.L[a] > 0)) return bad("L must be finite and > 0");
        if (!isfinite(d.g[a])) return bad("g must be finite");
    }
    if (!(isfinite(d.mu_f) && d.mu_f > 0) || !(isfinite(d.rho_p) && d.rho_p > 0) ||
        !(isfinite(d.parcel_weight) && d.parcel_weight > 0) || !isfinite(d.rho_f))
        return bad("material constants must be finite and > 0");
    if (d.form < 0 || d.form > 2) return bad("unknown form");
    if (d.interp < 0 || d.interp > 1) return bad("unknown interpolation");
    if (d.drag < 0 || d.drag > 1) return bad("unknown drag law");
    if (d.reserved != 0) return bad("reserved must be 0");
    if (d.drag == ST_DRAG_SCHILLER_NAUMANN && !(d.rho_f >= 0))
        return bad("rho_f must be >= 0 for Schiller-Naumann drag");
    if (d.capacity < 1) return bad("capacity must be >= 1");
    const int64_t ncell = (int64_t)d.n[0] * d.n[1] * d.n[2];
    if (ncell > ((int64_t)1 << 34)) return bad("mesh too large");

    c->desc = d;
    c->device = device;
    c->form = d.form;
    c->tsize = d.form == ST_FORM_FP64 ? 8 : 4;
    c->asize = d.form == ST_FORM_FP32 ? 4 : 8;
    st::Params &p = c->prm;
    memset(&p, 0, sizeof p);
    p.E = E;
    p.interp = d.interp;
    p.drag = d.drag;
    for (int a = 0; a < 3; ++a) {
        p.n[a] = d.n[a];
        p.nc[a] = d.n[a] / E;
        p.L[a] = d.L[a];
        p.h[a] = d.L[a] / d.n[a];
        p.inv_h[a] = 1.0 / p.h[a];
        p.g[a] = d.g[a];
    }
    p.global = d.form == ST_FORM_FP32 ? 1 : 0;
    for (int a = 0; a < 3; ++a) {
        p.inv_hf[a] = (float)(d.n[a] / d.L[a]);
        p.Lf[a] = (float)d.L[a];
    }
    p.C = (int64_t)p.nc[0] * p.nc[1] * p.nc[2];
    p.inv_V = 1.0 / (p.h[0] * p.h[1] * p.h[2]);
    p.tau_coef = d.rho_p / (18.0 * d.mu_f);
    p.mass_coef = d.parcel_weight * d.rho_p * kPi / 6.0;
    p.re_coef = d.rho_f / d.mu_f;

    c->C = p.C;
    c->cap = d.capacity;
    // spare slots: a quarter of the capacity (at least kSlackMin per chunk),
    // plus what rounding every room up to kAlign can take
    c->slots = d.capacity + std::max<int64_t>(d.capacity / 4, (int64_t)st::kSlackMin * p.C) +
               (int64_t)st::kAlign * p.C;
    c->mcap = std::max<int64_t>(std::min<int64_t>(d.capacity, 1 << 16), d.capacity / 8);
    c->max_items = p.C + (d.capacity + st::kSeg - 1) / st::kSeg;
    if (c->slots >= ((int64_t)1 << 31) - 1 || c->max_items >= ((int64_t)1 << 30))
        return bad("capacity too large for 32-bit slot indices");

    auto dev_bad = [&](st_status st, const std::string &m) {
        free_all(c);
        delete c;
        g_create_err = "st_create_mesh: " + m;
        return st;
    };
    hipError_t e = hipSetDevice(device);
    if (e != hipSuccess) return dev_bad(ST_ERR_DEVICE, hipGetErrorString(e));
    size_t total = 0;
    const int64_t C = p.C;
    hipError_t ok = hipSuccess;
    auto A = [&](auto **ptr, size_t bytes) {
        if (ok == hipSuccess) ok = dalloc(ptr, bytes, total);
    };
    for (int b = 0; b < 2; ++b) {
        for (int k = 0; k < 8; ++k) {
            const size_t off = (size_t)(8 * b + k) * st::kStagger;
            A(&c->store_raw[b][k], (size_t)c->slots * (k < 7 ? c->tsize : 4) + off);
            if (c->store_raw[b][k]) c->store[b][k] = (char *)c->store_raw[b][k] + off;
        }
    }
    A(&c->base, (size_t)(C + 1) * 8);
    A(&c->room, (size_t)C * 4);
    A(&c->cnt, (size_t)C * 4);
    A(&c->ndead, (size_t)C * 4);
    A(&c->mov[0], (size_t)c->mcap * (c->tsize == 8 ? sizeof(st::MoverRec<double>)
                                                   : sizeof(st::MoverRec<float>)));
    A(&c->mov[1], (size_t)c->mcap * 4);
    A(&c->mov[2], (size_t)c->mcap * 4);
    A(&c->out_cnt, (size_t)C * 4);
    A(&c->in_cnt, (size_t)C * 4);
    A(&c->cursor, (size_t)C * 4);
    A(&c->new_cnt, (size_t)C * 4);
    A(&c->nbase, (size_t)(C + 1) * 8);
    A(&c->nroom, (size_t)C * 4);
    A(&c->hole, (size_t)c->slots * 4);
    A(&c->items, (size_t)c->max_items * 8);
    A(&c->nseg, (size_t)(C + 1) * 4);
    A(&c->scan_tmp, (size_t)(C / 1024 + 4) * 8);
    A(&c->room_denom, 8);
    A(&c->flags, (size_t)st::F_COUNT * 4);
    A(&c->src, (size_t)3 * ncell * c->asize);
    if (ok != hipSuccess)
        return dev_bad(ST_ERR_OOM, "device allocation failed after " + std::to_string(total) +
                                       " bytes");
    // this device's address of the fixed scratch of st_bounding_boxes_noalloc
    e = st::noalloc_scratch_init(device);
    if (e != hipSuccess) return dev_bad(ST_ERR_DEVICE, hipGetErrorString(e));
    hipStream_t s = nullptr;
    e = st::launch_init(c, s);
    if (e == hipSuccess) e = st::launch_zero_sources(c, s);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) return dev_bad(ST_ERR_DEVICE, hipGetErrorString(e));
    *out = c;
    return ST_OK;
}

st_status st_destroy(st_ctx *c)
{
    if (!c) return ST_ERR_INVALID;
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    free_all(c);
    delete c;
    return ST_OK;
}

const char *st_last_error(const st_ctx *c)
{
    if (!c) return g_create_err.c_str();
    return c->err.c_str();
}

st_status st_count(const st_ctx *c, int64_t *n)
{
    if (!c || !n) return ST_ERR_INVALID;
    *n = c->count + c->pending;
    return ST_OK;
}

st_status st_inject(st_ctx *c, int64_t n, const double *x, const double *up, const double *d,
                    int on_device, void *hip_stream)
{
    if (!c) return ST_ERR_INVALID;
    try {
        if (n < 0) return fail(c, ST_ERR_INVALID, "st_inject: n < 0");
        if (n == 0) return ST_OK;
        if (!x || !up || !d) return fail(c, ST_ERR_INVALID, "st_inject: null array");
        if (c->count + c->pending + n > c->cap)
            return fail(c, ST_ERR_CAPACITY, "st_inject: capacity exceeded");
        if (!c->tape.empty()) return fail(c, ST_ERR_STATE, "st_inject: a tape is recorded");
        if (!on_device) {
            for (int64_t i = 0; i < n; ++i)
                if (!finite3(x + 3 * i) || !finite3(up + 3 * i) || !isfinite(d[i]) || !(d[i] > 0))
                    return fail(c, ST_ERR_INVALID, "st_inject: non-finite value or d <= 0 at " +
                                                       std::to_string(i));
        }
        ST_HIP(hipSetDevice(c->device));
        hipStream_t s = (hipStream_t)hip_stream;
        if (on_device) {
            ST_HIP(st::launch_zero_i32(c->flags + st::F_BADINPUT, 1, s));
        }
        const int64_t stage_batch = std::min<int64_t>(c->mcap, 1 << 22);
        if (!on_device && !c->stage64) {
            size_t bytes = (size_t)stage_batch * 7 * 8;
            hipError_t e = hipMalloc((void **)&c->stage64, bytes);
            if (e != hipSuccess) return fail(c, ST_ERR_OOM, "st_inject: staging buffer");
        }
        const int64_t pend0 = c->pending, id0 = c->next_id, count0 = c->count;
        int64_t done = 0;
        while (done < n) {
            if (c->pending == c->mcap) {
                st_status r = ensure_flushed(c, s);
                if (r != ST_OK) return r;
            }
            int64_t k = std::min<int64_t>(n - done, c->mcap - c->pending);
            if (!on_device) k = std::min<int64_t>(k, stage_batch);
            const double *xs = x + 3 * done, *us = up + 3 * done, *ds = d + done;
            if (!on_device) {
                double *sx = c->stage64, *su = sx + 3 * stage_batch, *sd = su + 3 * stage_batch;
                ST_HIP(hipMemcpyAsync(sx, xs, (size_t)k * 24, hipMemcpyHostToDevice, s));
                ST_HIP(hipMemcpyAsync(su, us, (size_t)k * 24, hipMemcpyHostToDevice, s));
                ST_HIP(hipMemcpyAsync(sd, ds, (size_t)k * 8, hipMemcpyHostToDevice, s));
                xs = sx;
                us = su;
                ds = sd;
            }
            ST_HIP(st::launch_stage_inject(c, k, xs, us, ds, c->pending, s));
            if (!on_device) ST_HIP(hipStreamSynchronize(s));
            c->pending += k;
            c->next_id += k;
            done += k;
        }
        if (on_device) {
            int32_t badflag = 0;
            ST_HIP(hipMemcpyAsync(&badflag, c->flags + st::F_BADINPUT, 4, hipMemcpyDeviceToHost, s));
            ST_HIP(hipStreamSynchronize(s));
            if (badflag) {
                // only possible when no flush happened in between (n <= mcap);
                // otherwise the state already holds the batch
                if (c->count == count0) {
                    c->pending = pend0;
                    c->next_id = id0;
                    return fail(c, ST_ERR_INVALID, "st_inject: non-finite value or d <= 0");
                }
                return fail(c, ST_ERR_INVALID,
                            "st_inject: non-finite value or d <= 0 (partially injected)");
            }
        }
        return ST_OK;
    } catch (...) {
        return fail(c, ST_ERR_OOM, "st_inject: host allocation failed");
    }
}

st_status st_step(st_ctx *c, const void *u_cells, double dt, int32_t nsub, int32_t tape,
                  void *hip_stream)
{
    if (!c) return ST_ERR_INVALID;
    try {
        if (!u_cells) return fail(c, ST_ERR_INVALID, "st_step: null field");
        if (!(isfinite(dt) && dt > 0)) return fail(c, ST_ERR_INVALID, "st_step: dt must be finite and > 0");
        if (nsub < 1) return fail(c, ST_ERR_INVALID, "st_step: nsub must be >= 1");
        if (tape < 0) return fail(c, ST_ERR_INVALID, "st_step: tape must be >= 0");
        if (tape > 0 && c->form == ST_FORM_FP32)
            return fail(c, ST_ERR_INVALID,
                        "st_step: taped steps need the FP64 or FP32 chunk-local form");
        if (tape > 0 && c->tape.empty() && c->tape_every == 0) c->tape_every = tape;
        if (tape == 0 && !c->tape.empty())
            return fail(c, ST_ERR_STATE, "st_step: untaped step while a tape is recorded");
        ST_HIP(hipSetDevice(c->device));
        hipStream_t s = (hipStream_t)hip_stream;
        st_status r = ensure_flushed(c, s);
        if (r != ST_OK) return r;
        const double dts = dt / nsub;
        for (int32_t k = 0; k < nsub; ++k) {
            if (tape > 0) {
                if (c->tape.size() % (size_t)c->tape_every == 0) {
                    st::Snapshot sn;
                    if (!c->spare.empty()) {   // a buffer of a consumed tape
                        sn = c->spare.back();
                        c->spare.pop_back();
                    } else {
                        sn.bytes = st::snapshot_bytes(c);
                        hipError_t e = hipMalloc(&sn.buf, sn.bytes);
                        if (e != hipSuccess) return fail(c, ST_ERR_OOM, "st_step: checkpoint");
                    }
                    c->snaps.push_back(sn);
                    ST_HIP(st::launch_snapshot(c, sn.buf, 0, s));
                }
                c->tape.push_back(st::TapeStep{u_cells, dts});
            }
            ST_HIP(st::launch_step(c, u_cells, dts, 1, s));
        }
        return ST_OK;
    } catch (...) {
        return fail(c, ST_ERR_OOM, "st_step: host allocation failed");
    }
}

st_status st_get_sources(st_ctx *c, double *out, int32_t reset, int on_device, void *hip_stream)
{
    if (!c) return ST_ERR_INVALID;
    if (!out) return fail(c, ST_ERR_INVALID, "st_get_sources: null output");
    ST_HIP(hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)hip_stream;
    const size_t n = 3 * (size_t)c->prm.n[0] * c->prm.n[1] * c->prm.n[2];
    if (on_device) {
        ST_HIP(st::launch_get_sources(c, out, reset, s));
        return ST_OK;
    }
    double *tmp = nullptr;
    hipError_t e = hipMalloc((void **)&tmp, n * 8);
    if (e != hipSuccess) return fail(c, ST_ERR_OOM, "st_get_sources: temporary");
    e = st::launch_get_sources(c, tmp, reset, s);
    if (e == hipSuccess) e = hipMemcpyAsync(out, tmp, n * 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(tmp);
    if (e != hipSuccess) return dev_fail(c, e, "st_get_sources");
    return ST_OK;
}

st_status st_get_particles(st_ctx *c, double *x, double *up, double *d, int64_t *id,
                           int32_t *cell, int on_device, void *hip_stream)
{
    if (!c) return ST_ERR_INVALID;
    ST_HIP(hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)hip_stream;
    st_status r = ensure_flushed(c, s);
    if (r != ST_OK) return r;
    const size_t n = (size_t)c->count;
    if (on_device) {
        ST_HIP(st::launch_get_particles(c, x, up, d, id, cell, s));
        return ST_OK;
    }
    if (n == 0) return ST_OK;
    // one device temporary laid out as x, up, d, id, cell
    size_t bytes = n * (24 + 24 + 8 + 8 + 12);
    char *tmp = nullptr;
    hipError_t e = hipMalloc((void **)&tmp, bytes);
    if (e != hipSuccess) return fail(c, ST_ERR_OOM, "st_get_particles: temporary");
    double *tx = (double *)tmp, *tu = tx + 3 * n, *td = tu + 3 * n;
    int64_t *ti = (int64_t *)(td + n);
    int32_t *tc = (int32_t *)(ti + n);
    e = st::launch_get_particles(c, x ? tx : nullptr, up ? tu : nullptr, d ? td : nullptr,
                                 id ? ti : nullptr, cell ? tc : nullptr, s);
    if (e == hipSuccess && x) e = hipMemcpyAsync(x, tx, n * 24, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess && up) e = hipMemcpyAsync(up, tu, n * 24, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess && d) e = hipMemcpyAsync(d, td, n * 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess && id) e = hipMemcpyAsync(id, ti, n * 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess && cell) e = hipMemcpyAsync(cell, tc, n * 12, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(tmp);
    if (e != hipSuccess) return dev_fail(c, e, "st_get_particles");
    return ST_OK;
}

namespace {

// Drops the tape; its checkpoint buffers are kept for the next tape, or
// released with the backward workspace.
void tape_reset(st_ctx *c, bool keep_buffers)
{
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    for (auto &sn : c->snaps) {
        if (keep_buffers) c->spare.push_back(sn);
        else (void)hipFree(sn.buf);
    }
    c->snaps.clear();
    if (!keep_buffers) {
        for (auto &sn : c->spare) (void)hipFree(sn.buf);
        c->spare.clear();
        (void)hipFree(c->bwd_ws);
        c->bwd_ws = nullptr;
        c->bwd_ws_bytes = 0;
    }
    c->tape.clear();
    c->tape_every = 0;
}

}  // namespace

st_status st_tape_clear(st_ctx *c)
{
    if (!c) return ST_ERR_INVALID;
    tape_reset(c, false);
    return ST_OK;
}

st_status st_tape_reserve(st_ctx *c, int32_t tape, int64_t substeps)
{
    if (!c) return ST_ERR_INVALID;
    if (tape <= 0 || substeps < 0)
        return fail(c, ST_ERR_INVALID, "st_tape_reserve: tape must be > 0 and substeps >= 0");
    if (c->form == ST_FORM_FP32)
        return fail(c, ST_ERR_INVALID,
                    "st_tape_reserve: taped steps need the FP64 or FP32 chunk-local form");
    if (!c->tape.empty()) return fail(c, ST_ERR_STATE, "st_tape_reserve: a tape is recorded");
    try {
        ST_HIP(hipSetDevice(c->device));
        const int64_t need = (substeps + tape - 1) / tape;
        while ((int64_t)c->spare.size() < need) {
            st::Snapshot sn;
            sn.bytes = st::snapshot_bytes(c);
            if (hipMalloc(&sn.buf, sn.bytes) != hipSuccess)
                return fail(c, ST_ERR_OOM, "st_tape_reserve: checkpoint");
            c->spare.push_back(sn);
        }
        if (st::reserve_backward(c, tape) != hipSuccess)
            return fail(c, ST_ERR_OOM, "st_tape_reserve: backward workspace");
        return ST_OK;
    } catch (...) {
        return fail(c, ST_ERR_OOM, "st_tape_reserve: host allocation failed");
    }
}

st_status st_backward(st_ctx *c, const double *dL_dSint, double *dL_du, double *dL_dd,
                      void *hip_stream)
{
    if (!c) return ST_ERR_INVALID;
    if (!dL_dSint || !dL_du || (!dL_dd && c->count > 0))
        return fail(c, ST_ERR_INVALID, "st_backward: null pointer");
    if (c->tape.empty()) return fail(c, ST_ERR_STATE, "st_backward: nothing taped");
    ST_HIP(hipSetDevice(c->device));
    ST_HIP(st::launch_backward(c, dL_dSint, dL_du, dL_dd, (hipStream_t)hip_stream));
    tape_reset(c, true);
    return ST_OK;
}

st_status st_run_coupled(st_ctx *c, const void *u0, const double *cs, int32_t nsteps, double dt,
                         float *field_ms, float *step_ms, float *total_ms, void *hip_stream)
{
    if (!c) return ST_ERR_INVALID;
    if (!u0 || !cs) return fail(c, ST_ERR_INVALID, "st_run_coupled: null pointer");
    if (nsteps < 0) return fail(c, ST_ERR_INVALID, "st_run_coupled: nsteps < 0");
    if (!(isfinite(dt) && dt > 0)) return fail(c, ST_ERR_INVALID, "st_run_coupled: bad dt");
    if (!c->tape.empty()) return fail(c, ST_ERR_STATE, "st_run_coupled: a tape is recorded");
    for (int32_t k = 0; k < nsteps; ++k)
        if (!isfinite(cs[2 * k]) || !isfinite(cs[2 * k + 1]))
            return fail(c, ST_ERR_INVALID, "st_run_coupled: non-finite rotation");
    if (nsteps == 0) return ST_OK;
    ST_HIP(hipSetDevice(c->device));
    hipStream_t sa = (hipStream_t)hip_stream;
    st_status r = ensure_flushed(c, sa);
    if (r != ST_OK) return r;
    const size_t fbytes = 3 * (size_t)c->prm.n[0] * c->prm.n[1] * c->prm.n[2] * c->tsize;
    for (int b = 0; b < 2; ++b)
        if (!c->fieldbuf[b]) {
            hipError_t e = hipMalloc(&c->fieldbuf[b], fbytes);
            if (e != hipSuccess) return fail(c, ST_ERR_OOM, "st_run_coupled: field buffers");
        }
    if (!c->side) ST_HIP(hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking));
    hipStream_t sb = c->side;
    const bool timed = field_ms || step_ms || total_ms;
    // events: field k ready, step k done (its field buffer may be reused)
    std::vector<hipEvent_t> ev_field(nsteps), ev_step(nsteps);
    std::vector<hipEvent_t> tf0(nsteps), tf1(nsteps), ts0(nsteps), ts1(nsteps);
    hipEvent_t t_begin = nullptr, t_end = nullptr;
    auto cleanup = [&]() {
        for (auto *v : {&ev_field, &ev_step, &tf0, &tf1, &ts0, &ts1})
            for (hipEvent_t e : *v)
                if (e) (void)hipEventDestroy(e);
        if (t_begin) (void)hipEventDestroy(t_begin);
        if (t_end) (void)hipEventDestroy(t_end);
    };
    hipError_t e = hipSuccess;
    for (int32_t k = 0; k < nsteps && e == hipSuccess; ++k) {
        e = hipEventCreateWithFlags(&ev_field[k], hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&ev_step[k], hipEventDisableTiming);
        if (timed) {
            if (e == hipSuccess) e = hipEventCreate(&tf0[k]);
            if (e == hipSuccess) e = hipEventCreate(&tf1[k]);
            if (e == hipSuccess) e = hipEventCreate(&ts0[k]);
            if (e == hipSuccess) e = hipEventCreate(&ts1[k]);
        }
    }
    if (e == hipSuccess && timed) e = hipEventCreate(&t_begin);
    if (e == hipSuccess && timed) e = hipEventCreate(&t_end);
    // the side stream starts after everything already on the caller's stream
    hipEvent_t ev_start = nullptr;
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ev_start, hipEventDisableTiming);
    if (e == hipSuccess && timed) e = hipEventRecord(t_begin, sa);
    if (e == hipSuccess) e = hipEventRecord(ev_start, sa);
    if (e == hipSuccess) e = hipStreamWaitEvent(sb, ev_start, 0);
    // field 0 first
    for (int32_t k = 0; k <= nsteps && e == hipSuccess; ++k) {
        // stream B: build U^(k) ... lagging the particle stream by one step
        if (k < nsteps) {
            void *buf = c->fieldbuf[k & 1];
            if (k >= 2) e = hipStreamWaitEvent(sb, ev_step[k - 2], 0);  // buffer free again
            if (e == hipSuccess && timed) e = hipEventRecord(tf0[k], sb);
            if (e == hipSuccess) e = st::launch_rotate_field(c, u0, buf, cs[2 * k], cs[2 * k + 1], sb);
            if (e == hipSuccess && timed) e = hipEventRecord(tf1[k], sb);
            if (e == hipSuccess) e = hipEventRecord(ev_field[k], sb);
        }
        // stream A: step k-1 with U^(k-1) while U^(k) is being built
        if (k >= 1 && e == hipSuccess) {
            const int32_t j = k - 1;
            e = hipStreamWaitEvent(sa, ev_field[j], 0);
            if (e == hipSuccess && timed) e = hipEventRecord(ts0[j], sa);
            if (e == hipSuccess) e = st::launch_step(c, c->fieldbuf[j & 1], dt, 1, sa);
            if (e == hipSuccess && timed) e = hipEventRecord(ts1[j], sa);
            if (e == hipSuccess) e = hipEventRecord(ev_step[j], sa);
        }
    }
    // the caller's stream must not run ahead of the side stream
    if (e == hipSuccess) e = hipEventRecord(ev_start, sb);
    if (e == hipSuccess) e = hipStreamWaitEvent(sa, ev_start, 0);
    if (e == hipSuccess && timed) e = hipEventRecord(t_end, sa);
    if (e == hipSuccess && timed) e = hipEventSynchronize(t_end);
    if (e == hipSuccess && timed) {
        float fsum = 0, ssum = 0, ms = 0;
        for (int32_t k = 0; k < nsteps && e == hipSuccess; ++k) {
            e = hipEventElapsedTime(&ms, tf0[k], tf1[k]);
            fsum += ms;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, ts0[k], ts1[k]);
            ssum += ms;
        }
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, t_begin, t_end);
        if (field_ms) *field_ms = fsum;
        if (step_ms) *step_ms = ssum;
        if (total_ms) *total_ms = ms;
    }
    if (!timed && e == hipSuccess) e = hipStreamSynchronize(sa);
    if (ev_start) (void)hipEventDestroy(ev_start);
    cleanup();
    if (e != hipSuccess) return dev_fail(c, e, "st_run_coupled");
    return ST_OK;
}

st_status st_ec_reset(st_ctx *c, void *hip_stream)
{
    if (!c) return ST_ERR_INVALID;
    ST_HIP(hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)hip_stream;
    const int64_t n = 3 * (int64_t)c->prm.n[0] * c->prm.n[1] * c->prm.n[2];
    if (!c->ec_prev) {
        if (hipMalloc((void **)&c->ec_prev, (size_t)n * 8) != hipSuccess)
            return fail(c, ST_ERR_OOM, "st_ec_reset: history buffers");
        if (hipMalloc((void **)&c->ec_ext, (size_t)n * 8) != hipSuccess) {
            (void)hipFree(c->ec_prev);
            c->ec_prev = nullptr;
            return fail(c, ST_ERR_OOM, "st_ec_reset: history buffers");
        }
    }
    ST_HIP(st::launch_zero_f64(c->ec_prev, n, s));
    ST_HIP(st::launch_zero_f64(c->ec_ext, n, s));
    return ST_OK;
}

st_status st_ec_estimate(st_ctx *c, int32_t kind, const double *S_last, double *applied,
                         int on_device, void *hip_stream)
{
    if (!c) return ST_ERR_INVALID;
    if (!S_last || !applied) return fail(c, ST_ERR_INVALID, "st_ec_estimate: null array");
    if (kind < ST_EXTRAP_ZERO || kind > ST_EXTRAP_LINEAR)
        return fail(c, ST_ERR_INVALID, "st_ec_estimate: unknown extrapolator");
    if (!c->ec_prev) {
        st_status r = st_ec_reset(c, hip_stream);
        if (r != ST_OK) return r;
    }
    ST_HIP(hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)hip_stream;
    const size_t n = 3 * (size_t)c->prm.n[0] * c->prm.n[1] * c->prm.n[2];
    if (on_device) {
        ST_HIP(st::launch_ec(c, kind, S_last, applied, s));
        return ST_OK;
    }
    double *tmp = nullptr;
    if (hipMalloc((void **)&tmp, 2 * n * 8) != hipSuccess)
        return fail(c, ST_ERR_OOM, "st_ec_estimate: temporaries");
    hipError_t e = hipMemcpyAsync(tmp, S_last, n * 8, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = st::launch_ec(c, kind, tmp, tmp + n, s);
    if (e == hipSuccess) e = hipMemcpyAsync(applied, tmp + n, n * 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipStreamSynchronize(s);
    (void)hipFree(tmp);
    if (e != hipSuccess) return dev_fail(c, e, "st_ec_estimate");
    return ST_OK;
}

st_status st_stats(st_ctx *c, int64_t *last_movers, int64_t *repacks, int64_t *particles,
                   int64_t *slots, int64_t *items, int64_t *holes, void *hip_stream)
{
    if (!c) return ST_ERR_INVALID;
    ST_HIP(hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)hip_stream;
    int32_t f[st::F_COUNT];
    ST_HIP(hipMemcpyAsync(f, c->flags, sizeof f, hipMemcpyDeviceToHost, s));
    ST_HIP(hipStreamSynchronize(s));
    if (last_movers) *last_movers = f[st::F_LASTMOV];
    if (repacks) *repacks = f[st::F_REPACKS];
    if (particles) *particles = c->count + c->pending;
    if (slots) *slots = c->slots;
    if (items) *items = f[st::F_NITEMS];
    if (holes) *holes = f[st::F_DEAD];
    return ST_OK;
}

st_status st_stream_copy(const void *src, void *dst, int64_t bytes, void *hip_stream)
{
    if (!src || !dst || bytes < 0 || bytes % 16 != 0 || ((uintptr_t)src | (uintptr_t)dst) % 16)
        return ST_ERR_INVALID;
    if (bytes == 0) return ST_OK;
    return st::launch_stream_copy(src, dst, bytes, (hipStream_t)hip_stream) == hipSuccess
               ? ST_OK : ST_ERR_DEVICE;
}

st_status st_timing(st_ctx *c, int32_t enable, double *kernel_ms, int64_t *launches)
{
    if (!c) return ST_ERR_INVALID;
    ST_HIP(hipSetDevice(c->device));
    double sum = 0.0;
    for (size_t k = 0; k + 1 < c->tev.size(); k += 2) {
        ST_HIP(hipEventSynchronize(c->tev[k + 1]));
        float ms = 0.f;
        ST_HIP(hipEventElapsedTime(&ms, c->tev[k], c->tev[k + 1]));
        sum += ms;
    }
    if (kernel_ms) *kernel_ms = sum;
    if (launches) *launches = (int64_t)(c->tev.size() / 2);
    if (enable) {
        for (hipEvent_t e : c->tev) (void)hipEventDestroy(e);
        c->tev.clear();
    }
    c->timing = enable ? 1 : 0;
    return ST_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Hilbert-segment placement and partition bounding boxes
// ---------------------------------------------------------------------------
namespace {

const char *hilbert_args_error(int32_t order, int64_t nseg, int64_t seg_begin, int64_t seg_end,
                               int64_t per_seg)
{
    if (order < 1 || order > 10) return "order must be 1..10";
    if (nseg < 1 || nseg > ((int64_t)1 << (3 * order))) return "nseg must be 1..8^order";
    if (seg_begin < 0 || seg_end > nseg || seg_begin > seg_end)
        return "need 0 <= seg_begin <= seg_end <= nseg";
    if (per_seg < 1 || per_seg > ((int64_t)1 << 31)) return "per_seg must be 1..2^31";
    return nullptr;
}

}  // namespace

st_status st_hilbert_positions(st_ctx *c, int32_t order, int64_t nseg, int64_t seg_begin,
                               int64_t seg_end, int64_t per_seg, const double *u, double *x,
                               int on_device, void *hip_stream)
{
    if (!c) return ST_ERR_INVALID;
    try {
        if (const char *m = hilbert_args_error(order, nseg, seg_begin, seg_end, per_seg))
            return fail(c, ST_ERR_INVALID, std::string("st_hilbert_positions: ") + m);
        const int64_t n = (seg_end - seg_begin) * per_seg;
        if (n == 0) return ST_OK;
        if (!u || !x) return fail(c, ST_ERR_INVALID, "st_hilbert_positions: null array");
        ST_HIP(hipSetDevice(c->device));
        hipStream_t s = (hipStream_t)hip_stream;
        if (on_device) {
            ST_HIP(st::launch_hilbert_positions(order, nseg, seg_begin, per_seg, c->prm.L, 0, n,
                                                u, x, s));
            return ST_OK;
        }
        double *tmp = nullptr;
        if (hipMalloc((void **)&tmp, (size_t)n * 48) != hipSuccess)
            return fail(c, ST_ERR_OOM, "st_hilbert_positions: temporaries");
        hipError_t e = hipMemcpyAsync(tmp, u, (size_t)n * 24, hipMemcpyHostToDevice, s);
        if (e == hipSuccess)
            e = st::launch_hilbert_positions(order, nseg, seg_begin, per_seg, c->prm.L, 0, n, tmp,
                                             tmp + 3 * n, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(x, tmp + 3 * n, (size_t)n * 24, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        (void)hipStreamSynchronize(s);
        (void)hipFree(tmp);
        if (e != hipSuccess) return dev_fail(c, e, "st_hilbert_positions");
        return ST_OK;
    } catch (...) {
        return fail(c, ST_ERR_OOM, "st_hilbert_positions: host allocation failed");
    }
}

st_status st_inject_hilbert(st_ctx *c, int32_t order, int64_t nseg, int64_t seg_begin,
                            int64_t seg_end, int64_t per_seg, const double *u, const double *up,
                            const double *d, int on_device, void *hip_stream)
{
    if (!c) return ST_ERR_INVALID;
    try {
        if (const char *m = hilbert_args_error(order, nseg, seg_begin, seg_end, per_seg))
            return fail(c, ST_ERR_INVALID, std::string("st_inject_hilbert: ") + m);
        const int64_t n = (seg_end - seg_begin) * per_seg;
        if (n == 0) return ST_OK;
        if (!u || !up || !d) return fail(c, ST_ERR_INVALID, "st_inject_hilbert: null array");
        if (c->count + c->pending + n > c->cap)
            return fail(c, ST_ERR_CAPACITY, "st_inject_hilbert: capacity exceeded");
        if (!c->tape.empty()) return fail(c, ST_ERR_STATE, "st_inject_hilbert: a tape is recorded");
        if (!on_device) {
            for (int64_t i = 0; i < n; ++i) {
                for (int a = 0; a < 3; ++a)
                    if (!(u[3 * i + a] >= 0.0 && u[3 * i + a] < 1.0))
                        return fail(c, ST_ERR_INVALID,
                                    "st_inject_hilbert: u outside [0, 1) at " + std::to_string(i));
                if (!finite3(up + 3 * i) || !isfinite(d[i]) || !(d[i] > 0))
                    return fail(c, ST_ERR_INVALID, "st_inject_hilbert: non-finite value or d <= 0 at " +
                                                       std::to_string(i));
            }
        }
        ST_HIP(hipSetDevice(c->device));
        hipStream_t s = (hipStream_t)hip_stream;
        // positions (and, from the host, the other inputs) in device batches,
        // each injected as device arrays
        const int64_t batch = std::min<int64_t>(n, (int64_t)1 << 22);
        double *tmp = nullptr;
        const size_t per = on_device ? 24 : 24 + 24 + 24 + 8;
        if (hipMalloc((void **)&tmp, (size_t)batch * per) != hipSuccess)
            return fail(c, ST_ERR_OOM, "st_inject_hilbert: temporaries");
        st_status r = ST_OK;
        hipError_t e = hipSuccess;
        for (int64_t done = 0; done < n && r == ST_OK && e == hipSuccess; done += batch) {
            const int64_t k = std::min<int64_t>(batch, n - done);
            double *xs = tmp;
            const double *us = u + 3 * done, *vs = up + 3 * done, *ds = d + done;
            if (!on_device) {
                double *tu = tmp + 3 * batch, *tv = tu + 3 * batch, *td = tv + 3 * batch;
                e = hipMemcpyAsync(tu, us, (size_t)k * 24, hipMemcpyHostToDevice, s);
                if (e == hipSuccess) e = hipMemcpyAsync(tv, vs, (size_t)k * 24, hipMemcpyHostToDevice, s);
                if (e == hipSuccess) e = hipMemcpyAsync(td, ds, (size_t)k * 8, hipMemcpyHostToDevice, s);
                us = tu;
                vs = tv;
                ds = td;
            }
            if (e == hipSuccess)
                e = st::launch_hilbert_positions(order, nseg, seg_begin, per_seg, c->prm.L, done, k,
                                                 us, xs, s);
            if (e == hipSuccess) r = st_inject(c, k, xs, vs, ds, 1, hip_stream);
        }
        (void)hipStreamSynchronize(s);
        (void)hipFree(tmp);
        if (e != hipSuccess) return dev_fail(c, e, "st_inject_hilbert");
        return r;
    } catch (...) {
        return fail(c, ST_ERR_OOM, "st_inject_hilbert: host allocation failed");
    }
}

st_status st_bounding_boxes(st_ctx *c, int64_t id0, int64_t per_part, int64_t nparts,
                            double *boxes, int on_device, void *hip_stream)
{
    if (!c) return ST_ERR_INVALID;
    if (!boxes) return fail(c, ST_ERR_INVALID, "st_bounding_boxes: null array");
    if (id0 < 0 || per_part < 1 || nparts < 1)
        return fail(c, ST_ERR_INVALID, "st_bounding_boxes: need id0 >= 0, per_part >= 1, nparts >= 1");
    ST_HIP(hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)hip_stream;
    st_status r = ensure_flushed(c, s);
    if (r != ST_OK) return r;
    if (on_device) {
        ST_HIP(st::launch_bounding_boxes(c, id0, per_part, nparts, boxes, s));
        return ST_OK;
    }
    double *tmp = nullptr;
    if (hipMalloc((void **)&tmp, (size_t)nparts * 48) != hipSuccess)
        return fail(c, ST_ERR_OOM, "st_bounding_boxes: temporaries");
    hipError_t e = st::launch_bounding_boxes(c, id0, per_part, nparts, tmp, s);
    if (e == hipSuccess) e = hipMemcpyAsync(boxes, tmp, (size_t)nparts * 48, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipStreamSynchronize(s);
    (void)hipFree(tmp);
    if (e != hipSuccess) return dev_fail(c, e, "st_bounding_boxes");
    return ST_OK;
}

st_status st_bounding_boxes_noalloc(st_ctx *c, int64_t id0, int64_t per_part, int64_t nparts,
                                    double *boxes, int32_t on_device, void *hip_stream)
{
    if (!c) return ST_ERR_INVALID;
    if (!boxes) return fail(c, ST_ERR_INVALID, "st_bounding_boxes_noalloc: null array");
    if (id0 < 0 || per_part < 1 || nparts < 1)
        return fail(c, ST_ERR_INVALID,
                    "st_bounding_boxes_noalloc: need id0 >= 0, per_part >= 1, nparts >= 1");
    if (nparts > st::kNoAllocMaxParts)
        return fail(c, ST_ERR_INVALID, "st_bounding_boxes_noalloc: nparts " +
                                           std::to_string(nparts) + " exceeds the maximum " +
                                           std::to_string(st::kNoAllocMaxParts));
    ST_HIP(hipSetDevice(c->device));
    double *sc = nullptr;
    ST_HIP(st::noalloc_scratch(c->device, &sc));
    hipStream_t s = (hipStream_t)hip_stream;
    st_status r = ensure_flushed(c, s);
    if (r != ST_OK) return r;
    ST_HIP(st::launch_bounding_boxes(c, id0, per_part, nparts, sc, s));
    ST_HIP(hipMemcpyAsync(boxes, sc, (size_t)nparts * 48,
                          on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s));
    if (!on_device) ST_HIP(hipStreamSynchronize(s));
    return ST_OK;
}
