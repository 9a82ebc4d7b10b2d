"""Python face of the scaletrack library: a particle tracker on one GPU.

Every call marshals torch tensors (device memory) or numpy arrays (host
memory) into the C ABI of include/st.h; all of the method runs in the HIP
kernels behind it.  Work is ordered on torch's current stream.
"""
import ctypes

import numpy as np
import torch

from . import _native as N


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dptr(t):
    return ctypes.c_void_p(t.data_ptr())


class Tracker:
    """Particles on a uniform periodic mesh (see include/st.h).

    n: cells per axis (multiples of chunk_edge); L: domain extent [m];
    form: "fp64", "fp32_local" or "fp32"; interp: "trilinear" or "ngp";
    drag: "stokes" or "schiller_naumann"; capacity: maximum number of particles.
    """

    def __init__(self, n, L, capacity, form="fp32_local", interp="trilinear", chunk_edge=8,
                 rho_f=1.2, mu_f=1.8e-5, g=(0.0, 0.0, -9.81), rho_p=1000.0,
                 parcel_weight=1.0, drag="stokes", device=0):
        d = N.MeshDesc()
        d.n[:] = [int(v) for v in n]
        d.chunk_edge = int(chunk_edge)
        d.L[:] = [float(v) for v in L]
        d.rho_f = float(rho_f)
        d.mu_f = float(mu_f)
        d.g[:] = [float(v) for v in g]
        d.rho_p = float(rho_p)
        d.parcel_weight = float(parcel_weight)
        d.form = N.FORMS[form] if isinstance(form, str) else int(form)
        d.interp = N.INTERPS[interp] if isinstance(interp, str) else int(interp)
        d.drag = N.DRAGS[drag] if isinstance(drag, str) else int(drag)
        d.capacity = int(capacity)
        self.desc = d
        self.form = form
        self.n = tuple(int(v) for v in n)
        self.L = tuple(float(v) for v in L)
        self.device = torch.device("cuda", device)
        self._taped = []   # fields borrowed by taped steps
        ctx = ctypes.c_void_p()
        st = N.lib().st_create_mesh(ctypes.byref(d), int(device), ctypes.byref(ctx))
        if st != N.ST_OK:
            raise N.STError(st, "st_create_mesh failed")
        self.ctx = ctx

    # ------------------------------------------------------------------
    @property
    def field_dtype(self):
        return torch.float64 if self.desc.form == 0 else torch.float32

    @property
    def field_shape(self):
        return (3, self.n[2], self.n[1], self.n[0])

    def close(self):
        if getattr(self, "ctx", None):
            N.lib().st_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # ------------------------------------------------------------------
    def inject(self, x, up, d):
        """Adds particles; torch tensors on the device or numpy arrays (float64)."""
        if isinstance(x, torch.Tensor):
            x = x.to(self.device, torch.float64).contiguous()
            up = up.to(self.device, torch.float64).contiguous()
            d = d.to(self.device, torch.float64).contiguous()
            n = d.numel()
            assert x.numel() == 3 * n and up.numel() == 3 * n
            N.check(N.lib().st_inject(self.ctx, n, _dptr(x), _dptr(up), _dptr(d), 1, _stream()),
                    self.ctx)
        else:
            x = np.ascontiguousarray(x, dtype=np.float64)
            up = np.ascontiguousarray(up, dtype=np.float64)
            d = np.ascontiguousarray(d, dtype=np.float64)
            n = d.size
            assert x.size == 3 * n and up.size == 3 * n
            P = ctypes.c_void_p
            N.check(N.lib().st_inject(self.ctx, n, P(x.ctypes.data), P(up.ctypes.data),
                                      P(d.ctypes.data), 0, _stream()), self.ctx)

    def hilbert_positions(self, order, nseg, seg_begin, seg_end, per_seg, u):
        """Positions [n, 3] float64 of segments [seg_begin, seg_end) placed along
        the Hilbert curve (include/st.h); u [n, 3] uniforms, torch (device) or numpy."""
        # the library validates the arguments; the arrays only need to match
        n = max((seg_end - seg_begin) * per_seg, 0)
        if isinstance(u, torch.Tensor):
            u = u.to(self.device, torch.float64).contiguous()
            assert u.numel() == 3 * n
            x = torch.empty((n, 3), dtype=torch.float64, device=self.device)
            N.check(N.lib().st_hilbert_positions(self.ctx, int(order), int(nseg), int(seg_begin),
                                                 int(seg_end), int(per_seg), _dptr(u), _dptr(x), 1,
                                                 _stream()), self.ctx)
            return x
        u = np.ascontiguousarray(u, dtype=np.float64)
        assert u.size == 3 * n
        x = np.empty((n, 3))
        P = ctypes.c_void_p
        N.check(N.lib().st_hilbert_positions(self.ctx, int(order), int(nseg), int(seg_begin),
                                             int(seg_end), int(per_seg), P(u.ctypes.data),
                                             P(x.ctypes.data), 0, _stream()), self.ctx)
        return x

    def inject_hilbert(self, order, nseg, seg_begin, seg_end, per_seg, u, up, d):
        """Adds the particles of segments [seg_begin, seg_end) placed along the
        Hilbert curve; torch tensors on the device or numpy arrays."""
        args = (int(order), int(nseg), int(seg_begin), int(seg_end), int(per_seg))
        n = max((seg_end - seg_begin) * per_seg, 0)
        if isinstance(u, torch.Tensor):
            u, up, d = (t.to(self.device, torch.float64).contiguous() for t in (u, up, d))
            assert u.numel() == 3 * n and up.numel() == 3 * n and d.numel() == n
            N.check(N.lib().st_inject_hilbert(self.ctx, *args, _dptr(u), _dptr(up), _dptr(d), 1,
                                              _stream()), self.ctx)
        else:
            u, up, d = (np.ascontiguousarray(a, dtype=np.float64) for a in (u, up, d))
            assert u.size == 3 * n and up.size == 3 * n and d.size == n
            P = ctypes.c_void_p
            N.check(N.lib().st_inject_hilbert(self.ctx, *args, P(u.ctypes.data), P(up.ctypes.data),
                                              P(d.ctypes.data), 0, _stream()), self.ctx)

    def bounding_boxes(self, id0, per_part, nparts):
        """[nparts, 6] float64 on the device: (min xyz, max xyz) of the particles
        with id in [id0 + p per_part, id0 + (p+1) per_part)."""
        out = torch.empty((nparts, 6), dtype=torch.float64, device=self.device)
        N.check(N.lib().st_bounding_boxes(self.ctx, int(id0), int(per_part), int(nparts),
                                          _dptr(out), 1, _stream()), self.ctx)
        return out

    def bounding_boxes_noalloc(self, id0, per_part, nparts, out=None):
        """The boxes of bounding_boxes() from the library's allocation-free
        entry point (at most NOALLOC_MAX_PARTS partitions): into `out`, a
        float64 [nparts, 6] device tensor or host numpy array, made on the
        device when None."""
        if out is None:
            out = torch.empty((nparts, 6), dtype=torch.float64, device=self.device)
        if isinstance(out, torch.Tensor):
            assert out.is_cuda and out.dtype == torch.float64 and out.is_contiguous()
            assert out.numel() >= 6 * nparts
            ptr, on_device = _dptr(out), 1
        else:
            assert out.dtype == np.float64 and out.flags.c_contiguous and out.size >= 6 * nparts
            ptr, on_device = ctypes.c_void_p(out.ctypes.data), 0
        N.check(N.lib().st_bounding_boxes_noalloc(self.ctx, int(id0), int(per_part), int(nparts),
                                                  ptr, on_device, _stream()), self.ctx)
        return out

    def count(self):
        v = ctypes.c_int64()
        N.check(N.lib().st_count(self.ctx, ctypes.byref(v)), self.ctx)
        return v.value

    def step(self, u, dt, nsub=1, tape=0):
        """One step of dt with the device field u [3, nz, ny, nx].  A taped
        step borrows u until backward() or tape_clear(); the tracker holds a
        reference to it until then."""
        assert u.is_cuda and u.dtype == self.field_dtype and u.is_contiguous()
        assert tuple(u.shape) == self.field_shape
        N.check(N.lib().st_step(self.ctx, _dptr(u), float(dt), int(nsub), int(tape), _stream()),
                self.ctx)
        if tape:
            self._taped.append(u)

    def sources(self, reset=False):
        """Time-integrated momentum source, float64 [3, nz, ny, nx] on the device."""
        out = torch.empty(self.field_shape, dtype=torch.float64, device=self.device)
        N.check(N.lib().st_get_sources(self.ctx, _dptr(out), int(bool(reset)), 1, _stream()),
                self.ctx)
        return out

    def particles(self):
        """State by id: dict of x [P,3], up [P,3], d [P] (float64), id [P] int64, cell [P,3] int32."""
        P = self.count()
        dev = self.device
        out = {
            "x": torch.empty((P, 3), dtype=torch.float64, device=dev),
            "up": torch.empty((P, 3), dtype=torch.float64, device=dev),
            "d": torch.empty((P,), dtype=torch.float64, device=dev),
            "id": torch.full((P,), -1, dtype=torch.int64, device=dev),
            "cell": torch.empty((P, 3), dtype=torch.int32, device=dev),
        }
        N.check(N.lib().st_get_particles(self.ctx, _dptr(out["x"]), _dptr(out["up"]),
                                         _dptr(out["d"]), _dptr(out["id"]), _dptr(out["cell"]),
                                         1, _stream()), self.ctx)
        return out

    def backward(self, dL_dS):
        """(dL/du [3, nz, ny, nx], dL/dd [P]) float64 for dL/dSu_int = dL_dS."""
        lam = dL_dS.to(self.device, torch.float64).contiguous()
        dU = torch.zeros(self.field_shape, dtype=torch.float64, device=self.device)
        dd = torch.zeros((self.count(),), dtype=torch.float64, device=self.device)
        N.check(N.lib().st_backward(self.ctx, _dptr(lam), _dptr(dU), _dptr(dd), _stream()),
                self.ctx)
        self._taped = []
        return dU, dd

    def tape_clear(self):
        N.check(N.lib().st_tape_clear(self.ctx), self.ctx)
        self._taped = []

    def tape_reserve(self, tape, substeps):
        """Allocate the buffers of a taped run of `substeps` sub-steps (checkpoint
        every `tape`) and of its backward ahead of the run."""
        N.check(N.lib().st_tape_reserve(self.ctx, int(tape), int(substeps)), self.ctx)

    def run_coupled(self, u0, cs, dt, timed=True):
        """Coupled run with the rotating field; returns (field_ms, step_ms, total_ms)."""
        assert u0.is_cuda and u0.dtype == self.field_dtype and tuple(u0.shape) == self.field_shape
        cs = np.ascontiguousarray(cs, dtype=np.float64)
        nsteps = cs.size // 2
        f, s, t = ctypes.c_float(), ctypes.c_float(), ctypes.c_float()
        args = (ctypes.byref(f), ctypes.byref(s), ctypes.byref(t)) if timed else (None, None, None)
        N.check(N.lib().st_run_coupled(self.ctx, _dptr(u0), ctypes.c_void_p(cs.ctypes.data),
                                       nsteps, float(dt), *args, _stream()), self.ctx)
        return (f.value, s.value, t.value) if timed else None

    def ec_estimate(self, kind, S_last):
        """Source to apply at the current step from the previous step's actual
        source (extrapolator-corrector, kind "zero", "const" or "linear")."""
        k = N.EXTRAPOLATORS[kind] if isinstance(kind, str) else int(kind)
        S_last = S_last.to(self.device, torch.float64).contiguous()
        assert tuple(S_last.shape) == self.field_shape
        out = torch.empty_like(S_last)
        N.check(N.lib().st_ec_estimate(self.ctx, k, _dptr(S_last), _dptr(out), 1, _stream()),
                self.ctx)
        return out

    def ec_reset(self):
        N.check(N.lib().st_ec_reset(self.ctx, _stream()), self.ctx)

    def stats(self):
        m, r, p, s, i, h = (ctypes.c_int64() for _ in range(6))
        N.check(N.lib().st_stats(self.ctx, ctypes.byref(m), ctypes.byref(r), ctypes.byref(p),
                                 ctypes.byref(s), ctypes.byref(i), ctypes.byref(h), _stream()),
                self.ctx)
        return {"movers": m.value, "repacks": r.value, "particles": p.value, "slots": s.value,
                "items": i.value, "holes": h.value}

    def timing(self, enable):
        """Starts (True) or stops (False) timing the step kernel; returns
        (summed ms, launches) measured so far."""
        ms, n = ctypes.c_double(), ctypes.c_int64()
        N.check(N.lib().st_timing(self.ctx, int(bool(enable)), ctypes.byref(ms), ctypes.byref(n)),
                self.ctx)
        return ms.value, n.value
