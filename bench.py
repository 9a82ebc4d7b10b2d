"""Benchmark of the per-particle time step on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-fp64] [--no-plume256] [--no-tg128]
                [--no-hilbert] [--no-adjoint] [--no-cpu]

A step is one pass of the whole hot path (gather, integrate, deposit,
relocate and re-bin) over every particle of the workload.  The headline is
the largest single-GPU workload: 512^3 cells, 1.4e9 droplets (60 % in one
plume), FP32 chunk-local form, the fluid field rotated by 1 degree per step on
a second stream that runs one step ahead of the particles.  W coupled
warm-up steps, then K coupled steps timed with events on the stream the
kernels run on, bracketed by device synchronisations; the step kernel's own
duration comes from a pair of events attached to each of its launches in the
same timed steps.  Inputs are seeded synthetic data resident in HBM before
the timed region starts.

Printed as one JSON line: the whole-job particle-steps/s, the step kernel's
roofline (algorithmic bytes per launch over its average launch time) and the
whole step's (the same bytes over the whole step's time), and beside them:
the FP64 form on the same workload, the 256^3 precision-study workload in
both forms, the 128^3 workload, Hilbert-segment placement and partition
bounding boxes, forward+adjoint throughput (64^3, 1e6 droplets, checkpoints
every 20 steps), a plain streaming copy of 1 GiB with the particle state's
access pattern (the practical streaming ceiling beside the published HBM
peak), and the FP64 oracle timed on this host's cores on a bounded sample of
the headline workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
METRIC = ("particle-steps/s on 1 MI355X (fwd, fwd+adjoint) vs FP64 form; "
          "% of HBM roofline")


def algorithmic_bytes(form, particles, items, E=8):
    """Bytes the step kernel must move per launch: each particle's state read
    (position, velocity, diameter) and written (position, velocity), plus per
    work item the fluid tile with its one-cell halo and the read-modify-write
    of the chunk's source cells."""
    ts = 8 if form == "fp64" else 4
    acc = 4 if form == "fp32" else 8
    per_particle = 7 * ts + 6 * ts            # 52 B (binary32), 104 B (binary64)
    tile = 3 * (E + 2) ** 3 * ts              # 12000 B / 24000 B
    deposit = 2 * 3 * E ** 3 * acc            # 24576 B (binary64 accumulation)
    return particles * per_particle + items * (tile + deposit), per_particle, tile + deposit


def make_tracker(pkg, w, form, drag="stokes"):
    return pkg.Tracker(w.n, w.L, w.P, form=form, chunk_edge=w.chunk_edge, rho_f=w.rho_f,
                       mu_f=w.mu_f, g=w.g, rho_p=w.rho_p, parcel_weight=w.parcel_weight,
                       drag=drag)


def inject_host(t, w):
    for b in range(w.n_batches()):
        x, up, d = w.batch(b)
        t.inject(x, up, d)


def inject_device(t, w):
    for b in range(w.n_device_batches()):
        x, up, d = w.device_batch(b)
        t.inject(x, up, d)
        del x, up, d


def inject(t, w):
    if w.P > 50_000_000:
        inject_device(t, w)   # too many to draw on the host in time
    else:
        inject_host(t, w)


_FIELDS = {}


def host_field(w):
    """The workload's cell-centred field (binary64, host), drawn once."""
    if w.name not in _FIELDS:
        _FIELDS[w.name] = w.field()
    return _FIELDS[w.name]


def field_of(torch, np, w, form):
    U = host_field(w)
    return torch.from_numpy(U if form == "fp64" else U.astype(np.float32)).cuda()


KERNEL_SOURCE = os.path.join(ROOT, "paper_2603_26691_amd", "csrc", "st_device.hip")


def measured_traffic(workload, form):
    """HBM bytes per step-kernel launch from the committed rocprofv3 counter
    record (FETCH_SIZE and WRITE_SIZE, each scaled by what it reads for a
    plain 1 GiB streaming copy), or None when there is no record for this
    workload or the kernel source changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"k_step_{workload}_{form}_counters.txt")
    if not os.path.exists(path):
        return None
    rec = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            rec[k.strip()] = v.strip()
    digest = hashlib.sha256(open(KERNEL_SOURCE, "rb").read()).hexdigest()
    if rec.get("kernel_source_sha256") != digest:
        return None
    return float(rec["hbm_bytes_per_launch"])


def roofline(form, w, kernel_ms, launches, items, ms_per_step, drag="stokes"):
    """The step kernel's roofline (its algorithmic bytes per launch over its
    average launch duration) and the whole step's (the same bytes over the
    whole step's duration: every other launch of the step is overhead)."""
    bytes_launch, per_p, per_item = algorithmic_bytes(form, w.P, items, w.chunk_edge)
    avg_s = kernel_ms / max(launches, 1) / 1e3
    achieved = bytes_launch / avg_s / 1e9
    step_gbps = bytes_launch / (ms_per_step / 1e3) / 1e9
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": measured_traffic(w.name, form) if drag == "stokes" else None,
            "kernel": "k_step", "avg_kernel_ms": avg_s * 1e3, "bytes_per_launch": bytes_launch,
            "kernel_timing": "events attached to each step-kernel launch of the timed steps",
            "model": f"{per_p} B/particle + {per_item} B/work item, {items} items",
            "whole_step": {"achieved": step_gbps, "frac": step_gbps / HBM_PEAK_GBS,
                           "ms_per_step": ms_per_step}}


def stream_copy_gbps(torch, N, mib=1024, reps=20):
    """Bytes read + written per second by a plain streaming copy of `mib` MiB
    with the particle state's access pattern (st_stream_copy: one 16-byte
    non-temporal load and store per thread)."""
    import ctypes
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    copy = lambda: N.check(N.lib().st_stream_copy(ctypes.c_void_p(a.data_ptr()),  # noqa: E731
                                                  ctypes.c_void_p(b.data_ptr()), 4 * n, s),
                           None, "st_stream_copy")
    for _ in range(3):
        copy()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        copy()
    e1.record()
    torch.cuda.synchronize()
    assert torch.equal(a[:1024], b[:1024])
    gbps = 2 * 4 * n * reps / (e0.elapsed_time(e1) / 1e3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    return gbps


def time_steps(torch, t, U, dt, steps, warmup):
    """(ms for `steps` steps, summed step-kernel ms, launches); the kernel's
    own duration from events attached to its launches in the timed steps."""
    for _ in range(warmup):
        t.step(U, dt)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t.timing(True)
    e0.record()
    for _ in range(steps):
        t.step(U, dt)
    e1.record()
    torch.cuda.synchronize()
    kernel_ms, launches = t.timing(False)
    return e0.elapsed_time(e1), kernel_ms, launches


def leg_forward(pkg, torch, np, w, form, steps, warmup, drag="stokes"):
    t = make_tracker(pkg, w, form, drag)
    inject(t, w)
    U = field_of(torch, np, w, form)
    ms, kernel_ms, launches = time_steps(torch, t, U, w.dt, steps, warmup)
    st = t.stats()
    t.close()
    del U
    torch.cuda.empty_cache()
    out = {"workload": w.name, "particles": w.P, "form": form, "steps": steps,
           "value": w.P * steps / (ms / 1e3), "unit": "particle-steps/s",
           "ms_per_step": ms / steps,
           "roofline": roofline(form, w, kernel_ms, launches, st["items"], ms / steps, drag),
           "last_step_movers": st["movers"], "holes": st["holes"], "repacks": st["repacks"]}
    return out


def leg_coupled(pkg, torch, np, w, form, steps, warmup):
    """The coupled run: W warm-up steps, then K timed steps, the field of step k
    rotated by k degrees on the second stream while the particles step."""
    t0 = time.perf_counter()
    t = make_tracker(pkg, w, form)
    inject_device(t, w)
    U0 = field_of(torch, np, w, form)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    if warmup:
        t.run_coupled(U0, w.rotation(warmup), w.dt)
    t.timing(True)
    field_ms, step_ms, total_ms = t.run_coupled(U0, w.rotation(steps, first=warmup), w.dt)
    kernel_ms, launches = t.timing(False)
    st = t.stats()
    t.close()
    del U0
    torch.cuda.empty_cache()
    ms = total_ms / steps
    return {"workload": w.name, "particles": w.P, "form": form, "steps": steps,
            "value": w.P * steps / (total_ms / 1e3), "unit": "particle-steps/s",
            "ms_per_step": ms, "field_update_ms_per_step": field_ms / steps,
            "particle_step_ms_per_step": step_ms / steps,
            "overlap": "total vs field + particle stream time: "
                       f"{total_ms:.2f} ms vs {field_ms + step_ms:.2f} ms",
            "roofline": roofline(form, w, kernel_ms, launches, st["items"], ms),
            "last_step_movers": st["movers"], "holes": st["holes"], "repacks": st["repacks"],
            "setup_s": setup_s}


def leg_adjoint(pkg, torch, np, synth):
    """Forward with checkpoints every 20 steps plus the adjoint, 64^3, 1e6."""
    w = synth.get("adj64")
    U = field_of(torch, np, w, "fp32_local")
    # warm-up: a short taped run of a few particles and its adjoint, so that
    # first-launch costs stay out of the timed region
    tw = make_tracker(pkg, w, "fp32_local")
    x, up, d = w.batch(0)
    tw.inject(x[:4096], up[:4096], d[:4096])
    for _ in range(3):
        tw.step(U, w.dt, tape=2)
    tw.backward(2.0 * tw.sources())
    tw.close()
    # the loss's target: the source field of the same droplets with their
    # diameters scaled by 1.1 (input preparation, untimed)
    tt = make_tracker(pkg, w, "fp32_local")
    for b in range(w.n_batches()):
        x, up, d = w.batch(b)
        tt.inject(x, up, d * 1.1)
    for _ in range(w.nsteps):
        tt.step(U, w.dt)
    T = tt.sources()
    tt.close()

    def run(form, Uf, lam_given=None):
        t = make_tracker(pkg, w, form)
        inject_host(t, w)
        # the checkpoint buffers and the backward's workspace are allocated
        # with the tracker, before the timed region
        t.tape_reserve(20, w.nsteps)
        torch.cuda.synchronize()
        e0, e1, e2, e3 = (torch.cuda.Event(enable_timing=True) for _ in range(4))
        e0.record()
        for _ in range(w.nsteps):
            t.step(Uf, w.dt, tape=20)
        S = t.sources()
        e1.record()
        # the loss's derivative is the caller's (torch elementwise work,
        # outside the timed forward and adjoint)
        lam = (2.0 * (S - T)).contiguous()  # dL/dS of L = |S - T|^2
        if lam_given is not None:
            lam = lam_given
        e2.record()
        dU, dd = t.backward(lam)
        e3.record()
        torch.cuda.synchronize()
        t.close()
        return e0.elapsed_time(e1), e2.elapsed_time(e3), lam, dU, dd

    fwd_ms, bwd_ms, lam, dU, dd = run("fp32_local", U)
    # the same problem in the FP64 form (the field widened from binary32, the
    # same dL/dS), timed too, and how far the binary32 forward moves the
    # gradient
    fwd64, bwd64, _, dU64, dd64 = run("fp64", U.double(), lam)
    rel = {"dL_du": float((dU - dU64).norm() / dU64.norm()),
           "dL_dd": float((dd - dd64).norm() / dd64.norm())}
    value = w.P * w.nsteps / ((fwd_ms + bwd_ms) / 1e3)
    # byte model of forward + adjoint with recomputation, per particle-step:
    # forward 52; recompute 52 + 32 (the saved state, 28, and its anchor, 4);
    # reverse 28 (saved state) + 4 (anchor) + 56 (the seven binary32 adjoint
    # values, xbar, ubar and dbar, read and written)
    model_b = 224
    return {"workload": w.name, "particles": w.P, "steps": w.nsteps, "checkpoint_every": 20,
            "value": value, "unit": "particle-steps/s",
            "model_bytes_per_particle_step": model_b,
            "model_GBps": value * model_b / 1e9,
            "model_frac_of_peak": value * model_b / 1e9 / HBM_PEAK_GBS,
            "forward_ms": fwd_ms, "backward_ms": bwd_ms,
            "fp64_form": {"value": w.P * w.nsteps / ((fwd64 + bwd64) / 1e3),
                          "forward_ms": fwd64, "backward_ms": bwd64},
            "loss": "L2 misfit of the source field against that of diameters x 1.1",
            "grad_finite": bool(torch.isfinite(dU).all() and torch.isfinite(dd).all()),
            "grad_rel_l2_vs_fp64_form": rel}


def leg_hilbert(pkg, torch, np, w, reps=10):
    """Hilbert-segment placement and partition bounding boxes on the workload's
    particle count: the 2^k-per-axis voxel lattice of the mesh cut into 4096
    segments (one per chunk of the mesh), uniforms drawn on the device."""
    order = max(1, int(round(np.log2(w.n[0]))))
    nseg = 4096
    per_seg = w.P // nseg
    n = nseg * per_seg
    t = make_tracker(pkg, w, "fp32_local")
    gen = torch.Generator(device="cuda")
    gen.manual_seed(w.seed)
    u = torch.rand((n, 3), dtype=torch.float64, device="cuda", generator=gen)
    x = t.hilbert_positions(order, nseg, 0, nseg, per_seg, u)   # warm-up
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        x = t.hilbert_positions(order, nseg, 0, nseg, per_seg, u)
    e1.record()
    torch.cuda.synchronize()
    place_ms = e0.elapsed_time(e1) / reps
    up = torch.zeros((n, 3), dtype=torch.float64, device="cuda")
    d = torch.full((n,), 20e-6, dtype=torch.float64, device="cuda")
    t.inject_hilbert(order, nseg, 0, nseg, per_seg, u, up, d)
    del x, up, d, u
    U = field_of(torch, np, w, "fp32_local")
    t.step(U, w.dt)
    box = t.bounding_boxes(0, per_seg, nseg)                      # warm-up
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        box = t.bounding_boxes(0, per_seg, nseg)
    e1.record()
    torch.cuda.synchronize()
    box_ms = e0.elapsed_time(e1) / reps
    vol = (box[:, 3:] - box[:, :3]).prod(dim=1).mean().item() / float(np.prod(w.L))
    t.close()
    torch.cuda.empty_cache()
    return {"particles": n, "order": order, "segments": nseg,
            "placement_ms": place_ms, "placement_particles_per_s": n / (place_ms / 1e3),
            "placement_GBps": n * 48 / (place_ms / 1e3) / 1e9,
            "placement_bytes": "48 B/particle (uniforms in, positions out)",
            "bbox_ms": box_ms, "bbox_particles_per_s": n / (box_ms / 1e3),
            "bbox_GBps": n * 16 / (box_ms / 1e3) / 1e9,
            "bbox_bytes": "16 B/particle (offsets and id), after one step",
            "mean_box_volume_fraction": vol}


def cpu_baseline(w, np, steps=10, sample=24_000_000, single_sample=1_500_000):
    """The FP64 oracle on this host: its particle-parallel driver on all the
    host's cores (OMP_NUM_THREADS, else the cores, at most 16) over the first
    `sample` droplets of the workload for `steps` steps with the binary32
    field widened; and the serial oracle on one core over the first
    `single_sample` droplets."""
    from oracle.oracle import MeshParams, default_threads, load
    orc = load()
    U = host_field(w).astype(np.float32).astype(np.float64)
    mesh = MeshParams(**w.mesh_kwargs())
    x, up, d = w.particles(sample)
    threads = default_threads()
    out = None
    while threads >= 1:
        try:
            t0 = time.perf_counter()
            orc.run_par(mesh, U, x, up, d, w.dt, steps, threads=threads)
            sec = time.perf_counter() - t0
            out = {"value": sample * steps / sec, "unit": "particle-steps/s", "cores": threads,
                   "kind": "oracle",
                   "sample": f"first {sample} droplets of {w.name} (its recipe, drawn on the "
                             f"host), {steps} steps, FP64 C oracle split over {threads} threads "
                             "with per-thread source arrays"}
            break
        except MemoryError:
            threads //= 2
    t0 = time.perf_counter()
    orc.run(mesh, U, x[:single_sample], up[:single_sample], d[:single_sample], w.dt, steps)
    sec1 = time.perf_counter() - t0
    single = {"value": single_sample * steps / sec1, "cores": 1,
              "sample": f"first {single_sample} droplets, {steps} steps, serial oracle"}
    if out is None:
        out = dict(single, unit="particle-steps/s", kind="oracle")
    out["single_core"] = single
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64-form legs")
    ap.add_argument("--no-plume256", action="store_true", help="skip the 256^3 legs")
    ap.add_argument("--no-tg128", action="store_true", help="skip the 128^3 legs")
    ap.add_argument("--no-hilbert", action="store_true",
                    help="skip the Hilbert placement and bounding-box leg")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the forward+adjoint leg")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--only", default=None,
                    help="run one leg alone: plume512, plume256, plume256_fp64, tg128, "
                         "adjoint (for profiling)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run the streaming copy of MIB MiB three times (the reference "
                         "for scaling hardware byte counters) and exit")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE "
              f"{world}); the particle step is measured on one MI355X", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2603_26691_amd as pkg
    from paper_2603_26691_amd import _native as N
    from workloads import synth

    if args.copy_calibration:
        import ctypes
        n = args.copy_calibration * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        for _ in range(3):
            N.check(N.lib().st_stream_copy(ctypes.c_void_p(a.data_ptr()),
                                           ctypes.c_void_p(b.data_ptr()), 4 * n, s))
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "launches": 3}))
        return
    if args.only == "adjoint":
        print(json.dumps(leg_adjoint(pkg, torch, np, synth)), flush=True)
        return
    if args.only:
        name = args.only.replace("_fp64", "")
        form = "fp64" if args.only.endswith("_fp64") else "fp32_local"
        w = synth.get(name)
        if name == "plume512":
            r = leg_coupled(pkg, torch, np, w, form, args.steps, args.warmup)
        else:
            r = leg_forward(pkg, torch, np, w, form, args.steps, args.warmup)
        print(json.dumps(r), flush=True)
        return

    w = synth.get("plume512")
    head = leg_coupled(pkg, torch, np, w, "fp32_local", args.steps, args.warmup)
    out = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "mesh": list(w.n), "particles": w.P, "dt": w.dt,
                   "form": "fp32_local", "chunk_edge": w.chunk_edge, "drag": "stokes",
                   "source_accumulation": "f64", "plume_fraction": w.plume_fraction,
                   "coupling": "field rotated 1 degree per step on a second stream, one step "
                               "ahead of the particles",
                   "parallelism": "single GPU"},
        "roofline": head["roofline"],
        "coupled": {k: head[k] for k in ("field_update_ms_per_step", "particle_step_ms_per_step",
                                         "overlap", "last_step_movers", "holes", "repacks",
                                         "setup_s")},
    }
    out["stream_copy"] = {"GBps": stream_copy_gbps(torch, N),
                          "bytes": "1 GiB read + 1 GiB written, 16-byte non-temporal accesses"}
    out["stream_copy"]["frac_of_peak"] = out["stream_copy"]["GBps"] / HBM_PEAK_GBS
    out["roofline"]["frac_of_stream_copy"] = out["roofline"]["achieved"] / out["stream_copy"]["GBps"]
    if not args.no_fp64:
        # the FP64 form of the same run needs about 245 GB; where it does not
        # fit, the reason is reported instead
        try:
            r64 = leg_coupled(pkg, torch, np, w, "fp64", args.steps, args.warmup)
            out["fp64_form"] = {k: r64[k] for k in ("value", "ms_per_step", "roofline")}
            out["speedup_vs_fp64_form"] = out["value"] / r64["value"]
        except (N.STError, RuntimeError) as e:
            out["fp64_form"] = {"value": None, "reason": str(e)[:200]}
            torch.cuda.empty_cache()
    if not args.no_plume256:
        w256 = synth.get("plume256")
        out["plume256"] = leg_forward(pkg, torch, np, w256, "fp32_local", w256.nsteps, 2)
        if not args.no_fp64:
            r = leg_forward(pkg, torch, np, w256, "fp64", w256.nsteps, 2)
            out["plume256"]["fp64_form"] = {k: r[k] for k in ("value", "ms_per_step", "roofline")}
            out["plume256"]["speedup_vs_fp64_form"] = out["plume256"]["value"] / r["value"]
    if not args.no_tg128:
        w128 = synth.get("tg128")
        out["tg128"] = leg_forward(pkg, torch, np, w128, "fp32_local", 20, 3)
        if not args.no_fp64:
            r = leg_forward(pkg, torch, np, w128, "fp64", 20, 3)
            out["tg128"]["fp64_form"] = {k: r[k] for k in ("value", "ms_per_step", "roofline")}
        r = leg_forward(pkg, torch, np, w128, "fp32_local", 20, 3, "schiller_naumann")
        out["tg128"]["schiller_naumann"] = {k: r[k] for k in ("value", "ms_per_step", "roofline")}
        if not args.no_hilbert:
            out["hilbert"] = leg_hilbert(pkg, torch, np, w128)
    if not args.no_adjoint:
        out["fwd_adjoint"] = leg_adjoint(pkg, torch, np, synth)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w, np)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
