"""Benchmark of the per-particle time step on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload tg128] [--form fp32_local]
                [--drag stokes] [--no-fp64] [--no-sn] [--no-hilbert] [--no-adjoint] [--no-scale]
                [--no-cpu]

A step is one pass of the whole hot path (gather, integrate, deposit,
relocate and re-bin) over every particle of the workload.  Inputs are
seeded synthetic data resident in HBM before the timed region starts; K
steps are timed with events on the stream the kernels run on, bracketed by
device synchronisations, and a second pass of K steps times the step kernel
itself with events attached to each of its launches.  Prints one JSON line with the whole-job
particle-steps/s, the step kernel's roofline figures, and beside them: the
FP64 form on the same workload, the same run with Schiller-Naumann drag,
Hilbert-segment placement and partition bounding boxes, forward+adjoint
throughput (64^3, 1e6 particles, checkpoints every 20 steps), the
1.4e9-particle 512^3 run with
the field update on a second stream, and the FP64 oracle timed on this
host's cores on a bounded sample of the workload.  Next to the published
HBM peak, the rate of a plain 1 GiB device copy is measured in the same run
as the practical streaming ceiling.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published


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


def field_of(torch, np, w, form):
    U = w.field()
    return torch.from_numpy(U if form == "fp64" else U.astype(np.float32)).cuda()


KERNEL_SOURCE = os.path.join(ROOT, "paper_2603_26691_amd", "csrc", "st_device.hip")


def measured_traffic(workload, form):
    """HBM bytes per step-kernel launch from the committed rocprofv3 counter
    record (FETCH_SIZE and WRITE_SIZE, each scaled by what it reads for a
    plain 1 GiB device copy), or None when there is no record for this
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


def roofline(form, w, kernel_ms, launches, items, drag="stokes"):
    bytes_launch, per_p, per_item = algorithmic_bytes(form, w.P, items, w.chunk_edge)
    avg_s = kernel_ms / max(launches, 1) / 1e3
    achieved = bytes_launch / avg_s / 1e9
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(w.name, form) if drag == "stokes" else None,
            "kernel": "k_step", "avg_kernel_ms": avg_s * 1e3, "bytes_per_launch": bytes_launch,
            "kernel_timing": "events attached to each step-kernel launch",
            "model": f"{per_p} B/particle + {per_item} B/work item, {items} items"}


def device_copy_gbps(torch, mib=1024, reps=20):
    """Bytes read + written per second by a plain device-to-device copy of
    `mib` MiB (torch's copy kernel): what streaming HBM traffic reaches in
    practice, beside the published peak."""
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    gbps = 2 * 4 * n * reps / (e0.elapsed_time(e1) / 1e3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    return gbps


def time_steps(torch, t, U, dt, steps, warmup):
    """(ms for `steps` steps, summed step-kernel ms, launches).  The steps are
    timed without per-launch instrumentation; the step kernel's own duration
    comes from a second pass of `steps` steps with a pair of events attached to
    each of its launches (recording them adds about 10 us per step)."""
    for _ in range(warmup):
        t.step(U, dt)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        t.step(U, dt)
    e1.record()
    torch.cuda.synchronize()
    t.timing(True)
    for _ in range(steps):
        t.step(U, dt)
    torch.cuda.synchronize()
    kernel_ms, launches = t.timing(False)
    return e0.elapsed_time(e1), kernel_ms, launches


def leg_forward(pkg, torch, np, w, form, steps, warmup, drag="stokes"):
    t = make_tracker(pkg, w, form, drag)
    if w.P > 50_000_000:
        inject_device(t, w)   # too many to draw on the host in time
    else:
        inject_host(t, w)
    U = field_of(torch, np, w, form)
    ms, kernel_ms, launches = time_steps(torch, t, U, w.dt, steps, warmup)
    st = t.stats()
    t.close()
    del U
    torch.cuda.empty_cache()
    return {"ms": ms, "kernel_ms": kernel_ms, "launches": launches, "stats": st}


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
    t = make_tracker(pkg, w, "fp32_local")
    inject_host(t, w)
    torch.cuda.synchronize()
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    e0.record()
    for _ in range(w.nsteps):
        t.step(U, w.dt, tape=20)
    S = t.sources()
    e1.record()
    lam = (2.0 * (S - T)).contiguous()  # dL/dS of L = |S - T|^2
    dU, dd = t.backward(lam)
    e2.record()
    torch.cuda.synchronize()
    fwd_ms, bwd_ms = e0.elapsed_time(e1), e1.elapsed_time(e2)
    t.close()
    # the same problem in the FP64 form (the field widened from binary32, the
    # same dL/dS), untimed: how far the binary32 forward moves the gradient
    t64 = make_tracker(pkg, w, "fp64")
    inject_host(t64, w)
    U64 = U.double()
    for _ in range(w.nsteps):
        t64.step(U64, w.dt, tape=20)
    dU64, dd64 = t64.backward(lam)
    t64.close()
    rel = {"dL_du": float((dU - dU64).norm() / dU64.norm()),
           "dL_dd": float((dd - dd64).norm() / dd64.norm())}
    value = w.P * w.nsteps / ((fwd_ms + bwd_ms) / 1e3)
    # byte model of forward + adjoint with recomputation, per particle-step:
    # forward 52, recompute with the saved state 52 + 24, reverse 28 (saved
    # state) + 48 (position and velocity adjoints) + 8 (diameter adjoint) + 4
    model_b = 216
    return {"workload": w.name, "particles": w.P, "steps": w.nsteps, "checkpoint_every": 20,
            "value": value, "unit": "particle-steps/s",
            "model_bytes_per_particle_step": model_b,
            "model_GBps": value * model_b / 1e9,
            "model_frac_of_peak": value * model_b / 1e9 / HBM_PEAK_GBS,
            "forward_ms": fwd_ms, "backward_ms": bwd_ms,
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


def leg_scale(pkg, torch, np, synth):
    """512^3, 1.4e9 particles (60 % in one plume), field rotated 1 degree per
    step on the second stream: throughput, overlap and the step kernel's
    roofline at full size."""
    w = synth.get("plume512")
    t0 = time.perf_counter()
    t = make_tracker(pkg, w, "fp32_local")
    inject_device(t, w)
    U0 = field_of(torch, np, w, "fp32_local")
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    cs = w.rotation()
    t.run_coupled(U0, w.rotation(2), w.dt)  # warm-up: two steps
    t.timing(True)
    field_ms, step_ms, total_ms = t.run_coupled(U0, cs, w.dt)
    kernel_ms, launches = t.timing(False)
    st = t.stats()
    t.close()
    del U0
    torch.cuda.empty_cache()
    return {"workload": w.name, "particles": w.P, "steps": w.nsteps, "form": "fp32_local",
            "value": w.P * w.nsteps / (total_ms / 1e3), "unit": "particle-steps/s",
            "ms_per_step": total_ms / w.nsteps, "field_update_ms_per_step": field_ms / w.nsteps,
            "particle_step_ms_per_step": step_ms / w.nsteps,
            "overlap": "total vs field + particle stream time: "
                       f"{total_ms:.2f} ms vs {field_ms + step_ms:.2f} ms",
            "roofline": roofline("fp32_local", w, kernel_ms, launches, st["items"]),
            "last_step_movers": st["movers"], "setup_s": setup_s}


def cpu_baseline(w, np, steps=4, max_particles=4_000_000):
    from oracle.oracle import MeshParams, load
    orc = load()
    k = min(w.P, max_particles)
    x, up, d = w.particles(k)
    # the oracle gets the field the binary32 forms use, promoted
    U = w.field().astype(np.float32).astype(np.float64)
    mesh = MeshParams(**w.mesh_kwargs())
    t0 = time.perf_counter()
    orc.run(mesh, U, x, up, d, w.dt, steps)
    sec = time.perf_counter() - t0
    return {"value": k * steps / sec, "unit": "particle-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"first {k} particles of {w.name}, {steps} steps, single-threaded FP64 C"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="tg128")
    ap.add_argument("--form", default="fp32_local")
    ap.add_argument("--drag", default="stokes", choices=["stokes", "schiller_naumann"])
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64-form leg")
    ap.add_argument("--no-sn", action="store_true", help="skip the Schiller-Naumann leg")
    ap.add_argument("--no-hilbert", action="store_true",
                    help="skip the Hilbert placement and bounding-box leg")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the forward+adjoint leg")
    ap.add_argument("--no-scale", action="store_true", help="skip the 1.4e9-particle leg")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB three times (the reference "
                         "for scaling hardware byte counters) and exit")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        n = args.copy_calibration * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "launches": 3}))
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE "
              f"{world}); the particle step is measured on one MI355X", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2603_26691_amd as pkg
    from workloads import synth

    w = synth.get(args.workload)
    steps = args.steps if args.steps is not None else w.nsteps
    res = leg_forward(pkg, torch, np, w, args.form, steps, args.warmup, args.drag)
    value = w.P * steps / (res["ms"] / 1e3)
    form_name = {"fp64": "FP64 form", "fp32_local": "FP32 chunk-local form",
                 "fp32": "FP32 form"}[args.form]
    out = {
        "metric": f"particle-steps/s on 1 MI355X (fwd), {form_name}",
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": res["ms"] / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.form == "fp64" else "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "mesh": list(w.n), "particles": w.P, "dt": w.dt,
                   "form": args.form, "chunk_edge": w.chunk_edge, "drag": args.drag,
                   "source_accumulation": "f32" if args.form == "fp32" else "f64",
                   "parallelism": "single GPU"},
        "roofline": roofline(args.form, w, res["kernel_ms"], res["launches"],
                             res["stats"]["items"], args.drag),
        "step_kernel_share": res["kernel_ms"] / res["ms"],
        "device_copy": {"GBps": device_copy_gbps(torch), "bytes": "1 GiB read + 1 GiB written",
                        "frac_of_peak": None},
        "last_step_movers": res["stats"]["movers"],
        "repacks": res["stats"]["repacks"],
    }
    if not args.no_fp64 and args.form != "fp64":
        r64 = leg_forward(pkg, torch, np, w, "fp64", steps, args.warmup, args.drag)
        out["fp64_form"] = {"value": w.P * steps / (r64["ms"] / 1e3),
                            "ms_per_step": r64["ms"] / steps,
                            "avg_kernel_ms": r64["kernel_ms"] / max(r64["launches"], 1)}
        out["speedup_vs_fp64_form"] = value / out["fp64_form"]["value"]
    if not args.no_sn and args.drag == "stokes":
        rsn = leg_forward(pkg, torch, np, w, args.form, steps, args.warmup, "schiller_naumann")
        out["schiller_naumann"] = {
            "value": w.P * steps / (rsn["ms"] / 1e3), "ms_per_step": rsn["ms"] / steps,
            "roofline": roofline(args.form, w, rsn["kernel_ms"], rsn["launches"],
                                 rsn["stats"]["items"], "schiller_naumann")}
    if not args.no_hilbert:
        out["hilbert"] = leg_hilbert(pkg, torch, np, w)
    if not args.no_adjoint:
        out["fwd_adjoint"] = leg_adjoint(pkg, torch, np, synth)
    if not args.no_scale:
        out["scale_512"] = leg_scale(pkg, torch, np, synth)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w, np)
    out["device_copy"]["frac_of_peak"] = out["device_copy"]["GBps"] / HBM_PEAK_GBS
    out["roofline"]["frac_of_device_copy"] = out["roofline"]["achieved"] / out["device_copy"]["GBps"]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
