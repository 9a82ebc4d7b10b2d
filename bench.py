"""Benchmark of the per-particle time step on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload tg128] [--form fp32_local]

A step is one pass of the whole hot path (gather, integrate, deposit,
relocate and re-bin) over every particle of the workload.  Inputs are
seeded synthetic data resident in HBM before the timed region starts; K
steps are timed with events on the stream the kernels run on, bracketed by
device synchronisations.  Prints one JSON line with the whole-job
particle-steps/s, the step kernel's roofline figures, the FP64 form on the
same workload and the FP64 oracle timed on this host's cores on a bounded
sample of the same workload.
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


def make_tracker(pkg, w, form):
    return pkg.Tracker(w.n, w.L, w.P, form=form, chunk_edge=w.chunk_edge, rho_f=w.rho_f,
                       mu_f=w.mu_f, g=w.g, rho_p=w.rho_p, parcel_weight=w.parcel_weight)


def inject_all(t, w):
    for b in range(w.n_batches()):
        x, up, d = w.batch(b)
        t.inject(x, up, d)


def time_form(pkg, torch, np, w, form, steps, warmup):
    t = make_tracker(pkg, w, form)
    inject_all(t, w)
    U = w.field()
    U = torch.from_numpy(U if form == "fp64" else U.astype(np.float32)).cuda()
    for _ in range(warmup):
        t.step(U, w.dt)
    torch.cuda.synchronize()
    t.timing(True)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(steps):
        t.step(U, w.dt)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    kernel_ms, launches = t.timing(False)
    st = t.stats()
    t.close()
    del U
    torch.cuda.empty_cache()
    return {"ms": ms, "kernel_ms": kernel_ms, "launches": launches, "stats": st}


def cpu_baseline(w, np, steps=4, max_particles=4_000_000):
    from oracle.oracle import MeshParams, load
    orc = load()
    k = min(w.P, max_particles)
    x, up, d = w.particles(k)
    U = w.field()
    if True:  # the oracle gets the field the FP32 forms use, promoted
        U = U.astype(np.float32).astype(np.float64)
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
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64-form leg")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    args = ap.parse_args()
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
    res = time_form(pkg, torch, np, w, args.form, steps, args.warmup)
    value = w.P * steps / (res["ms"] / 1e3)
    items = res["stats"]["items"]
    bytes_launch, per_p, per_item = algorithmic_bytes(args.form, w.P, items, w.chunk_edge)
    avg_kernel_s = res["kernel_ms"] / max(res["launches"], 1) / 1e3
    achieved = bytes_launch / avg_kernel_s / 1e9
    out = {
        "metric": "particle-steps/s on 1 MI355X (fwd), FP32 chunk-local form",
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
                   "form": args.form, "chunk_edge": w.chunk_edge,
                   "source_accumulation": "f32" if args.form == "fp32" else "f64",
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_step", "avg_kernel_ms": avg_kernel_s * 1e3,
                     "bytes_per_launch": bytes_launch,
                     "model": f"{per_p} B/particle + {per_item} B/work item, {items} items"},
        "step_kernel_share": res["kernel_ms"] / res["ms"],
        "last_step_movers": res["stats"]["movers"],
        "repacks": res["stats"]["repacks"],
    }
    if not args.no_fp64 and args.form != "fp64":
        r64 = time_form(pkg, torch, np, w, "fp64", steps, args.warmup)
        out["fp64_form"] = {"value": w.P * steps / (r64["ms"] / 1e3),
                            "ms_per_step": r64["ms"] / steps,
                            "avg_kernel_ms": r64["kernel_ms"] / max(r64["launches"], 1)}
        out["speedup_vs_fp64_form"] = value / out["fp64_form"]["value"]
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w, np)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
