"""Benchmark of the spline particle-tracking path on one MI355X.

One step = one pass of the whole path on resident device data:
  spline coefficients of the field (3 axis solves per component)
  -> cell keys + stable radix sort + permutation
  -> Heun RK2 step (two 64-point gathers of (u,v,w) per particle)
  -> adjoint of that RK2 step (re-sort, derivative gathers, scatter-add of the
     coefficient gradient) -> adjoint of the spline solve.
value = 2 * N_p particle interpolations of (u,v,w) per step / step time.

    python bench.py [--steps K] [--warmup W] [--config c3] [--dtype f32|bf16]
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("particle-interpolations/s (u,v,w) at 1024^3, 64M particles; "
          "fwd+adjoint step time")
HBM_PEAK_GBS = 8000.0

CONFIGS = {
    # name: (grid n, particles, kmax, clustered, description)
    "c1": (32, 4096, 15, False, "32^3 grid, 4096 uniform particles"),
    "c2": (512, 16 * 2 ** 20, 170, False, "512^3 grid, 16M uniform particles"),
    "c3": (1024, 64 * 2 ** 20, 341, True,
           "1024^3 grid, 64M particles (half uniform, half in 64 Gaussian blobs, sigma=0.1)"),
    "c4": (256, 2 ** 20, 85, False, "256^3 grid, 1M uniform particles"),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def interp_bytes(n, np_, coeff_bytes, n_out=3):
    """Algorithmic HBM bytes of one interpolation pass: the padded field read
    once plus the particle I/O (FP64 positions in, FP32 outputs out)."""
    return 3 * (n + 3) ** 3 * coeff_bytes + np_ * (24 + 4 * n_out)


def cpu_baseline(n_full, np_full):
    """FP64 oracle, timed on this host, on a bounded sample of the same step:
    the spline solve on a 256^3 grid and the fwd+adjoint particle work for
    2^21 particles, each scaled linearly to the full grid and particle count."""
    import numpy as np

    import oracle
    import synth

    ns, nps = 256, 2 ** 21
    f = synth.spectral_field_np(ns, 85, seed=0)
    pos = synth.uniform_particles_np(nps, seed=1)
    g = oracle.Grid(ns)
    dt = synth.cfl_dt(np.abs(f).max(), ns)
    t0 = time.perf_counter()
    coeff = oracle.spline_coeffs(f)
    t1 = time.perf_counter()
    ps, _, _ = oracle.sort_particles(g, pos, 32, 32)
    p1 = oracle.rk2_step(g, coeff, ps, dt)
    ps2, _, _ = oracle.sort_particles(g, pos, 32, 32)  # the adjoint re-sorts the step input
    gc = np.zeros_like(coeff)
    oracle.rk2_step_bwd(g, coeff, ps2, dt, 2.0 * p1, gc)
    t2 = time.perf_counter()
    gfield = oracle.spline_coeffs_bwd(gc)
    t3 = time.perf_counter()
    del gfield
    grid_scale = (n_full / ns) ** 3
    part_scale = np_full / nps
    t_step = ((t1 - t0) + (t3 - t2)) * grid_scale + (t2 - t1) * part_scale
    return {"value": 2.0 * np_full / t_step, "unit": "particle-interpolations/s",
            "cores": oracle.num_threads(), "kind": "oracle",
            "sample": (f"FP64 oracle: spline solve + solve adjoint on a {ns}^3 grid "
                       f"(x{grid_scale:.0f} to {n_full}^3) and sort + Heun step + step adjoint "
                       f"for {nps} uniform particles (x{part_scale:.0f} to {np_full}); "
                       f"sample took {t3 - t0:.1f} s"),
            "ms_per_step_est": 1e3 * t_step}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="c3", choices=sorted(CONFIGS))
    ap.add_argument("--dtype", default="f32", choices=["f32", "bf16"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--uniform", action="store_true",
                    help="uniform particles instead of the configuration's distribution")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); this build has "
              "no multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2005_13193_amd as pt
    from paper_2005_13193_amd import _binding as B
    import synth

    n, np_, kmax, clustered, desc = CONFIGS[args.config]
    if args.uniform and clustered:
        clustered = False
        desc = desc.split(" (")[0].replace("particles", "uniform particles")
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    cdt = torch.float32 if args.dtype == "f32" else torch.bfloat16
    cb = 4 if args.dtype == "f32" else 2
    g = pt.Grid(n)

    log(f"[bench] config {args.config}: {desc}; coefficients {args.dtype}")
    field = synth.spectral_field_torch(n, kmax, seed=0, device=dev)
    umax = float(field.abs().max())
    dt = synth.cfl_dt(umax, n)
    torch.cuda.synchronize()
    if clustered:
        pos = synth.clustered_particles_torch(np_, sigma=0.1, device=dev)
    else:
        pos = synth.uniform_particles_torch(np_, seed=1, device=dev)
    ids = torch.arange(np_, dtype=torch.int32, device=dev)
    coeff = torch.empty(g.padded_shape, dtype=cdt, device=dev)
    g_coeff = torch.zeros(g.padded_shape, dtype=torch.float32, device=dev)
    g_field = torch.empty(g.field_shape, dtype=torch.float32, device=dev)
    pos_prev = torch.empty_like(pos)
    g_pos = torch.empty_like(pos)
    ws_sp = pt.workspace(B.PT_OP_SPLINE, g, 0, cdt, dev)
    ws_spb = pt.workspace(B.PT_OP_SPLINE_BWD, g, 0, torch.float32, dev)
    ws_f = pt.workspace(B.PT_OP_RK2, g, np_, cdt, dev)
    ws_b = pt.workspace(B.PT_OP_RK2_BWD, g, np_, cdt, dev)
    torch.cuda.synchronize()
    log(f"[bench] inputs ready: dt={dt:.3e}, |u|max={umax:.3f}, "
        f"mem={torch.cuda.memory_allocated() / 2**30:.1f} GiB")

    names = ["spline", "rk2_fwd", "rk2_bwd", "spline_bwd"]
    ev = {k: (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for k in names}
    acc = {k: 0.0 for k in names}

    def step(timed):
        def mark(k, i):
            if timed:
                ev[k][i].record()
        mark("spline", 0)
        B.pt_spline_coeffs(g, field, coeff, ws_sp)
        mark("spline", 1)
        pos_prev.copy_(pos)
        mark("rk2_fwd", 0)
        B.pt_rk2_step(g, coeff, dt, pos, ids, True, ws_f)
        mark("rk2_fwd", 1)
        torch.mul(pos, 2.0, out=g_pos)  # dL/dx for L = sum |x|^2
        mark("rk2_bwd", 0)
        B.pt_rk2_step_bwd(g, coeff, dt, pos_prev, True, g_pos, g_coeff, ws_b)
        mark("rk2_bwd", 1)
        mark("spline_bwd", 0)
        B.pt_spline_coeffs_bwd(g, g_coeff, g_field, ws_spb)
        mark("spline_bwd", 1)
        if timed:
            torch.cuda.synchronize()
            for k in names:
                acc[k] += ev[k][0].elapsed_time(ev[k][1])

    for i in range(args.warmup):
        step(False)
        torch.cuda.synchronize()
        log(f"[bench] warmup step {i + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(True)
        log(f"[bench] timed step {i + 1}/{args.steps} done")
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t0
    ms_step = 1e3 * t_total / args.steps
    status = B.pt_last_device_error()
    if status != 0:
        raise RuntimeError(f"device error flag set: {B.status_string(status)}")
    per = {k: acc[k] / args.steps for k in names}
    value = 2.0 * np_ / (ms_step * 1e-3)

    # algorithmic bytes per call
    n3, p3 = n ** 3, (n + 3) ** 3
    bytes_call = {
        "spline": 3 * n3 * (8 + 8 + 4 + cb),
        "spline_bwd": 3 * (p3 * 4 + n3 * 4) + 3 * 3 * n3 * 8,
        "rk2_fwd": 2 * interp_bytes(n, np_, cb) + np_ * 24,
        "rk2_bwd": 2 * interp_bytes(n, np_, cb) + 3 * p3 * 4 * 2 + np_ * 48,
    }
    dom = max(per, key=per.get)
    achieved = bytes_call[dom] / (per[dom] * 1e-3) / 1e9
    out = {
        "metric": METRIC, "value": value, "unit": "particle-interpolations/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": args.dtype, "data": "synthetic",
        "config": {"workload": desc + f", {args.dtype} coefficients, FP64 positions, "
                   "fwd+adjoint Heun step with cell sort", "grid": n, "particles": np_,
                   "kmax": kmax, "dt": dt, "coeff_dtype": args.dtype},
        "breakdown_ms": per,
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": None},
    }
    if not args.no_cpu_baseline:
        log("[bench] timing the FP64 oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(n, np_)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
