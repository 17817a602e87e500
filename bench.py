"""Benchmark of the spline particle-tracking path on one MI355X.

One step = one pass of the whole path on resident device data:
  spline coefficients of the field (3 axis solves per component)
  -> cell keys + stable radix sort + permutation of x_n (and the labels)
  -> Heun RK2 step on the sorted particles (two 64-point gathers of (u,v,w)
     per particle)
  -> adjoint of that RK2 step on the same order (derivative gathers,
     scatter-add of the coefficient gradient) -> adjoint of the spline solve.
value = 2 * N_p particle interpolations of (u,v,w) per step / step time.

With --workload tv a step is instead the forward step in a field that changes
over the step (coefficients recomputed at each Runge-Kutta sub-step):
  spline solve of the field at t_n -> sort + stage 1 (u^n at x)
  spline solve of the field at t_n + dt -> stage 2 (u^{n+1} at x*),
each solve on a second stream, overlapped with the gather stage before it.

With --workload slab a step is the spline solve of one device's z-slab of a
2048^3 grid split 8 ways (256 planes, z lines solved with open ends over 16
halo planes per side).

With --workload inertial a step is one inertial-particle step (Stokes drag,
response time tau = 2 dt, particles launched at twice the local fluid
velocity, so that they move up to about 1.2 cells per step) with the cell
sort, on the configuration's particles.

With --workload c5 (2048^3 grid, 256M uniform particles; coefficients of the
frozen field computed once, outside the timed steps) a step is the cell sort,
the 12-output gather of (u, v, w) and the nine velocity gradients at every
particle (column-tiled), and the Heun step on the sorted particles.

--dtype f64 runs the FP64 form of the same step (FP64 solves and gathers),
the baseline the FP32 and BF16 forms are compared with. The default run (FP32
coefficients) also times, after its timed steps and outside them, three steps
of the same path with BF16 and with FP64 coefficients on the same inputs
("forms" in the JSON line).

    python bench.py [--steps K] [--warmup W] [--config c3] [--dtype f32|bf16|f64]
                    [--workload fwd_adjoint|tv|slab|inertial|c5] [--no-overlap]
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
METRIC_SLAB = ("spline coefficient points/s, one 256-plane z-slab (halo 16) of a "
               "2048^3 grid")
METRIC_TV = ("particle-interpolations/s (u,v,w) at 1024^3, 64M particles; "
             "forward step with the coefficients recomputed at each RK sub-step")
METRIC_INERTIAL = ("inertial-particle steps/s at 1024^3, 64M particles (Stokes drag, "
                   "sort every step)")
METRIC_C5 = ("particle steps/s at 2048^3, 256M particles: sort, 12-output gather "
             "(u,v,w and 9 gradients), Heun step")
HBM_PEAK_GBS = 8000.0

CONFIGS = {
    # name: (grid n, particles, kmax, clustered, description)
    "c1": (32, 4096, 15, False, "32^3 grid, 4096 uniform particles"),
    "c2": (512, 16 * 2 ** 20, 170, False, "512^3 grid, 16M uniform particles"),
    "c3": (1024, 64 * 2 ** 20, 341, True,
           "1024^3 grid, 64M particles (half uniform, half in 64 Gaussian blobs, sigma=0.1)"),
    "c4": (256, 2 ** 20, 85, False, "256^3 grid, 1M uniform particles"),
    "c5": (2048, 256 * 2 ** 20, 682, False, "2048^3 grid, 256M uniform particles"),
}
DTYPES = {"f32": ("float32", 4), "bf16": ("bfloat16", 2), "f64": ("float64", 8)}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


KERNELS = ("spline_x", "spline_y", "spline_z", "spline_x_pad", "spline_x_fold",
           "spline_y_carry", "spline_yx_pad", "spline_fold_y_carry", "spline_fyx",
           "sorted_table", "sort_keys",
           "sort_pass", "sort_permute", "tile_rk2_fwd", "tile_rk2_fwd_save", "rk2_bwd_saved",
           "tile_rk2_fwd_grad",
           "tile_rk2_bwd_gather", "tile_scatter",
           "tile_tv_stage1", "tile_tv_stage2", "tile_inertial", "tile_interp", "tile_interp_grad",
           "inertial_direct", "interp", "rk2_direct_stage2", "rk2_direct_bwd",
           "rk2_direct_bwd_gather")


def key_bytes(n):
    """Bytes of one cell key on an n^3 grid (32 x 32-cell columns)."""
    total = -(-n // 32) ** 2 * n * 1024
    return 8 if (total - 1).bit_length() > 32 else 4


def launch_bytes(kernel, n, np_, cb, launches_per_step, vb=4):
    """Algorithmic HBM bytes of one launch: every array the kernel must touch,
    read or written once (n^3 grid points, (n+3)^3 padded coefficients per
    component, np_ particles with FP64 positions; cb bytes per stored
    coefficient, vb per velocity value: 8 for the FP64 form)."""
    n3, p3, kb = n ** 3, (n + 3) ** 3, key_bytes(n)
    per_step = {
        "spline_x": 8 * n3, "spline_y": 8 * n3, "spline_z": 8 * n3,
        "spline_x_pad": 4 * n3 + cb * p3,
        "spline_x_fold": 4 * p3 + 4 * n3,
        # fused y + x: the y lines' run carries (2 floats per 16 rows) are
        # written by the first pass and read by the second
        "spline_y_carry": 4 * n3 + 8 * n3 // 16,
        "spline_yx_pad": 4 * n3 + 8 * n3 // 16 + cb * p3,
        # the adjoint's fused fold + y + x: carries of the folded y lines
        # (padded gradient read, carries written), then the padded gradient
        # and the carries read and the plain field written
        "spline_fold_y_carry": 4 * p3 + 8 * n3 // 16,
        "spline_fyx": 4 * p3 + 8 * n3 // 16 + 4 * n3,
        "sort_keys": np_ * (24 + kb + 4),
        "sort_pass": np_ * 2 * (kb + 4),
        "sort_permute": np_ * (4 + 24 + 24),
        # the particle table of positions already in cell order
        "sorted_table": np_ * 24,
        # x in, x_out out; field once
        "tile_rk2_fwd": 3 * p3 * cb + np_ * 48,
        # x in; x_out, u0 and the velocity gradients at both stage points
        # (21 floats) out
        "tile_rk2_fwd_save": 3 * p3 * cb + np_ * (48 + 84),
        # x in; x_out and the 12 values at x_n out
        "tile_rk2_fwd_grad": 3 * p3 * cb + np_ * (48 + 48),
        # lambda and both gradients in; dL/dx_n and the adjoints of both
        # stage velocities out
        "rk2_bwd_saved": np_ * (24 + 72 + 24 + 24),
        # x, lambda in; dL/dx_n, stage-1 velocity and the adjoints of both
        # stage velocities out
        "tile_rk2_bwd_gather": 3 * p3 * cb + np_ * 108,
        # all colours of one step together: the FP32 gradient read and
        # written once, x, u0, ub0, ub1 read once
        "tile_scatter": (3 * p3 * 4 * 2 + np_ * 60) / launches_per_step,
        # x in, x (sorted order) and u^n out; field once
        "tile_tv_stage1": 3 * p3 * cb + np_ * 60,
        # x and u^n in, x out; field once
        "tile_tv_stage2": 3 * p3 * cb + np_ * 60,
        # x, v in; x, v out; field once
        "tile_inertial": 3 * p3 * cb + np_ * (48 + 24),
        "inertial_direct": 3 * p3 * cb + np_ * (48 + 6 * vb),
        # x in, 3 or 12 values out
        "tile_interp": 3 * p3 * cb + np_ * (24 + 12),
        "tile_interp_grad": 3 * p3 * cb + np_ * (24 + 48),
        # one thread per particle (FP64 form): u0 = u(x); x, u0 in, x out;
        # adjoint: two gathers and the FP32 gradient read and written once
        "interp": 3 * p3 * cb + np_ * (24 + 3 * vb),
        "rk2_direct_stage2": 3 * p3 * cb + np_ * (48 + 3 * vb),
        "rk2_direct_bwd": 2 * 3 * p3 * cb + 2 * 3 * p3 * 4 + np_ * (24 + 3 * vb + 48 + 96),
        # x, lambda in; dL/dx_n, u0, ub0, ub1 out (for the tiled scatter)
        "rk2_direct_bwd_gather": 3 * p3 * cb + np_ * (48 + 24 + 36),
    }
    return per_step[kernel]


def source_digest():
    """SHA-256 over the HIP sources, to tie a stored counter figure to the
    kernels it was measured on."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2005_13193_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, config, dtype, clustered):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary for this workload (FETCH_SIZE + WRITE_SIZE, scaled by the copy
    calibration), or None if there is none or the kernels changed since."""
    dist = "clustered" if clustered else "uniform"
    path = os.path.join(ROOT, "profiles", f"{kernel}_{config}_{dist}_{dtype}_hbm_traffic.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith(" "):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("source_digest") != source_digest():
        return None
    try:
        return float(vals["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(n_full, np_full, clustered):
    """FP64 oracle, timed on this host, on a bounded sample of the same step:
    the spline solve and its adjoint on a 512^3 grid and the fwd+adjoint
    particle work (sort, Heun step, step adjoint) for 2^24 particles
    of the workload's distribution, each scaled linearly to the full grid and
    particle count; then the same on one core for a 256^3 grid and 2^20
    particles."""
    import numpy as np

    import oracle
    import synth

    def sample(ns, nps):
        f = synth.spectral_field_torch(ns, ns // 3, seed=0, device="cuda:0").double().cpu().numpy()
        if clustered:
            pos = synth.clustered_particles_np(nps)
        else:
            pos = synth.uniform_particles_np(nps, seed=1)
        g = oracle.Grid(ns)
        dt = synth.cfl_dt(np.abs(f).max(), ns)
        t0 = time.perf_counter()
        coeff = oracle.spline_coeffs(f)
        t1 = time.perf_counter()
        ps, _, _ = oracle.sort_particles(g, pos, 32, 32)
        p1 = oracle.rk2_step(g, coeff, ps, dt)
        gc = np.zeros_like(coeff)
        oracle.rk2_step_bwd(g, coeff, ps, dt, 2.0 * p1, gc)
        t2 = time.perf_counter()
        oracle.spline_coeffs_bwd(gc)
        t3 = time.perf_counter()
        grid_scale = (n_full / ns) ** 3
        part_scale = np_full / nps
        t_step = ((t1 - t0) + (t3 - t2)) * grid_scale + (t2 - t1) * part_scale
        desc = (f"FP64 oracle: spline solve + solve adjoint on a {ns}^3 grid "
                f"(x{grid_scale:.0f} to {n_full}^3) and sort + Heun step + step adjoint "
                f"for {nps} {'clustered' if clustered else 'uniform'} particles "
                f"(x{part_scale:.0f} to {np_full}); sample took {t3 - t0:.1f} s")
        return t_step, desc

    cores = oracle.num_threads()
    t_step, desc = sample(512, 2 ** 24)
    out = {"value": 2.0 * np_full / t_step, "unit": "particle-interpolations/s",
           "cores": cores, "kind": "oracle", "sample": desc, "ms_per_step_est": 1e3 * t_step}
    oracle.set_num_threads(1)
    try:
        t1c, desc1 = sample(256, 2 ** 20)
    finally:
        oracle.set_num_threads(cores)
    out["one_core"] = {"value": 2.0 * np_full / t1c, "unit": "particle-interpolations/s",
                       "cores": 1, "kind": "oracle", "sample": desc1,
                       "ms_per_step_est": 1e3 * t1c}
    return out


def oracle_errors(g, field, pos_n, pos_1, uvw, dt, sample):
    """Max normwise error of the timed run against the FP64 oracle on a
    sample of particles (the windowed closed form of the oracle, read from the
    FP32 field the GPU used): the displacement of the last Heun step and
    (u, v, w) at the step's starting points."""
    import numpy as np

    import oracle

    fh = np.empty(tuple(field.shape), dtype=np.float32)
    n = field.shape[1]
    for c in range(3):
        for z0 in range(0, n, max(1, n // 16)):
            fh[c, z0:z0 + n // 16] = field[c, z0:z0 + n // 16].cpu().numpy()
    og = oracle.Grid(g.nx, g.ny, g.nz)
    x0 = pos_n[:, sample].double().cpu().numpy()
    x1 = pos_1[:, sample].double().cpu().numpy()
    u = uvw[:, sample].double().cpu().numpy()

    def normwise(y, ref):
        return max(float(np.abs(y[r] - ref[r]).max() / max(np.abs(ref[r]).max(), 1e-300))
                   for r in range(ref.shape[0]))

    ref1 = oracle.rk2_window(og, fh, x0, dt, 1)
    refu = oracle.interp_window(og, fh, x0, n_out=3)
    return {"displacement": normwise(x1 - x0, ref1 - x0), "uvw": normwise(u, refu),
            "sample": f"{x0.shape[1]} particles of the last timed step, windowed FP64 oracle "
                      "on the FP32 field"}


def c4_adjoint_time(torch, pt, synth, reps=3):
    """fwd+adjoint of K = 8 Heun steps with position checkpoints every 2
    steps (TrackParticles) at 256^3 with 1M particles, FP32: ms per call."""
    from paper_2005_13193_amd.autograd import TrackParticles
    n, np_, K = 256, 2 ** 20, 8
    g = pt.Grid(n)
    field = synth.spectral_field_torch(n, 85, seed=0, device="cuda:0")
    dt = synth.cfl_dt(float(field.abs().max()), n)
    pos0 = synth.uniform_particles_torch(np_, seed=1, device="cuda:0")

    def once():
        f = field.clone().requires_grad_(True)
        p = pos0.clone().requires_grad_(True)
        xk, _ = TrackParticles.apply(f, p, g, dt, K)
        (xk * xk).sum().backward()

    once()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        once()
    torch.cuda.synchronize()
    return 1e3 * (time.perf_counter() - t0) / reps


def cpu_baseline_tv(n_full, np_full, clustered):
    """FP64 oracle on a bounded sample of the time-varying step: two spline
    solves on a 512^3 grid, and sort + the two-field Heun step for 2^25
    particles, each scaled linearly to the full grid and particle count."""
    import numpy as np

    import oracle
    import synth

    ns, nps = 512, 2 ** 25
    fa = synth.spectral_field_torch(ns, ns // 3, seed=0, device="cuda:0").double().cpu().numpy()
    fb = synth.spectral_field_torch(ns, ns // 3, seed=1, device="cuda:0").double().cpu().numpy()
    pos = synth.clustered_particles_np(nps) if clustered else synth.uniform_particles_np(nps, seed=1)
    g = oracle.Grid(ns)
    dt = synth.cfl_dt(max(np.abs(fa).max(), np.abs(fb).max()), ns)
    t0 = time.perf_counter()
    ca = oracle.spline_coeffs(fa)
    cb = oracle.spline_coeffs(fb)
    t1 = time.perf_counter()
    ps, _, _ = oracle.sort_particles(g, pos, 32, 32)
    oracle.rk2_step_tv(g, ca, cb, ps, dt)
    t2 = time.perf_counter()
    t_step = (t1 - t0) * (n_full / ns) ** 3 + (t2 - t1) * (np_full / nps)
    return {"value": 2.0 * np_full / t_step, "unit": "particle-interpolations/s",
            "cores": oracle.num_threads(), "kind": "oracle",
            "sample": (f"FP64 oracle: two spline solves on a {ns}^3 grid "
                       f"(x{(n_full / ns) ** 3:.0f} to {n_full}^3) and sort + two-field Heun "
                       f"step for {nps} {'clustered' if clustered else 'uniform'} particles "
                       f"(x{np_full / nps:.0f} to {np_full}); sample took {t2 - t0:.1f} s"),
            "ms_per_step_est": 1e3 * t_step}


def kernel_stats(B, steps):
    out = {}
    for k in KERNELS:
        ms, nl = B.pt_timing_read(k)
        if nl:
            out[k] = {"ms_per_step": ms / steps, "launches_per_step": nl / steps,
                      "avg_launch_ms": ms / nl}
    return out


def roofline(kstats, n, np_, cb, config, dtype, clustered):
    dom = max(kstats, key=lambda k: kstats[k]["ms_per_step"])
    bpl = launch_bytes(dom, n, np_, cb, kstats[dom]["launches_per_step"], 8 if cb == 8 else 4)
    achieved = bpl / (kstats[dom]["avg_launch_ms"] * 1e-3) / 1e9
    return {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
            "traffic": measured_traffic(dom, config, dtype, clustered),
            "algorithmic_bytes_per_launch": bpl}


def cpu_baseline_slab(points_full):
    """FP64 oracle spline solve of an 896^3 periodic grid, scaled linearly to
    the slab's coefficient points."""
    import oracle
    import synth

    ns = 896
    f = synth.spectral_field_torch(ns, ns // 3, seed=0, device="cuda:0").double().cpu().numpy()
    t0 = time.perf_counter()
    oracle.spline_coeffs(f)
    t = time.perf_counter() - t0
    pts = 3 * (ns + 3) ** 3
    return {"value": pts / t, "unit": "points/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"FP64 oracle periodic solve of a {ns}^3 grid ({t:.1f} s), per point",
            "ms_per_step_est": 1e3 * t * points_full / pts}


def run_slab(args, torch, pt, B, synth, cdt, cb):
    """The spline solve of one device's z-slab: 256 planes of a 2048^3 grid
    (one of 8), z lines with open ends over 16 halo planes per side."""
    dev = torch.device("cuda:0")
    n, nzl, halo = 2048, 256, 16
    nzi = nzl + 3 + 2 * halo
    g = pt.Grid(n)
    # planes -1-halo .. nzl+1+halo (mod n) of the 2048^3 synthetic field
    full = synth.spectral_field_torch_chunked(n, n // 3, seed=0, device=dev)
    planes = torch.tensor([(-1 - halo + i) % n for i in range(nzi)], device=dev)
    field = full.index_select(1, planes).contiguous()
    del full
    torch.cuda.empty_cache()
    out = torch.empty((3, nzl + 3, n + 3, n + 3), dtype=cdt, device=dev)
    ws = pt.workspace(B.PT_OP_SPLINE_SLAB, g, nzi, cdt, dev)
    torch.cuda.synchronize()
    for i in range(args.warmup):
        B.pt_spline_coeffs_slab(g, nzl, halo, field, out, ws)
        torch.cuda.synchronize()
        log(f"[bench] warmup step {i + 1}/{args.warmup} done")
    for k in KERNELS:
        B.pt_timing_read(k)
    B.pt_timing_enable(True)
    t0 = time.perf_counter()
    for i in range(args.steps):
        B.pt_spline_coeffs_slab(g, nzl, halo, field, out, ws)
    torch.cuda.synchronize()
    ms_step = 1e3 * (time.perf_counter() - t0) / args.steps
    kstats = kernel_stats(B, args.steps)
    B.pt_timing_enable(False)
    points = 3 * (nzl + 3) * (n + 3) ** 2
    # algorithmic bytes per launch: z pass reads and writes nzi planes, y
    # pass nzl + 3 planes in place, x pass reads nzl + 3 planes and writes the
    # padded output
    plane = n * n
    per = {"spline_z": 8 * plane * nzi, "spline_y": 8 * plane * (nzl + 3),
           "spline_x_pad": 4 * plane * (nzl + 3) + cb * (nzl + 3) * (n + 3) ** 2}
    dom = max(kstats, key=lambda k: kstats[k]["ms_per_step"])
    achieved = per[dom] / (kstats[dom]["avg_launch_ms"] * 1e-3) / 1e9
    out_line = {
        "metric": METRIC_SLAB, "value": points / (ms_step * 1e-3), "unit": "points/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": args.dtype,
        "data": "synthetic",
        "config": {"workload": f"z-slab of a 2048^3 grid: {nzl} planes + 2 x {halo} halo planes, "
                   f"{args.dtype} coefficients", "grid": n, "slab_planes": nzl, "halo": halo},
        "kernels": kstats,
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(dom, "slab", args.dtype, False),
                     "algorithmic_bytes_per_launch": per[dom]},
    }
    if not args.no_cpu_baseline:
        log("[bench] timing the FP64 oracle on a bounded sample")
        out_line["cpu_baseline"] = cpu_baseline_slab(points)
    print(json.dumps(out_line), flush=True)


def run_tv(args, torch, pt, B, synth, n, np_, kmax, clustered, desc, cdt, cb):
    """Forward steps in a field that changes over the step: per step two
    spline solves (fields at t_n and t_n + dt) and the two gather stages; each
    solve runs on a second stream while the gather stage before it runs."""
    dev = torch.device("cuda:0")
    g = pt.Grid(n)
    fa = synth.spectral_field_torch(n, kmax, seed=0, device=dev)
    fb = synth.spectral_field_torch(n, kmax, seed=1, device=dev)
    dt = synth.cfl_dt(max(float(fa.abs().max()), float(fb.abs().max())), n)
    pos = (synth.clustered_particles_torch(np_, sigma=0.1, device=dev) if clustered
           else synth.uniform_particles_torch(np_, seed=1, device=dev))
    ids = torch.arange(np_, dtype=torch.int32, device=dev)
    ca = torch.empty(g.padded_shape, dtype=cdt, device=dev)
    cbuf = torch.empty(g.padded_shape, dtype=cdt, device=dev)
    u_n = torch.empty((3, np_), dtype=torch.float32, device=dev)
    ws_sp = pt.workspace(B.PT_OP_SPLINE, g, 0, cdt, dev)
    ws = pt.workspace(B.PT_OP_RK2, g, np_, cdt, dev)
    main_s = torch.cuda.current_stream()
    side = torch.cuda.Stream() if not args.no_overlap else main_s
    torch.cuda.synchronize()
    log(f"[bench] tv inputs ready: dt={dt:.3e}, mem={torch.cuda.memory_allocated() / 2**30:.1f} GiB")
    # the field at t_n of the first step
    B.pt_spline_coeffs(g, fa, ca, ws_sp)
    ev_a, ev_b, ev_s1, ev_s2 = (torch.cuda.Event() for _ in range(4))
    ev_a.record(main_s)   # ca holds the coefficients at t_n
    ev_s2.record(main_s)  # cbuf is free

    def step():
        # side: coefficients of the field at t_n + dt, while stage 1 runs
        side.wait_event(ev_s2)
        B.pt_spline_coeffs(g, fb, cbuf, ws_sp, stream=side)
        ev_b.record(side)
        main_s.wait_event(ev_a)
        B.pt_rk2_stage1(g, ca, pos, ids, True, u_n, ws)
        ev_s1.record(main_s)
        main_s.wait_event(ev_b)
        B.pt_rk2_stage2(g, cbuf, dt, pos, u_n, True, ws)
        ev_s2.record(main_s)
        # side: the next step's field at t_n, once stage 1 no longer reads ca
        side.wait_event(ev_s1)
        B.pt_spline_coeffs(g, fa, ca, ws_sp, stream=side)
        ev_a.record(side)

    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log(f"[bench] warmup step {i + 1}/{args.warmup} done")
    for k in KERNELS:
        B.pt_timing_read(k)
    B.pt_timing_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step()
        log(f"[bench] timed step {i + 1}/{args.steps} issued")
    torch.cuda.synchronize()
    ms_step = 1e3 * (time.perf_counter() - t0) / args.steps
    status = B.pt_last_device_error()
    if status != 0:
        raise RuntimeError(f"device error flag set: {B.status_string(status)}")
    kstats = kernel_stats(B, args.steps)
    B.pt_timing_enable(False)
    out = {
        "metric": METRIC_TV, "value": 2.0 * np_ / (ms_step * 1e-3),
        "unit": "particle-interpolations/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": args.dtype, "data": "synthetic",
        "config": {"workload": desc + f", {args.dtype} coefficients, FP64 positions, Heun step "
                   "with the coefficients of the field at t_n (predictor) and t_n+dt "
                   "(corrector) recomputed every step, cell sort every step"
                   + ("" if args.no_overlap else ", solves overlapped on a second stream"),
                   "grid": n, "particles": np_, "kmax": kmax, "dt": dt,
                   "coeff_dtype": args.dtype, "overlap": not args.no_overlap},
        "kernels": kstats,
        "roofline": roofline(kstats, n, np_, cb, args.config + "_tv", args.dtype, clustered),
    }
    if not args.no_cpu_baseline:
        log("[bench] timing the FP64 oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline_tv(n, np_, clustered)
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="c3", choices=sorted(CONFIGS))
    ap.add_argument("--dtype", default="f32", choices=sorted(DTYPES))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the sorted-gather timing, the C4 adjoint timing and the "
                         "sampled oracle error after the timed steps")
    ap.add_argument("--workload", default="fwd_adjoint",
                    choices=["fwd_adjoint", "tv", "slab", "inertial", "c5"])
    ap.add_argument("--no-save", action="store_true",
                    help="fwd_adjoint: the forward step keeps nothing and the adjoint "
                         "gathers the velocity gradients itself (pt_rk2_step_out + "
                         "pt_rk2_step_bwd instead of pt_rk2_step_save + "
                         "pt_rk2_step_bwd_saved)")
    ap.add_argument("--no-overlap", action="store_true",
                    help="tv: run the solves on the main stream (no overlap)")
    ap.add_argument("--uniform", action="store_true",
                    help="uniform particles instead of the configuration's distribution")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB between two device buffers 3 times (reference "
                         "kernel for scaling HBM counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}): the library "
              "has no multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.copy_calibration:
        nb = args.copy_calibration * 2 ** 20
        a = torch.ones(nb // 4, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        for i in range(3):
            b.copy_(a)
            torch.cuda.synchronize()
            log(f"[bench] copy {i + 1}/3 of {nb} bytes done")
        print(json.dumps({"copy_bytes_read": nb, "copy_bytes_written": nb}), flush=True)
        return

    import paper_2005_13193_amd as pt
    from paper_2005_13193_amd import _binding as B
    import synth

    if args.workload == "c5":
        args.config = "c5"
    n, np_, kmax, clustered, desc = CONFIGS[args.config]
    if args.uniform and clustered:
        clustered = False
        desc = desc.split(" (")[0].replace("particles", "uniform particles")
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    cdt = getattr(torch, DTYPES[args.dtype][0])
    cb = DTYPES[args.dtype][1]
    g = pt.Grid(n)

    log(f"[bench] config {args.config}: {desc}; coefficients {args.dtype}")
    if args.workload == "tv":
        run_tv(args, torch, pt, B, synth, n, np_, kmax, clustered, desc, cdt, cb)
        return
    if args.workload == "slab":
        run_slab(args, torch, pt, B, synth, cdt, cb)
        return
    if args.workload == "inertial":
        run_inertial(args, torch, pt, B, synth, n, np_, kmax, clustered, desc, cdt, cb)
        return
    if args.workload == "c5":
        run_c5(args, torch, pt, B, synth, n, np_, kmax, desc, cdt, cb)
        return
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
    pos_n = torch.empty_like(pos)
    perm = torch.empty(np_, dtype=torch.int32, device=dev)
    g_pos = torch.empty_like(pos)
    ws_sp = pt.workspace(B.PT_OP_SPLINE, g, 0, cdt, dev)
    ws_spb = pt.workspace(B.PT_OP_SPLINE_BWD, g, 0, torch.float32, dev)
    ws_s = pt.workspace(B.PT_OP_SORT, g, np_, cdt, dev)
    ws_f = pt.workspace(B.PT_OP_RK2, g, np_, cdt, dev)
    ws_b = pt.workspace(B.PT_OP_RK2_BWD, g, np_, cdt, dev)
    # the forward keeps u0 and both stages' velocity gradients for the
    # adjoint (the tiled FP32 / BF16 forms)
    save = args.dtype != "f64" and not args.no_save
    saved = torch.empty((21, np_), dtype=torch.float32, device=dev) if save else None
    torch.cuda.synchronize()
    log(f"[bench] inputs ready: dt={dt:.3e}, |u|max={umax:.3f}, "
        f"mem={torch.cuda.memory_allocated() / 2**30:.1f} GiB")

    names = ["spline", "sort", "rk2_fwd", "rk2_bwd", "spline_bwd"]
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
        # one cell sort per step: x_n (and the labels) into cell order, kept
        # for the adjoint; the step and its adjoint then skip their own sort
        mark("sort", 0)
        B.pt_sort_particles(g, pos, pos_n, perm, ids, None, ws_s)
        mark("sort", 1)
        mark("rk2_fwd", 0)
        # x_n stays in pos_n for the adjoint; x_{n+1} goes to pos
        if save:
            B.pt_rk2_step_save(g, coeff, dt, pos_n, pos, saved, ws_f)
        else:
            B.pt_rk2_step_out(g, coeff, dt, pos_n, pos, B.PT_SORTED, ws_f)
        mark("rk2_fwd", 1)
        torch.mul(pos, 2.0, out=g_pos)  # dL/dx for L = sum |x|^2
        mark("rk2_bwd", 0)
        if save:
            B.pt_rk2_step_bwd_saved(g, dt, pos_n, saved, g_pos, g_coeff, ws_b)
        else:
            B.pt_rk2_step_bwd(g, coeff, dt, pos_n, B.PT_SORTED, g_pos, g_coeff, ws_b)
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
    for k in KERNELS:  # drop anything recorded before the timed region
        B.pt_timing_read(k)
    B.pt_timing_enable(True)
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

    kstats = kernel_stats(B, args.steps)
    B.pt_timing_enable(False)
    out = {
        "metric": METRIC, "value": value, "unit": "particle-interpolations/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": args.dtype, "data": "synthetic",
        "config": {"workload": desc + f", {args.dtype} coefficients, FP64 positions, "
                   "fwd+adjoint Heun step with cell sort", "grid": n, "particles": np_,
                   "kmax": kmax, "dt": dt, "coeff_dtype": args.dtype,
                   "adjoint": ("from the forward's saved gradients" if save
                               else "gathers its own gradients")},
        "breakdown_ms": per,
        "kernels": kstats,
        "roofline": roofline(kstats, n, np_, cb, args.config, args.dtype, clustered),
    }
    if args.dtype != "f64":
        out["deferred_particles"] = B.pt_tiled_deferred(B.PT_OP_RK2, g, pt._code(cdt), np_, ws_f)
    del saved
    uvw = None
    if not args.no_extras:
        # after the timed steps: (u, v, w) alone at the last step's sorted x_n
        del ws_s, ws_b, g_field, perm
        torch.cuda.empty_cache()
        ws_i = pt.workspace(B.PT_OP_INTERP_SORTED, g, np_, cdt, dev)
        uvw = torch.empty((3, np_), dtype=B.value_dtype(coeff), device=dev)
        B.pt_interp_sorted(g, coeff, pos_n, uvw, ws_i)
        torch.cuda.synchronize()
        for k in KERNELS:
            B.pt_timing_read(k)
        B.pt_timing_enable(True)
        reps = 5
        t0 = time.perf_counter()
        for _ in range(reps):
            B.pt_interp_sorted(g, coeff, pos_n, uvw, ws_i)
        torch.cuda.synchronize()
        ms_i = 1e3 * (time.perf_counter() - t0) / reps
        ks = kernel_stats(B, reps)
        B.pt_timing_enable(False)
        kname = "tile_interp" if args.dtype != "f64" else "interp"
        kb = launch_bytes(kname, n, np_, cb, 1, 8 if cb == 8 else 4)
        k_ms = ks[kname]["avg_launch_ms"] if kname in ks else ms_i
        out["interp_sorted"] = {
            "what": "(u,v,w) alone at the sorted x_n of the last step (pt_interp_sorted)",
            "ms": ms_i, "particles_per_s": np_ / (ms_i * 1e-3), "kernel": kname,
            "kernel_ms": k_ms, "hbm_frac": kb / (k_ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
        del ws_i
        torch.cuda.empty_cache()
        log("[bench] timing the 256^3 / 1M / K=8 fwd+adjoint (checkpoints every 2 steps)")
        out["c4_fwd_adjoint_k8_ms"] = c4_adjoint_time(torch, pt, synth)
        if args.dtype == "f32":
            # the same step with the other coefficient storages, on the same
            # field and particles (after the timed steps, outside them)
            out["forms"] = {}
            for other in ("bf16", "f64"):
                log(f"[bench] the same step with {other} coefficients")
                ms_o = other_form_step_ms(torch, pt, B, g, field, pos, ids, dt, other)
                out["forms"][other] = {"ms_per_step": ms_o,
                                       "value": 2.0 * np_ / (ms_o * 1e-3),
                                       "steps": 3, "warmup": 1,
                                       "what": "the same fwd+adjoint step with "
                                               f"{other} coefficients, same inputs"}
    if not args.no_cpu_baseline:
        if uvw is not None:
            log("[bench] sampled error against the FP64 oracle")
            sample = torch.arange(0, np_, max(1, np_ // 256), device=dev)
            out["error"] = oracle_errors(g, field, pos_n, pos, uvw, dt, sample)
        log("[bench] timing the FP64 oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(n, np_, clustered)
    print(json.dumps(out), flush=True)


def other_form_step_ms(torch, pt, B, g, field, pos, ids, dt, dtype_name, steps=3):
    """ms per fwd+adjoint step (the benchmark's step: solve, sort, Heun
    step, its adjoint, solve adjoint) with another coefficient storage, on
    the given field and particles; buffers of its own (x and the labels
    included: the caller's are left as they were), freed on return."""
    dev = pos.device
    cdt = getattr(torch, DTYPES[dtype_name][0])
    np_ = pos.shape[1]
    pos, ids = pos.clone(), ids.clone()
    coeff = torch.empty(g.padded_shape, dtype=cdt, device=dev)
    g_coeff = torch.zeros(g.padded_shape, dtype=torch.float32, device=dev)
    g_field = torch.empty(g.field_shape, dtype=torch.float32, device=dev)
    pos_n = torch.empty_like(pos)
    perm = torch.empty(np_, dtype=torch.int32, device=dev)
    g_pos = torch.empty_like(pos)
    ws_sp = pt.workspace(B.PT_OP_SPLINE, g, 0, cdt, dev)
    ws_spb = pt.workspace(B.PT_OP_SPLINE_BWD, g, 0, torch.float32, dev)
    ws_s = pt.workspace(B.PT_OP_SORT, g, np_, cdt, dev)
    ws_f = pt.workspace(B.PT_OP_RK2, g, np_, cdt, dev)
    ws_b = pt.workspace(B.PT_OP_RK2_BWD, g, np_, cdt, dev)
    save = dtype_name != "f64"  # as the timed steps: the tiled forms keep the gradients
    saved = torch.empty((21, np_), dtype=torch.float32, device=dev) if save else None

    def step():
        B.pt_spline_coeffs(g, field, coeff, ws_sp)
        B.pt_sort_particles(g, pos, pos_n, perm, ids, None, ws_s)
        if save:
            B.pt_rk2_step_save(g, coeff, dt, pos_n, pos, saved, ws_f)
        else:
            B.pt_rk2_step_out(g, coeff, dt, pos_n, pos, B.PT_SORTED, ws_f)
        torch.mul(pos, 2.0, out=g_pos)
        if save:
            B.pt_rk2_step_bwd_saved(g, dt, pos_n, saved, g_pos, g_coeff, ws_b)
        else:
            B.pt_rk2_step_bwd(g, coeff, dt, pos_n, B.PT_SORTED, g_pos, g_coeff, ws_b)
        B.pt_spline_coeffs_bwd(g, g_coeff, g_field, ws_spb)

    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / steps
    status = B.pt_last_device_error()
    if status != 0:
        raise RuntimeError(f"device error flag set: {B.status_string(status)}")
    del pos, ids, coeff, g_coeff, g_field, pos_n, perm, g_pos, ws_sp, ws_spb, ws_s, ws_f, ws_b
    del saved
    torch.cuda.empty_cache()
    return ms


def run_inertial(args, torch, pt, B, synth, n, np_, kmax, clustered, desc, cdt, cb):
    """Inertial particles (Stokes drag, tau = 2 dt) launched at twice the
    local fluid velocity: one step with the cell sort per timed step, the
    coefficients of the frozen field computed once before."""
    dev = torch.device("cuda:0")
    g = pt.Grid(n)
    field = synth.spectral_field_torch(n, kmax, seed=0, device=dev)
    dt = synth.cfl_dt(float(field.abs().max()), n)
    tau = 2.0 * dt
    coeff = pt.spline_coeffs(g, field, cdt)
    del field
    torch.cuda.empty_cache()
    pos = (synth.clustered_particles_torch(np_, sigma=0.1, device=dev) if clustered
           else synth.uniform_particles_torch(np_, seed=1, device=dev))
    vel = 2.0 * pt.interp_uvw(g, coeff, pos)
    ids = torch.arange(np_, dtype=torch.int32, device=dev)
    ws = pt.workspace(B.PT_OP_INERTIAL, g, np_, cdt, dev)
    torch.cuda.synchronize()

    def step():
        B.pt_inertial_step(g, coeff, dt, tau, pos, vel, None, ids, B.PT_SORT, ws)

    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log(f"[bench] warmup step {i + 1}/{args.warmup} done")
    for k in KERNELS:
        B.pt_timing_read(k)
    B.pt_timing_enable(True)
    t0 = time.perf_counter()
    for i in range(args.steps):
        step()
        log(f"[bench] timed step {i + 1}/{args.steps} issued")
    torch.cuda.synchronize()
    ms_step = 1e3 * (time.perf_counter() - t0) / args.steps
    if B.pt_last_device_error() != 0:
        raise RuntimeError("device error flag set")
    kstats = kernel_stats(B, args.steps)
    B.pt_timing_enable(False)
    out = {
        "metric": METRIC_INERTIAL, "value": np_ / (ms_step * 1e-3), "unit": "particle-steps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": args.dtype,
        "data": "synthetic",
        "config": {"workload": desc + f", {args.dtype} coefficients, inertial particles "
                   "(tau = 2 dt, launched at 2x the fluid velocity), sort every step, frozen "
                   "field", "grid": n, "particles": np_, "dt": dt, "tau": tau},
        "kernels": kstats,
        "roofline": roofline(kstats, n, np_, cb, args.config + "_inertial", args.dtype, clustered),
    }
    if args.dtype != "f64":
        d = B.pt_tiled_deferred(B.PT_OP_INERTIAL, g, pt._code(cdt), np_, ws)
        out["deferred_particles"] = d
        out["deferred_fraction"] = d / np_
    if not args.no_cpu_baseline:
        import numpy as np

        import oracle
        log("[bench] timing the FP64 oracle on a bounded sample")
        ns, nps = 512, 2 ** 22
        f = synth.spectral_field_torch(ns, ns // 3, seed=0, device=dev).double().cpu().numpy()
        og = oracle.Grid(ns)
        p0 = (synth.clustered_particles_np(nps) if clustered
              else synth.uniform_particles_np(nps, seed=1))
        dts = synth.cfl_dt(np.abs(f).max(), ns)
        co = oracle.spline_coeffs(f)
        v0 = 2.0 * oracle.interp(og, co, p0)
        t0 = time.perf_counter()
        ps, perm, _ = oracle.sort_particles(og, p0, 32, 32)
        oracle.inertial_step(og, co, ps, v0[:, perm], dts, 2.0 * dts)
        t = (time.perf_counter() - t0) * np_ / nps
        out["cpu_baseline"] = {"value": np_ / t, "unit": "particle-steps/s",
                               "cores": oracle.num_threads(), "kind": "oracle",
                               "sample": f"FP64 oracle: sort + inertial step of {nps} particles "
                                         f"on a {ns}^3 grid (x{np_ / nps:.0f})",
                               "ms_per_step_est": 1e3 * t}
    print(json.dumps(out), flush=True)


def run_c5(args, torch, pt, B, synth, n, np_, kmax, desc, cdt, cb):
    """2048^3 grid, 256M uniform particles: per step the cell sort, the
    column-tiled 12-output gather at x_n and the Heun step on the sorted
    particles; the coefficients of the frozen field are computed once before
    (and timed once, reported apart).  The gather and the step are one pass
    (pt_rk2_step_grad: the 12 outputs at x_n and the step) unless --no-save,
    which runs pt_interp_sorted and pt_rk2_step_out."""
    dev = torch.device("cuda:0")
    g = pt.Grid(n)
    field = synth.spectral_field_torch_chunked(n, kmax, seed=0, device=dev)
    dt = synth.cfl_dt(max(float(field.max()), -float(field.min())), n)
    coeff = torch.empty(g.padded_shape, dtype=cdt, device=dev)
    ws_sp = pt.workspace(B.PT_OP_SPLINE, g, 0, cdt, dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    B.pt_spline_coeffs(g, field, coeff, ws_sp)
    torch.cuda.synchronize()
    solve_ms = 1e3 * (time.perf_counter() - t0)
    del field, ws_sp
    torch.cuda.empty_cache()
    pos = synth.uniform_particles_torch(np_, seed=1, device=dev)
    pos_n = torch.empty_like(pos)
    perm = torch.empty(np_, dtype=torch.int32, device=dev)
    ids = torch.arange(np_, dtype=torch.int32, device=dev)
    fused = args.dtype != "f64" and not args.no_save
    out12 = torch.empty((12, np_), dtype=B.value_dtype(coeff), device=dev)
    if not fused:
        ws_i = pt.workspace(B.PT_OP_INTERP_SORTED, g, np_, cdt, dev)
    ws_s = pt.workspace(B.PT_OP_SORT, g, np_, cdt, dev)
    ws_f = pt.workspace(B.PT_OP_RK2, g, np_, cdt, dev)
    torch.cuda.synchronize()
    log(f"[bench] c5 inputs ready: solve {solve_ms:.1f} ms, "
        f"mem={torch.cuda.memory_allocated() / 2**30:.1f} GiB")

    def step():
        B.pt_sort_particles(g, pos, pos_n, perm, ids, None, ws_s)
        if fused:
            B.pt_rk2_step_grad(g, coeff, dt, pos_n, pos, out12, ws_f)
        else:
            B.pt_interp_sorted(g, coeff, pos_n, out12, ws_i)
            B.pt_rk2_step_out(g, coeff, dt, pos_n, pos, B.PT_SORTED, ws_f)

    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log(f"[bench] warmup step {i + 1}/{args.warmup} done")
    for k in KERNELS:
        B.pt_timing_read(k)
    B.pt_timing_enable(True)
    t0 = time.perf_counter()
    for i in range(args.steps):
        step()
        torch.cuda.synchronize()
        log(f"[bench] timed step {i + 1}/{args.steps} done")
    ms_step = 1e3 * (time.perf_counter() - t0) / args.steps
    if B.pt_last_device_error() != 0:
        raise RuntimeError("device error flag set")
    kstats = kernel_stats(B, args.steps)
    B.pt_timing_enable(False)
    out = {
        "metric": METRIC_C5, "value": np_ / (ms_step * 1e-3), "unit": "particle-steps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": args.dtype,
        "data": "synthetic",
        "config": {"workload": desc + f", {args.dtype} coefficients of a frozen field, per "
                   "step: cell sort, 12-output gather (u,v,w and 9 gradients), Heun step"
                   + (" (the gather fused into the step)" if fused else ""),
                   "grid": n, "particles": np_, "dt": dt, "solve_ms_once": solve_ms},
        "kernels": kstats,
        "roofline": roofline(kstats, n, np_, cb, "c5", args.dtype, False),
    }
    for kname in ("tile_interp_grad", "tile_rk2_fwd_grad"):
        if kname not in kstats:
            continue
        kb = launch_bytes(kname, n, np_, cb, 1)
        k_ms = kstats[kname]["avg_launch_ms"]
        out["grad_gather"] = {"kernel": kname, "ms": k_ms,
                              "interpolations_per_s": np_ / (k_ms * 1e-3),
                              "algorithmic_bytes": kb,
                              "hbm_frac": kb / (k_ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
    if not args.no_cpu_baseline:
        import numpy as np

        import oracle
        log("[bench] timing the FP64 oracle on a bounded sample")
        ns, nps = 512, 2 ** 22
        f = synth.spectral_field_torch(ns, ns // 3, seed=0, device=dev).double().cpu().numpy()
        og = oracle.Grid(ns)
        p0 = synth.uniform_particles_np(nps, seed=1)
        dts = synth.cfl_dt(np.abs(f).max(), ns)
        co = oracle.spline_coeffs(f)
        t0 = time.perf_counter()
        ps, _, _ = oracle.sort_particles(og, p0, 32, 32)
        oracle.interp(og, co, ps, n_out=12)
        oracle.rk2_step(og, co, ps, dts)
        t = (time.perf_counter() - t0) * np_ / nps
        out["cpu_baseline"] = {"value": np_ / t, "unit": "particle-steps/s",
                               "cores": oracle.num_threads(), "kind": "oracle",
                               "sample": f"FP64 oracle: sort + 12-output interpolation + Heun "
                                         f"step of {nps} particles on a {ns}^3 grid "
                                         f"(x{np_ / nps:.0f})",
                               "ms_per_step_est": 1e3 * t}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
