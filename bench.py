"""Throughput of the LES substep on one MI355X.

A step is one full RK3 time step of the hot path: the device-side time-step reduction
and three substeps (predictor, CN-z Helmholtz solves, Poisson solve, projection, flow-rate
forcing, wall model, eddy viscosity), replayed from a hipGraph.  The metric is grid
points x substeps per second (Mpts.substeps/s), for the plain method (dynamic
Smagorinsky) and for the learned closure on the same grid.

Default workload (--config c4): turbulent channel 512 x 256 x 128 (x, y periodic; z
wall-bounded, tanh stretching beta = 1.5), Lx = 2 pi, Ly = pi, Lz = 2, FP64, Re_b = 40000
(nu = 5e-5 with U_b = 1, h = 1), log-law wall model at the first off-wall cell,
Crank-Nicolson in z, constant flow rate; initial field laminar Poiseuille plus 10 % seeded
uniform noise (synthetic), projected onto discretely divergence-free fields.  `value` is
the dynamic-Smagorinsky throughput on developed flow (20000 spin-up steps by default); the
learned closure (trained on the GPU from dynamic-model samples of the same run, checked on
later held-out snapshots) is timed on the same state and reported beside it, with its
coefficient error and an a-posteriori comparison of mean profiles over one flow-through
against the dynamic model and static Smagorinsky with van Driest damping.  Each throughput
is the median of five timed runs of --steps steps.

Printed: one JSON line with the throughput, the roofline of the dominant kernel (HIP
events on the library's stream, algorithmic bytes per launch from the library) and the
CPU oracle timed on a bounded sample of the same workload (in a child process whose
thread count is fixed and measured).
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "Mpts·substeps/s per GPU (plain vs learned closure) + % HBM roofline"

CONFIGS = {
    "c2": dict(name="channel 256x128x96 fp64 DSM+WM CN-z", nx=256, ny=128, nz=96, lx=2 * 3.141592653589793,
               ly=3.141592653589793, lz=2.0, zbc=2, beta=1.5, nu=5e-5, sgs=3, cs=0.17, implicit_z=1,
               precision=0, ubulk=1.0, init="channel", seed=2, dtype="f64"),
    "c1": dict(name="isotropic 32^3 fp64 Smagorinsky explicit", nx=32, ny=32, nz=32, lx=2 * 3.141592653589793,
               ly=2 * 3.141592653589793, lz=2 * 3.141592653589793, zbc=0, beta=0.0, nu=1e-3, sgs=1, cs=0.17,
               implicit_z=0, precision=0, ubulk=0.0, init="iso", seed=1, dtype="f64"),
    "c3": dict(name="channel 1024x512x256 mixed DSM+WM explicit", nx=1024, ny=512, nz=256,
               lx=2 * 3.141592653589793, ly=3.141592653589793, lz=2.0, zbc=2, beta=1.5, nu=1.6e-5, sgs=3,
               cs=0.17, implicit_z=0, precision=1, ubulk=1.0, init="channel", seed=3, dtype="f32/f64"),
    "c4": dict(name="channel 512x256x128 fp64 learned closure vs DSM, WM, CN-z", nx=512, ny=256, nz=128,
               lx=2 * 3.141592653589793, ly=3.141592653589793, lz=2.0, zbc=2, beta=1.5, nu=5e-5, sgs=3,
               cs=0.17, implicit_z=1, precision=0, ubulk=1.0, init="channel", seed=4, dtype="f64"),
    "f1": dict(name="channel 256x128x96 fp64 DSM+WM CN in x, y and z", nx=256, ny=128, nz=96,
               lx=2 * 3.141592653589793, ly=3.141592653589793, lz=2.0, zbc=2, beta=1.5, nu=5e-5, sgs=3, cs=0.17,
               implicit_z=2, precision=0, ubulk=1.0, init="channel", seed=2, dtype="f64"),
    # square duct of Sec. 4.4 (Table duct, 512 x 80 x 80, AR = 1, SM): walls with the wall model on y and z
    # (h_wm = 0.1 h), uniform spacing, Re_b = 40000 (nu = 5e-5), C_s = 0.18 with van Driest damping
    "f2": dict(name="square duct 512x80x80 fp64 Smagorinsky+van Driest, WM on four walls, explicit", nx=512, ny=80,
               nz=80, lx=12.8, ly=2.0, lz=2.0, zbc=2, beta=0.0, nu=5e-5, sgs=2, cs=0.18, implicit_z=0, precision=0,
               ubulk=1.0, h_wm=0.1, ybc=1, init="duct", seed=7, dtype="f64"),
    # the same duct with the dynamic model (Table duct, DSM rows): coefficients along x lines
    "f2d": dict(name="square duct 512x80x80 fp64 dynamic Smagorinsky, WM on four walls, explicit", nx=512, ny=80,
                nz=80, lx=12.8, ly=2.0, lz=2.0, zbc=2, beta=0.0, nu=5e-5, sgs=3, cs=0.18, implicit_z=0, precision=0,
                ubulk=1.0, h_wm=0.1, ybc=1, init="duct", seed=7, dtype="f64"),
    "c5": dict(name="64 isotropic boxes 32^3/48^3/64^3/96^3 fp32 DSM explicit, batched", nbox=64, seed=5,
               dtype="f32"),
}

def note(msg):
    """Progress line on stderr (the JSON result is the only line on stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="c4", choices=sorted(CONFIGS))
    ap.add_argument("--runs", type=int, default=5, help="timed runs of --steps steps; the median is reported")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--compare-steps", type=int, default=100, help="c3: steps of the mixed vs FP64 comparison")
    ap.add_argument("--spinup", type=int, default=20000, help="c4: dynamic-model steps before sampling")
    ap.add_argument("--snapshots", type=int, default=20, help="c4: training snapshots")
    ap.add_argument("--per-snapshot", type=int, default=1 << 19, help="c4: samples per snapshot")
    ap.add_argument("--epochs", type=int, default=20, help="c4: training epochs")
    ap.add_argument("--aposteriori", type=float, default=1.0,
                    help="c4: flow-through times of the a-posteriori comparison (0: skipped)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain device copy of known size (calibration of HBM counters)")
    ap.add_argument("--cpu-leg", default=None, help=argparse.SUPPRESS)     # child process of cpu_baseline
    ap.add_argument("--fft-workers", type=int, default=0, help=argparse.SUPPRESS)
    return ap.parse_args()


def make_solver(cfgd):
    from paper_2411_09364_amd import les
    cfg = les.make_config(cfgd["nx"], cfgd["ny"], cfgd["nz"], cfgd["lx"], cfgd["ly"], cfgd["lz"],
                          zbc=cfgd["zbc"], beta=cfgd["beta"], nu=cfgd["nu"], sgs=cfgd["sgs"], cs=cfgd["cs"],
                          implicit_z=cfgd["implicit_z"], precision=cfgd["precision"], ubulk=cfgd["ubulk"],
                          h_wm=cfgd.get("h_wm", 0.0), ybc=cfgd.get("ybc", 0))
    return les, les.Solver(cfg)


def initial_fields(cfgd, zc):
    from synth import isotropic_field, channel_field, duct_field
    if cfgd["init"] == "iso":
        return isotropic_field(cfgd["nx"], seed=cfgd["seed"], k0=4.0)
    if cfgd["init"] == "duct":
        return duct_field(cfgd["nx"], cfgd["ny"], cfgd["nz"], zc, cfgd["ly"], cfgd["lz"], seed=cfgd["seed"])
    return channel_field(cfgd["nx"], cfgd["ny"], cfgd["nz"], zc, seed=cfgd["seed"])


def cpu_leg(key, budget_s, fft_workers):
    """Child-process body of cpu_baseline: oracle substeps of workload `key` from its seeded
    initial state until about budget_s seconds have been spent (at least one), timed by the
    wall clock and by this process's CPU time.  With fft_workers > 0 the oracle's numpy FFT
    calls are routed to scipy.fft with that many workers (same transforms, threaded)."""
    import numpy as np
    if fft_workers > 0:
        import scipy.fft as sf
        for name in ("fft", "ifft", "fft2", "ifft2", "fftn", "ifftn"):
            def routed(*a, _f=getattr(sf, name), **kw):
                return _f(*a, workers=fft_workers, **kw)
            setattr(np.fft, name, routed)
    import oracle
    from oracle import substep as S
    cfgd = CONFIGS[key]
    case = oracle.Case(cfgd["nx"], cfgd["ny"], cfgd["nz"], cfgd["lx"], cfgd["ly"], cfgd["lz"], zbc=cfgd["zbc"],
                       beta=cfgd["beta"], nu=cfgd["nu"], sgs=cfgd["sgs"], cs=cfgd["cs"],
                       implicit_z=cfgd["implicit_z"] == 1, implicit_3d=cfgd["implicit_z"] == 2,
                       ubulk=cfgd["ubulk"], h_wm=cfgd.get("h_wm", 0.0), ybc=cfgd.get("ybc", 0))
    g = oracle.Grid(case)
    u, v, w = S.initial_projection(case, g, *initial_fields(cfgd, g.zc))
    st = S.initial_state(case, g, u, v, w)
    dt = S.time_step(case, g, st, cfl=0.5)
    del u, v, w
    t0, c0 = time.perf_counter(), time.process_time()
    n = 0
    while True:
        st = S.substep(case, g, st, n % 3, dt)
        n += 1
        if time.perf_counter() - t0 >= budget_s or n >= 30:
            break
    el, cpu = time.perf_counter() - t0, time.process_time() - c0
    cells = cfgd["nx"] * cfgd["ny"] * cfgd["nz"]
    return {"substeps": n, "seconds": el, "cpu_seconds": cpu, "value": cells * n / el / 1e6}


def cpu_baseline(key, budget_s, fft_workers=0):
    """The CPU oracle as it stands on the same workload, in a child process started with one
    thread for OpenMP and BLAS (numpy's elementwise work and FFTs are single-threaded), or
    with its FFTs on fft_workers scipy threads.  `cores` is what the child used: its CPU time
    over its wall time, rounded up."""
    import math
    import subprocess
    env = dict(os.environ)
    threads = max(1, fft_workers)
    for var in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS", "BLIS_NUM_THREADS"):
        env[var] = "1"
    cmd = [sys.executable, os.path.abspath(__file__), "--cpu-leg", key, "--cpu-seconds", str(budget_s),
           "--fft-workers", str(fft_workers)]
    r = subprocess.run(cmd, env=env, capture_output=True, text=True, timeout=max(600.0, 20 * budget_s))
    if r.returncode != 0:
        raise RuntimeError(f"oracle timing failed: {r.stderr[-2000:]}")
    res = json.loads(r.stdout.strip().splitlines()[-1])
    cfgd = CONFIGS[key]
    used = res["cpu_seconds"] / res["seconds"]
    cores = max(1, math.ceil(used - 0.05))
    fft = f", FFTs on {fft_workers} scipy.fft workers" if fft_workers else ""
    return {"value": res["value"], "unit": "Mpts·substeps/s", "cores": cores, "kind": "oracle",
            "sample": f"{res['substeps']} oracle substep(s) of the full {cfgd['nx']}x{cfgd['ny']}x{cfgd['nz']} "
                      f"workload in {res['seconds']:.1f} s, numpy float64{fft} (child process, "
                      f"OMP/BLAS threads 1; CPU time / wall time {used:.2f}; {os.cpu_count()} host threads)",
            "threads_requested": threads, "cpu_utilisation": round(used, 3)}


def initial_params(seed):
    """Seeded initial weights of the 7-64-64-1 network (uniform, half the Glorot limit;
    zero biases), flattened in the library's parameter order."""
    import numpy as np
    rng = np.random.Generator(np.random.PCG64(seed))
    init = []
    for shape in ((64, 7), (64,), (64, 64), (64,), (1, 64), (1,)):
        if len(shape) == 2:
            lim = np.sqrt(6.0 / shape[1]) * 0.5
            init.append(rng.uniform(-lim, lim, size=shape).ravel())
        else:
            init.append(np.zeros(shape))
    return np.concatenate(init)


def feature_range(torch, xr):
    """Scaling range of the raw features: the sample min/max widened by a quarter of the
    span on each side (inputs beyond it, with the 5 % margin, fall back to the dynamic
    model), and by at least 1e-5 of the value's size: the samples are float32, so an input
    that is constant over the grid (Delta on a uniform grid) differs from the kernels' FP64
    value by float32 rounding."""
    import numpy as np
    lo = xr.min(dim=0).values.double().cpu().numpy()
    hi = xr.max(dim=0).values.double().cpu().numpy()
    pad = 0.25 * (hi - lo) + 1e-5 * np.maximum(1.0, np.maximum(np.abs(lo), np.abs(hi)))
    return lo - pad, hi + pad


def run_steps(les, s, n, use_graph=True):
    for _ in range(n):
        les.les_dt(s.ctx, 0.5, sync=False)
        les.les_step(s.ctx, use_graph)


def timed_runs(les, s, args, use_graph):
    """--runs timed runs of --steps steps each (after --warmup untimed steps), each bracketed
    by stream synchronisation; returns (median seconds per run, all run seconds)."""
    import statistics
    import torch
    run_steps(les, s, args.warmup, use_graph)
    s.synchronize()
    torch.cuda.synchronize()
    runs = []
    for _ in range(max(1, args.runs)):
        t0 = time.perf_counter()
        run_steps(les, s, args.steps, use_graph)
        s.synchronize()
        torch.cuda.synchronize()
        runs.append(time.perf_counter() - t0)
    return statistics.median(runs), runs


def copy_state(torch, dst, src):
    """Device copy of u, v, w, p from one context's fields into another's."""
    src.synchronize()
    with torch.cuda.stream(dst.stream):
        for a, b in ((dst.u, src.u), (dst.v, src.v), (dst.w, src.w), (dst.p, src.p)):
            a.copy_(b)
    dst.synchronize()


def substep_roofline(value, cfgd):
    """Whole-substep HBM fraction: the minimal-sweep bytes per point and substep (25 words
    with explicit viscous terms, 34 with Crank-Nicolson in z or in all directions: the
    Helmholtz solves read and write each component once; 8-byte words in FP64, 4-byte in the
    mixed mode) times the measured points*substeps/s, against 8 TB/s."""
    words = 34 if cfgd["implicit_z"] else 25
    wb = 4 if cfgd["precision"] == 1 else 8
    gbps = value * 1e6 * words * wb / 1e9
    return {"bound": "hbm", "alg_bytes_per_point": words * wb, "achieved": round(gbps, 2), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(gbps / HBM_PEAK_GBS, 4)}


# Algorithmic FP64 (or FP32 in the mixed mode) flops per cell of the fused dynamic-model kernel,
# counting an add or multiply as 1, an FMA as 2, a square root as 1: strain and |S| at the
# centre 104; the 15 per-cell quantities (centre velocities, their products, |S| S_ij) 18; the
# separable 27-point test filter of 18 fields (those 15 and the 3 staggered velocities) 270;
# test-level strain and |S~| 104; L_ij 12; M_ij 20; the weighted L:M and M:M sums 24.
DSM_FLOPS_PER_CELL = 552
# MI355X vector peaks (256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz, FMA = 2 flops; FP32 packed 2x)
VALU_PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3}


def kernel_report(les, ctx, nsteps, workload, cells=None, fp64=True):
    """Per-kernel HIP-event timing over nsteps un-captured steps; returns (kernels, dominant).
    The dynamic-model kernel is bound by its FP64 (FP32) vector arithmetic, not by HBM: when it
    dominates, the roofline is taken against the vector peak with its algorithmic flops, and
    its HBM figures are kept alongside."""
    les.les_timing(ctx, True)
    for _ in range(nsteps):
        les.les_dt(ctx, 0.5, sync=False)
        les.les_step(ctx, False)
    les.les_timing(ctx, False)
    rep = les.les_timing_report(ctx)
    kernels = {k: {"launches": v["count"], "avg_us": 1e3 * v["ms"] / v["count"],
                   "GBps": (v["bytes"] / (v["ms"] * 1e-3) / 1e9) if v["ms"] > 0 and v["bytes"] > 0 else None,
                   "share": 0.0} for k, v in rep.items()}
    tot_ms = sum(v["ms"] for v in rep.values())
    for k, v in rep.items():
        kernels[k]["share"] = v["ms"] / tot_ms if tot_ms > 0 else 0.0
    dom = max((k for k in rep if rep[k]["bytes"] > 0), key=lambda k: rep[k]["ms"])
    d = rep[dom]
    achieved = d["bytes"] / (d["ms"] * 1e-3) / 1e9
    per_launch = d["bytes"] / d["count"]
    roof = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic_entry(dom, per_launch, workload),
            "alg_bytes_per_launch": per_launch, "avg_launch_us": round(1e3 * d["ms"] / d["count"], 3)}
    if dom == "dsm_fused" and cells is not None:
        sec = d["ms"] * 1e-3 / d["count"]
        tflops = cells * DSM_FLOPS_PER_CELL / sec / 1e12
        peak = VALU_PEAK_TFLOPS["f64" if fp64 else "f32"]
        hbm = {"achieved": roof["achieved"], "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": roof["frac"]}
        roof.update({"bound": "alu", "achieved": round(tflops, 3), "peak": peak, "unit": "TFLOP/s",
                     "frac": round(tflops / peak, 4), "alg_flops_per_cell": DSM_FLOPS_PER_CELL,
                     "alg_flops_per_launch": cells * DSM_FLOPS_PER_CELL, "hbm": hbm})
    return kernels, roof


def statistics_report(les, ctx, nsamples=20):
    """Per-sample cost of the long-run statistics (plane sums of u, v, w, p and nu_t of the
    current state added to the running sums), timed with HIP events like the kernels."""
    les.les_stats_reset(ctx)
    les.les_timing(ctx, True)
    for _ in range(nsamples):
        les.les_stats_sample(ctx)
    les.les_timing(ctx, False)
    rep = les.les_timing_report(ctx)
    les.les_stats_reset(ctx)
    p, f = rep["stats_partial"], rep["stats_final"]
    wall_ms = rep["stats_wall"]["ms"] if "stats_wall" in rep else 0.0   # ducts: the four walls' stresses
    gbps = p["bytes"] / (p["ms"] * 1e-3) / 1e9
    return {"sample_us": round(1e3 * (p["ms"] + f["ms"] + wall_ms) / nsamples, 3),
            "partial_us": round(1e3 * p["ms"] / p["count"], 3), "final_us": round(1e3 * f["ms"] / f["count"], 3),
            "alg_bytes_per_sample": p["bytes"] / p["count"], "GBps": round(gbps, 1),
            "frac": round(gbps / HBM_PEAK_GBS, 4)}


def learned_closure(les, torch, cfgd, solver, args, use_graph):
    """Same workload with the learned closure: the network is trained on the GPU from
    dynamic-model pairs sampled from the plain solver's current state (400 Adam steps on
    2^16 samples), bound to a second context started from the same initial field, and the
    same step loop is timed."""
    import numpy as np
    sys.path.insert(0, ROOT)
    xr, yr = solver.mlp_sample(7, 1 << 16)
    lo, hi = feature_range(torch, xr)
    x = torch.empty_like(xr)
    les.les_mlp_normalize(solver.stream.cuda_stream, xr.data_ptr(), xr.shape[0], lo, hi, x.data_ptr())
    mlp = les.Mlp(initial_params(5), stream=solver.stream)
    t0 = time.perf_counter()
    for it in range(400):
        loss = mlp.train_step(x, yr, 3e-3 if it < 300 else 1e-3)
    solver.synchronize()
    train_s = time.perf_counter() - t0
    _, s2 = make_solver(dict(cfgd, sgs=les.SGS_MLP))
    zf, zc = s2.zgrid()
    u, v, w = initial_fields(cfgd, zc)
    s2.set_state(u, v, w)
    s2.project()
    s2.mlp_bind(mlp, lo, hi)
    s2.nut()
    ctx = s2.ctx

    el, runs = timed_runs(les, s2, args, use_graph)
    steps = args.steps
    les.les_timing(ctx, True)
    run_steps(les, s2, 1, False)
    les.les_timing(ctx, False)
    rep = les.les_timing_report(ctx)
    d, _ = s2.diag()
    cells = cfgd["nx"] * cfgd["ny"] * cfgd["nz"]
    out = {"value": round(cells * 3 * steps / el / 1e6, 3), "unit": "Mpts·substeps/s",
           "ms_per_step": round(el / steps * 1e3, 4), "timed_runs_s": [round(r, 5) for r in runs],
           "train_loss": float(loss.item()),
           "train_seconds": round(train_s, 3), "fallback_points_last_eval": int(d.mlp_flagged),
           "nut_kernel_us": {k: round(1e3 * v["ms"] / v["count"], 2) for k, v in rep.items()
                             if k.startswith(("mlp", "dsm", "vd_duct"))}}
    s2.close()
    return out


def traffic_entry(kernel, launches_bytes, workload):
    """Counter-derived HBM traffic for the dominant kernel, if a summary for the current
    kernel source and this workload exists under profiles/ (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        data = json.load(open(path))
        # entries are keyed by kernel (the default channel) or by "kernel @ workload"
        ent = data.get(kernel)
        if not ent or ent.get("workload", CONFIGS["c2"]["name"]) != workload:
            ent = data.get(f"{kernel} @ {workload}")
        if not ent or ent.get("workload") != workload:
            return None
        src = os.path.join(ROOT, "paper_2411_09364_amd", "csrc", ent["source"])
        digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
        if digest != ent["sha256"]:
            return None
        return ent["bytes_per_launch"]
    except Exception:
        return None


def precision_check(les, torch, cfgd, steps):
    """Mixed precision against FP64 on the same workload.  Both contexts start from the same
    seeded field (rounded to FP32 so both hold identical values) and advance `steps` steps,
    each with its own device-side time step.  Reported: max |D u| and the flow rate of each
    run, the largest difference of the plane-mean streamwise velocity profiles (relative to
    U_b) and of the velocity fields (relative to the FP64 field's largest magnitude)."""
    import numpy as np
    _, s64 = make_solver(dict(cfgd, precision=0))
    _, s32 = make_solver(cfgd)
    zf, zc = s64.zgrid()
    u, v, w = initial_fields(cfgd, zc)
    u, v, w = (a.astype(np.float32).astype(np.float64) for a in (u, v, w))
    for s in (s64, s32):
        s.set_state(u, v, w)
        s.project()
        s.nut()
    del u, v, w
    secs = {}
    for name, s in (("fp64", s64), ("mixed", s32)):
        t0 = time.perf_counter()
        run_steps(les, s, steps)
        s.synchronize()
        secs[name] = round(time.perf_counter() - t0, 3)
    n = cfgd["nz"]
    out = {"steps": steps, "seconds": secs}
    for name, s in (("fp64", s64), ("mixed", s32)):
        d, _ = s.diag()
        out[name] = {"max_div": d.max_div, "ubulk": d.ubulk, "nonfinite": int(d.nonfinite)}
    p64 = s64.u[1:n + 1].mean(dim=(1, 2))
    p32 = s32.u[1:n + 1].double().mean(dim=(1, 2))
    out["mean_u_profile_max_abs_err_over_ub"] = float((p32 - p64).abs().max().item()) / cfgd["ubulk"]
    for name, a64, a32 in (("u", s64.u, s32.u), ("v", s64.v, s32.v), ("w", s64.w, s32.w)):
        ref = float(a64[1:n + 1].abs().max().item())
        out[f"{name}_max_rel_err"] = float((a32[1:n + 1].double() - a64[1:n + 1]).abs().max().item()) / ref
    s64.close()
    s32.close()
    return out


def solver_line(args, torch, cfgd):
    les, solver = make_solver(cfgd)
    zf, zc = solver.zgrid()
    u, v, w = initial_fields(cfgd, zc)
    solver.set_state(u, v, w)
    solver.project()
    solver.nut()
    del u, v, w
    ctx = solver.ctx
    use_graph = not args.no_graph
    cells = cfgd["nx"] * cfgd["ny"] * cfgd["nz"]
    el, runs = timed_runs(les, solver, args, use_graph)
    ms_per_step = el / args.steps * 1e3
    value = cells * 3 * args.steps / el / 1e6
    # per-kernel pass: same steps without the graph, every launch bracketed by HIP events
    kernels, roof = kernel_report(les, ctx, max(1, min(args.steps, 10)), cfgd["name"], cells,
                                  cfgd["precision"] == 0)
    stats = statistics_report(les, ctx)
    diag, status = solver.diag()
    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "Mpts·substeps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": cfgd["dtype"],
        "data": "synthetic",
        "config": {"workload": cfgd["name"], "grid": [cfgd["nx"], cfgd["ny"], cfgd["nz"]],
                   "substeps_per_step": 3, "graph": use_graph,
                   "closure": {3: "dynamic Smagorinsky", 2: "Smagorinsky + van Driest"}.get(cfgd["sgs"], "Smagorinsky")},
        "timed_runs_s": [round(r, 5) for r in runs],
        "roofline": roof,
        "substep_roofline": substep_roofline(value, cfgd),
        "kernels": kernels,
        "state_check": {"max_div": diag.max_div, "ubulk": diag.ubulk, "nonfinite": int(diag.nonfinite)},
        "statistics": stats,
    }
    if not args.no_learned and cfgd["sgs"] == 3 and args.config in ("c2", "f2d"):
        out["learned_closure"] = learned_closure(les, torch, cfgd, solver, args, use_graph)
    solver.close()
    if args.config == "c3":
        out["precision_check"] = precision_check(les, torch, cfgd, args.compare_steps)
    if not args.no_cpu_baseline and args.config in ("c1", "c2", "c3", "f1", "f2", "f2d"):
        out["cpu_baseline"] = cpu_baseline(args.config, args.cpu_seconds)
    return out


# Matrix-core work of the learned closure per cell: 2 (7 * 64 + 64 * 64 + 64) flops (the first
# layer's 7 inputs are padded to 16 on the matrix cores, not counted); dense BF16 peak of the
# MI355X matrix cores in TFLOP/s.
MLP_FLOPS_PER_CELL = 2 * (7 * 64 + 64 * 64 + 64)
MFMA_BF16_PEAK_TFLOPS = 2500.0


def a_posteriori(les, torch, cfgd, args, sd, sm, snap, zc, use_graph):
    """The dynamic model, the learned closure and static Smagorinsky with van Driest damping,
    each from the same state, for --aposteriori flow-through times L_x / U_b (with the time step
    of that state): mean streamwise velocity profiles (statistics every 10 steps, the two halves
    averaged) and C_f; the profile error of Eq. error over [0.1 h, h] of the learned closure and
    of the static model against the dynamic model."""
    import numpy as np
    n = cfgd["nz"]
    _, sv = make_solver(dict(cfgd, sgs=2))
    runs_ap = (("dynamic", sd), ("learned", sm), ("smagorinsky_van_driest", sv))
    for s in (sd, sm, sv):
        with torch.cuda.stream(s.stream):
            for a, b in zip((s.u, s.v, s.w, s.p), snap):
                a.copy_(b)
        s.nut()
    dt_est = sd.dt(0.5)
    nft = int(np.ceil(args.aposteriori * cfgd["lx"] / cfgd["ubulk"] / dt_est))
    note(f"c4: a-posteriori comparison, {nft} steps ({args.aposteriori} flow-through) per closure")
    prof, scal = {}, {}
    for name, s in runs_ap:
        s.stats_reset()
        t0 = time.perf_counter()
        for _ in range(nft // 10):
            run_steps(les, s, 10, use_graph)
            s.stats_sample()
        sc, pr = s.stats(8)
        d, _ = s.diag()
        prof[name] = pr["U"]
        scal[name] = {"c_f": sc["c_f"], "c_f_sigma": sc["c_f_sigma"], "re_tau": sc["re_tau"], "u_tau": sc["u_tau"],
                      "max_div": d.max_div, "nonfinite": int(d.nonfinite),
                      "seconds": round(time.perf_counter() - t0, 2)}
    # profiles of the two halves averaged; z from the wall to the centre (h = lz / 2 = 1)
    h = cfgd["lz"] / 2
    half = n // 2
    zl = np.append(zc[1:half + 1], h)

    def sym(p):
        lower = 0.5 * (p[:half] + p[::-1][:half])
        return np.append(lower, 0.5 * (p[half - 1] + p[half]))

    ref = sym(prof["dynamic"])
    eps = {name: les.les_profile_error(zl, sym(prof[name]), ref, 0.1 * h, h)
           for name in ("learned", "smagorinsky_van_driest")}
    umax_diff = {name: float(np.max(np.abs(sym(prof[name]) - ref))) / cfgd["ubulk"]
                 for name in ("learned", "smagorinsky_van_driest")}
    sv.close()
    return {"steps": nft, "flow_throughs": round(nft * dt_est * cfgd["ubulk"] / cfgd["lx"], 3),
            "reference": "dynamic", "profile_error_eq_error_0.1h_to_h": eps,
            "mean_u_max_abs_diff_over_ub": umax_diff, "closures": scal}


def c4_base(args, cfgd, value, ms_per_step, runs, roof, kernels, use_graph):
    """Fields of the C4 line common to the full run and the dynamic-model-only run."""
    return {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "Mpts·substeps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": cfgd["dtype"],
        "data": "synthetic",
        "config": {"workload": cfgd["name"], "grid": [cfgd["nx"], cfgd["ny"], cfgd["nz"]],
                   "substeps_per_step": 3, "graph": use_graph,
                   "closure": "dynamic Smagorinsky (value)" + ("" if args.no_learned else
                                                               "; learned closure beside it (learned_closure)")},
        "timed_runs_s": [round(r, 5) for r in runs],
        "roofline": roof,
        "substep_roofline": substep_roofline(value, cfgd),
        "kernels": kernels,
    }


def c4_line(args, torch):
    """Dynamic Smagorinsky against the learned closure on the 512 x 256 x 128 channel, on
    developed flow.
    1. Spin-up: the dynamic model from the seeded laminar-plus-noise field for `spinup` steps
       (Courant number 0.5); the friction coefficient of each window of 1000 steps (statistics
       sampled every 20 steps) is recorded, and the spin-up reports the relative change over
       its last two windows (plateau check).
    2. Training pairs (raw features, dynamic c_s of the cell's plane) sampled on the GPU at
       `snapshots` states 50 steps apart, `per_snapshot` cells each.
    3. Held-out pairs: 4 later states (a gap of 500 steps, then 50 steps apart), 2^18 cells each.
    4. Training on the GPU with the library's kernels (Adam, batches of 2^16, `epochs` passes).
    5. A-priori on the held-out pairs: mean-squared error of the network against the dynamic
       coefficient, and of the best constant (the training mean) for comparison.
    6. On the last held-out state: the learned and the dynamic eddy viscosity of the same
       velocity; the learned closure's effective plane coefficient c_eff(k) = c_s(k)
       <nu_t,learned>(k) / <nu_t,dynamic>(k) against c_s(k).
    7. Throughput of both closures from that state (graph-replayed steps, median of --runs
       timed runs each); `value` is the dynamic model's.
    8. Per-kernel HIP-event timing of both; roofline of the dynamic run's dominant kernel,
       matrix-core rate of the learned closure's inference kernel.
    9. A-posteriori: from the same state, the dynamic model, the learned closure and static
       Smagorinsky with van Driest damping each advance one flow-through time L_x / U_b;
       mean streamwise velocity profiles (statistics every 10 steps, the two halves averaged)
       and C_f; the profile error of Eq. error over [0.1 h, h] of the learned closure and of
       the static model against the dynamic model.
    10. The CPU oracle on a bounded sample of the same workload."""
    import numpy as np
    cfgd = CONFIGS["c4"]
    use_graph = not args.no_graph
    les, sd = make_solver(cfgd)
    zf, zc = sd.zgrid()
    u, v, w = initial_fields(cfgd, zc)
    sd.set_state(u, v, w)
    sd.project()
    sd.nut()
    del u, v, w
    n = cfgd["nz"]
    cells = cfgd["nx"] * cfgd["ny"] * cfgd["nz"]
    # 1. spin-up with the friction coefficient per window
    note(f"c4: {args.spinup} dynamic-model steps of spin-up")
    t0 = time.perf_counter()
    window, cf_hist, sim_t = 1000, [], 0.0
    sd.stats_reset()
    done = 0
    while done < args.spinup:
        m = min(window, args.spinup - done)
        for _ in range(m // 20):
            run_steps(les, sd, 20, use_graph)
            sd.stats_sample()
        run_steps(les, sd, m % 20, use_graph)
        done += m
        sc, _ = sd.stats(1)
        d, _ = sd.diag()
        sim_t += m * d.dt
        cf_hist.append([done, round(sim_t, 3), sc["c_f"], sc["re_tau"]])
        sd.stats_reset()
        note(f"c4: spin-up {done} steps, t = {sim_t:.1f}, C_f = {sc['c_f']:.4e}, Re_tau = {sc['re_tau']:.0f}")
    sd.synchronize()
    spin_s = time.perf_counter() - t0
    plateau = (abs(cf_hist[-1][2] - cf_hist[-2][2]) / abs(cf_hist[-1][2])) if len(cf_hist) > 1 else None
    if args.no_learned:
        # the dynamic model alone (no sampling, training or learned closure)
        el, runs = timed_runs(les, sd, args, use_graph)
        value = cells * 3 * args.steps / el / 1e6
        kernels, roof = kernel_report(les, sd.ctx, max(1, min(args.steps, 10)), cfgd["name"], cells,
                                      cfgd["precision"] == 0)
        out = c4_base(args, cfgd, value, el / args.steps * 1e3, runs, roof, kernels, use_graph)
        out["spinup"] = {"steps": args.spinup, "seconds": round(spin_s, 2), "c_f_windows": cf_hist}
        sd.close()
        if not args.no_cpu_baseline:
            out["cpu_baseline"] = cpu_baseline("c4", args.cpu_seconds)
        return out
    # 2. training snapshots, 3. held-out snapshots
    note(f"c4: sampling {args.snapshots} training and 4 held-out snapshots")
    xs, ys = [], []
    for q in range(args.snapshots):
        run_steps(les, sd, 50, use_graph)
        x, y = sd.mlp_sample(1000 + q, args.per_snapshot)
        xs.append(x)
        ys.append(y)
    run_steps(les, sd, 500, use_graph)
    hx, hy = [], []
    for q in range(4):
        run_steps(les, sd, 50, use_graph)
        x, y = sd.mlp_sample(5000 + q, 1 << 18)
        hx.append(x)
        hy.append(y)
    sd.synchronize()
    X = torch.stack(xs, 1).reshape(-1, 7).contiguous()
    Y = torch.stack(ys, 1).reshape(-1).contiguous()
    HX = torch.cat(hx, 0).contiguous()
    HY = torch.cat(hy, 0).contiguous()
    del xs, ys, hx, hy
    torch.cuda.synchronize()
    lo, hi = feature_range(torch, X)
    Xn = torch.empty_like(X)
    les.les_mlp_normalize(sd.stream.cuda_stream, X.data_ptr(), X.shape[0], lo, hi, Xn.data_ptr())
    HXn = torch.empty_like(HX)
    les.les_mlp_normalize(sd.stream.cuda_stream, HX.data_ptr(), HX.shape[0], lo, hi, HXn.data_ptr())
    # 4. training
    mlp = les.Mlp(initial_params(5), stream=sd.stream)
    note("c4: training")
    B = 1 << 16
    nb = X.shape[0] // B
    total = args.epochs * nb
    t0 = time.perf_counter()
    it = 0
    for ep in range(args.epochs):
        for b in range(nb):
            lr = 3e-3 if it < 0.6 * total else (1e-3 if it < 0.9 * total else 3e-4)
            loss = mlp.train_step(Xn[b * B:(b + 1) * B], Y[b * B:(b + 1) * B], lr)
            it += 1
    sd.synchronize()
    train_s = time.perf_counter() - t0
    final_loss = float(loss.item())
    target_var = float(Y.double().var().item())
    ymean = float(Y.double().mean().item())
    # 5. a-priori on the held-out snapshots (the network's output clipped at zero, as in the
    # eddy viscosity)
    pred = mlp.forward(HXn)
    sd.synchronize()
    pred = pred.double().clamp(min=0.0)
    hyd = HY.double()
    mse_net = float(((pred - hyd) ** 2).mean().item())
    mse_const = float(((ymean - hyd) ** 2).mean().item())
    held_var = float(hyd.var().item())
    del X, Xn, Y, HX, HXn, HY, pred, hyd
    cfg_m = les.make_config(cfgd["nx"], cfgd["ny"], cfgd["nz"], cfgd["lx"], cfgd["ly"], cfgd["lz"], zbc=cfgd["zbc"],
                            beta=cfgd["beta"], nu=cfgd["nu"], sgs=les.SGS_MLP, cs=cfgd["cs"],
                            implicit_z=cfgd["implicit_z"], precision=cfgd["precision"], ubulk=cfgd["ubulk"])
    sm = les.Solver(cfg_m)
    sm.mlp_bind(mlp, lo, hi)
    copy_state(torch, sm, sd)
    sd.nut()
    sm.nut()
    sd.synchronize()
    sm.synchronize()
    snap = [t.clone() for t in (sd.u, sd.v, sd.w, sd.p)]
    torch.cuda.synchronize()
    # 6. coefficient error on the same velocity
    nut_d = sd.eddy_viscosity()[1:n + 1]
    nut_m = sm.eddy_viscosity()[1:n + 1]
    cs_d = sd.coefficient()
    md, mm = nut_d.mean(axis=(1, 2)), nut_m.mean(axis=(1, 2))
    ok = md > 0
    ceff = np.where(ok, cs_d * mm / np.where(ok, md, 1.0), 0.0)
    coef_err = float(np.linalg.norm(ceff - cs_d) / max(np.linalg.norm(cs_d), 1e-300))
    nut_plane_err = float(np.linalg.norm(mm - md) / max(np.linalg.norm(md), 1e-300))
    nut_point_err = float(np.sqrt(np.mean((nut_m - nut_d) ** 2)) / max(np.sqrt(np.mean(nut_d ** 2)), 1e-300))
    dm, _ = sm.diag()
    flagged = int(dm.mlp_flagged)
    del nut_d, nut_m
    # 7. throughput
    thr = {}
    for name, s in (("dynamic", sd), ("learned", sm)):
        note(f"c4: timing the {name} closure")
        el, runs = timed_runs(les, s, args, use_graph)
        thr[name] = (cells * 3 * args.steps / el / 1e6, el / args.steps * 1e3, runs)
    # 8. per-kernel timing
    nrep = max(1, min(args.steps, 10))
    kernels, roof = kernel_report(les, sd.ctx, nrep, cfgd["name"], cells, cfgd["precision"] == 0)
    kernels_m, _ = kernel_report(les, sm.ctx, nrep, cfgd["name"] + " learned", cells, cfgd["precision"] == 0)
    mlp_us = kernels_m["mlp_nut"]["avg_us"]
    mlp_tflops = cells * MLP_FLOPS_PER_CELL / (mlp_us * 1e-6) / 1e12
    # 9. a-posteriori over --aposteriori flow-throughs from the same state
    if args.aposteriori <= 0:
        del snap
        ap_out = None
    else:
        ap_out = a_posteriori(les, torch, cfgd, args, sd, sm, snap, zc, use_graph)
        del snap
    value = thr["dynamic"][0]
    out = c4_base(args, cfgd, value, thr["dynamic"][1], thr["dynamic"][2], roof, kernels, use_graph)
    out.update({
        "learned_closure": {
            "value": round(thr["learned"][0], 3), "unit": "Mpts·substeps/s",
            "ms_per_step": round(thr["learned"][1], 4),
            "timed_runs_s": [round(r, 5) for r in thr["learned"][2]],
            "ratio_to_dynamic": round(thr["learned"][0] / value, 4),
            "substep_roofline": substep_roofline(thr["learned"][0], cfgd),
            "mlp_nut": {"bound": "mfma", "avg_launch_us": round(mlp_us, 3),
                        "alg_flops_per_cell": MLP_FLOPS_PER_CELL,
                        "achieved": round(mlp_tflops, 2), "peak": MFMA_BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                        "frac": round(mlp_tflops / MFMA_BF16_PEAK_TFLOPS, 4)},
            "kernels": kernels_m,
            "spinup": {"steps": args.spinup, "seconds": round(spin_s, 2), "window_steps": window,
                       "c_f_windows": cf_hist, "last_window_rel_change": plateau},
            "training": {"snapshots": args.snapshots, "snapshot_spacing_steps": 50, "samples": nb * B,
                         "epochs": args.epochs, "adam_steps": total, "seconds": round(train_s, 2),
                         "final_batch_mse": final_loss, "target_variance": target_var},
            "held_out": {"snapshots": 4, "gap_steps": 500, "samples": 4 << 18, "mse_network": mse_net,
                         "mse_best_constant": mse_const, "target_variance": held_var,
                         "mse_ratio_network_to_constant": mse_net / mse_const if mse_const > 0 else None},
            "coefficient_error": {"plane_coefficient_rel_l2": coef_err, "plane_nut_rel_l2": nut_plane_err,
                                  "pointwise_nut_rel_rms": nut_point_err, "fallback_points": flagged},
            "a_posteriori": ap_out,
        },
    })
    sd.close()
    sm.close()
    if not args.no_cpu_baseline:
        note("c4: CPU oracle, one thread")
        out["cpu_baseline"] = cpu_baseline("c4", args.cpu_seconds)
        workers = min(16, os.cpu_count() or 1)
        note(f"c4: CPU oracle, FFTs on {workers} threads")
        out["cpu_baseline_fft_threads"] = cpu_baseline("c4", args.cpu_seconds, fft_workers=workers)
    return out


def batch_line(args, torch):
    """64 periodic boxes of mixed sizes advanced together: one launch per kernel kind per
    substep for all boxes, per-box device time step, the whole step replayed from a
    hipGraph, tiles chosen by the autotuner first (its time reported separately).  Then the
    ensemble's final state is sampled as learned-closure training data (2^16 pairs per box,
    `training_samples`)."""
    from paper_2411_09364_amd import les
    from synth import box_ensemble, isotropic_field
    cfgd = CONFIGS["c5"]
    two_pi = 2 * 3.141592653589793
    ens = box_ensemble(cfgd["nbox"], seed=cfgd["seed"])
    cfgs = [les.make_config(e["n"], e["n"], e["n"], two_pi, two_pi, two_pi, zbc=0, nu=e["nu"], sgs=3, cs=0.17,
                            implicit_z=0, precision=1) for e in ens]
    # initial fields made discretely divergence-free by the library's projection, one
    # single-box context per box size
    projector, init = {}, []
    for e, cfg in zip(ens, cfgs):
        if e["n"] not in projector:
            projector[e["n"]] = les.Solver(cfg)
        s = projector[e["n"]]
        s.set_state(*isotropic_field(e["n"], seed=e["seed"], k0=e["k0"]))
        s.project()
        init.append(s.fields()[:3])
    for s in projector.values():
        s.close()
    b = les.Batch(cfgs)

    def load():
        for i, (u, v, w) in enumerate(init):
            b.set_state(i, u, v, w)
        b.nut()

    # the autotuner advances the state it times: tune on the initial fields, then reload them
    load()
    b.dt(0.5)
    t0 = time.perf_counter()
    tune = b.autotune(6)
    b.synchronize()
    tune_s = time.perf_counter() - t0
    load()
    use_graph = not args.no_graph
    for _ in range(args.warmup):
        b.step(0.5, use_graph)
    b.synchronize()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        b.step(0.5, use_graph)
    b.synchronize()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    cells = sum(e["n"] ** 3 for e in ens)
    value = cells * 3 * args.steps / el / 1e6
    divs, bad = [], 0
    for i in range(len(ens)):
        d = b.box_dt(i)
        divs.append(d.max_div)
        bad += int(d.nonfinite)
    alg = 25 * 4   # minimal-sweep words per point and substep (explicit), FP32 storage
    achieved = value * 1e6 * alg / 1e9
    # the ensemble as a training-data generator: 2^16 pairs per box from the final state
    npb = 1 << 16
    t0 = time.perf_counter()
    xs, ys = b.mlp_sample(11, npb)
    sample_s = time.perf_counter() - t0
    sampling = {"pairs": int(ys.shape[0]), "pairs_per_box": npb, "seconds": round(sample_s, 4),
                "pairs_per_s": round(ys.shape[0] / sample_s), "finite": bool(torch.isfinite(xs).all().item())}
    del xs, ys
    b.close()
    sizes = {}
    for e in ens:
        sizes[e["n"]] = sizes.get(e["n"], 0) + 1
    return {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "Mpts·substeps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(el / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": cfgd["dtype"],
        "data": "synthetic",
        "config": {"workload": cfgd["name"], "boxes": {str(k): v for k, v in sorted(sizes.items())},
                   "cells": cells, "substeps_per_step": 3, "graph": use_graph},
        "roofline": {"bound": "hbm", "kernel": "whole substep (all kernels, minimal-sweep bytes)",
                     "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None, "alg_bytes_per_point": alg},
        "autotune": {"seconds": round(tune_s, 3), "choice": tune},
        "state_check": {"max_div": max(divs), "nonfinite": bad},
        "training_samples": sampling,
    }


def main():
    args = parse()
    if args.cpu_leg is not None:
        # child process of cpu_baseline: the oracle only, no GPU
        print(json.dumps(cpu_leg(args.cpu_leg, args.cpu_seconds, args.fft_workers)), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU path is not "
              f"built in this library", file=sys.stderr)
        sys.exit(2)
    import torch
    torch.cuda.set_device(0)
    if args.copy_probe:
        # elementwise kernel reading 2^25 doubles and writing 2^25 doubles (256 MiB each way)
        n = 1 << 25
        src = torch.rand(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe": {"kernel": "elementwise mul by 1.0", "read_bytes": 8 * n,
                                         "write_bytes": 8 * n, "launches": 5}}), flush=True)
        return
    if args.config == "c5":
        out = batch_line(args, torch)
    elif args.config == "c4":
        out = c4_line(args, torch)
    else:
        out = solver_line(args, torch, CONFIGS[args.config])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
