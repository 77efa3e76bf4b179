"""Throughput of the LES substep on one MI355X.

A step is one full RK3 time step of the hot path: the device-side time-step reduction
and three substeps (predictor, CN-z Helmholtz solves, Poisson solve, projection, flow-rate
forcing, wall model, dynamic eddy viscosity), replayed from a hipGraph.  The metric is
grid points x substeps per second (Mpts.substeps/s).

Default workload: turbulent channel 256 x 128 x 96 (x, y periodic; z wall-bounded, tanh
stretching beta = 1.5), Lx = 2 pi, Ly = pi, Lz = 2, FP64, Re_b = 40000 (nu = 5e-5 with
U_b = 1, h = 1), dynamic Smagorinsky, log-law wall model at the first off-wall cell,
Crank-Nicolson in z, constant flow rate; initial field laminar Poiseuille plus 10 %
seeded uniform noise (synthetic).

Printed: one JSON line with the throughput, the roofline of the dominant kernel (HIP
events on the library's stream, algorithmic bytes per launch from the library) and the
CPU oracle timed on a bounded sample of the same workload.
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
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="c2", choices=sorted(CONFIGS))
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-learned", action="store_true")
    return ap.parse_args()


def make_solver(cfgd):
    from paper_2411_09364_amd import les
    cfg = les.make_config(cfgd["nx"], cfgd["ny"], cfgd["nz"], cfgd["lx"], cfgd["ly"], cfgd["lz"],
                          zbc=cfgd["zbc"], beta=cfgd["beta"], nu=cfgd["nu"], sgs=cfgd["sgs"], cs=cfgd["cs"],
                          implicit_z=cfgd["implicit_z"], precision=cfgd["precision"], ubulk=cfgd["ubulk"])
    return les, les.Solver(cfg)


def initial_fields(cfgd, zc):
    from synth import isotropic_field, channel_field
    if cfgd["init"] == "iso":
        return isotropic_field(cfgd["nx"], seed=cfgd["seed"], k0=4.0)
    return channel_field(cfgd["nx"], cfgd["ny"], cfgd["nz"], zc, seed=cfgd["seed"])


def cpu_baseline(cfgd, budget_s):
    """The CPU oracle as it stands, one thread, on the same workload: substeps from the
    same seeded initial field until about budget_s seconds have been spent (at least one)."""
    try:
        from threadpoolctl import threadpool_limits
        limiter = threadpool_limits(limits=1)
    except Exception:
        limiter = None
    import oracle
    from oracle import substep as S
    case = oracle.Case(cfgd["nx"], cfgd["ny"], cfgd["nz"], cfgd["lx"], cfgd["ly"], cfgd["lz"], zbc=cfgd["zbc"],
                       beta=cfgd["beta"], nu=cfgd["nu"], sgs=cfgd["sgs"], cs=cfgd["cs"],
                       implicit_z=bool(cfgd["implicit_z"]), ubulk=cfgd["ubulk"])
    g = oracle.Grid(case)
    u, v, w = initial_fields(cfgd, g.zc)
    st = S.initial_state(case, g, u, v, w)
    dt = S.time_step(case, g, st, cfl=0.5)
    t0 = time.perf_counter()
    n = 0
    while True:
        st = S.substep(case, g, st, n % 3, dt)
        n += 1
        if time.perf_counter() - t0 >= budget_s or n >= 30:
            break
    el = time.perf_counter() - t0
    if limiter is not None:
        limiter.unregister() if hasattr(limiter, "unregister") else None
    cells = cfgd["nx"] * cfgd["ny"] * cfgd["nz"]
    return {"value": cells * n / el / 1e6, "unit": "Mpts·substeps/s", "cores": 1, "kind": "oracle",
            "sample": f"{n} oracle substep(s) of the full {cfgd['nx']}x{cfgd['ny']}x{cfgd['nz']} workload "
                      f"in {el:.1f} s, numpy float64, 1 thread"}


def learned_closure(les, torch, cfgd, solver, steps, warmup, use_graph):
    """Same workload with the learned closure: the network is trained on the GPU from
    dynamic-model pairs sampled from the plain solver's current state (400 Adam steps on
    2^16 samples), bound to a second context started from the same initial field, and the
    same step loop is timed."""
    import numpy as np
    sys.path.insert(0, ROOT)
    xr, yr = solver.mlp_sample(7, 1 << 16)
    xn = xr.cpu().numpy().astype(np.float64)
    lo, hi = xn.min(axis=0), xn.max(axis=0)
    pad = 0.25 * (hi - lo) + 1e-12
    lo, hi = lo - pad, hi + pad
    x = torch.empty_like(xr)
    les.les_mlp_normalize(solver.stream.cuda_stream, xr.data_ptr(), xr.shape[0], lo, hi, x.data_ptr())
    rng = np.random.Generator(np.random.PCG64(5))
    init = []
    for shape in ((64, 7), (64,), (64, 64), (64,), (1, 64), (1,)):
        if len(shape) == 2:
            lim = np.sqrt(6.0 / shape[1]) * 0.5
            init.append(rng.uniform(-lim, lim, size=shape).ravel())
        else:
            init.append(np.zeros(shape))
    mlp = les.Mlp(np.concatenate(init), stream=solver.stream)
    t0 = time.perf_counter()
    for it in range(400):
        loss = mlp.train_step(x, yr, 3e-3 if it < 300 else 1e-3)
    solver.synchronize()
    train_s = time.perf_counter() - t0
    cfg = les.make_config(cfgd["nx"], cfgd["ny"], cfgd["nz"], cfgd["lx"], cfgd["ly"], cfgd["lz"], zbc=cfgd["zbc"],
                          beta=cfgd["beta"], nu=cfgd["nu"], sgs=les.SGS_MLP, cs=cfgd["cs"],
                          implicit_z=cfgd["implicit_z"], precision=cfgd["precision"], ubulk=cfgd["ubulk"])
    s2 = les.Solver(cfg)
    zf, zc = s2.zgrid()
    u, v, w = initial_fields(cfgd, zc)
    s2.set_state(u, v, w)
    s2.mlp_bind(mlp, lo, hi)
    s2.nut()
    ctx = s2.ctx

    def step(graph):
        les.les_dt(ctx, 0.5, sync=False)
        les.les_step(ctx, graph)

    for _ in range(warmup):
        step(use_graph)
    s2.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step(use_graph)
    s2.synchronize()
    el = time.perf_counter() - t0
    les.les_timing(ctx, True)
    step(False)
    les.les_timing(ctx, False)
    rep = les.les_timing_report(ctx)
    d, _ = s2.diag()
    cells = cfgd["nx"] * cfgd["ny"] * cfgd["nz"]
    out = {"value": round(cells * 3 * steps / el / 1e6, 3), "unit": "Mpts·substeps/s",
           "ms_per_step": round(el / steps * 1e3, 4), "train_loss": float(loss.item()),
           "train_seconds": round(train_s, 3), "fallback_points_last_eval": int(d.mlp_flagged),
           "nut_kernel_us": {k: round(1e3 * v["ms"] / v["count"], 2) for k, v in rep.items()
                             if k.startswith("mlp") or k.startswith("dsm")}}
    s2.close()
    return out


def traffic_entry(kernel, launches_bytes):
    """Counter-derived HBM traffic for the dominant kernel, if a summary for the current
    kernel source exists under profiles/ (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        data = json.load(open(path))
        ent = data.get(kernel)
        if not ent:
            return None
        src = os.path.join(ROOT, "paper_2411_09364_amd", "csrc", ent["source"])
        digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
        if digest != ent["sha256"]:
            return None
        return ent["bytes_per_launch"]
    except Exception:
        return None


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU path is not "
              f"built in this library", file=sys.stderr)
        sys.exit(2)
    import torch
    torch.cuda.set_device(0)
    cfgd = CONFIGS[args.config]
    les, solver = make_solver(cfgd)
    zf, zc = solver.zgrid()
    u, v, w = initial_fields(cfgd, zc)
    solver.set_state(u, v, w)
    solver.nut()
    ctx = solver.ctx
    use_graph = not args.no_graph
    cells = cfgd["nx"] * cfgd["ny"] * cfgd["nz"]

    def step(graph):
        les.les_dt(ctx, 0.5, sync=False)
        les.les_step(ctx, graph)

    for _ in range(args.warmup):
        step(use_graph)
    solver.synchronize()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(use_graph)
    solver.synchronize()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms_per_step = el / args.steps * 1e3
    value = cells * 3 * args.steps / el / 1e6

    # per-kernel pass: same steps without the graph, every launch bracketed by HIP events
    ksteps = max(1, min(args.steps, 10))
    les.les_timing(ctx, True)
    for _ in range(ksteps):
        step(False)
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
    traffic = traffic_entry(dom, per_launch)
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
                   "substeps_per_step": 3, "graph": use_graph, "closure": "dynamic Smagorinsky"
                   if cfgd["sgs"] == 3 else "Smagorinsky"},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "alg_bytes_per_launch": per_launch, "avg_launch_us": round(1e3 * d["ms"] / d["count"], 3)},
        "kernels": kernels,
        "state_check": {"max_div": diag.max_div, "ubulk": diag.ubulk, "nonfinite": int(diag.nonfinite)},
    }
    if not args.no_learned and cfgd["sgs"] == 3:
        out["learned_closure"] = learned_closure(les, torch, cfgd, solver, args.steps, args.warmup, use_graph)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfgd, args.cpu_seconds)
    solver.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
