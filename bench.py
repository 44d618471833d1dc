"""Benchmark: one fractional-step linear-solve pass at 256^3 (stretched y).

A step is the whole hot path on one batch of synthetic input:
  3 Crank-Nicolson Helmholtz solves (u, v, w in one batched call)
  -> divergence of the intermediate velocity (Poisson right-hand side)
  -> pressure Poisson solve -> projection of the velocity (gradient correction).
Metric: Mcell-solves/s = 4 * nx*ny*nz / t_step / 1e6 (v counted as nx*ny*nz).

Inputs: seeded N(0,1) face velocities low-pass filtered to index radius 16,
wall v = 0, beta = 2 tanh stretching, c = 0.5 nu dt with nu dt / h_min^2 =
0.25 (h_min = the wall cell height).  Inputs are resident in HBM before the
timed region.

Prints ONE JSON line (rank 0).  Only one GPU is used; --gpus > 1 exits.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"fp64_tflops": 78.6, "hbm_gbs": 8000.0}
# peak rate (TFLOP/s) each kernel class's algorithmic flops are priced at in
# the whole-step roofline: FP64 matrix cores, bf16 matrix cores (dense), or
# the vector units (FP64 78.6, FP32 157.3)
CLASS_PEAK = {"xgemm_f64": 78.6, "zgemm_f64": 78.6, "xgemm_split": 2500.0, "zgemm_split": 2500.0,
              "update": 2500.0, "tridiag_f64": 78.6, "tridiag_f32": 157.3, "divergence": 78.6,
              "correct": 78.6, "residual": 78.6}
# HBM bytes per launch measured with rocprofv3 counters on the 256^3 step
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_256cube.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_inputs(n, beta, seed):
    from paper_2406_19920_amd import synth
    u, v, w = synth.filtered_velocity(n, n, n, seed=seed, kmax=16.0)
    return u, v, w


def h_min(ny, beta, ly=1.0):
    j = np.arange(ny + 1)
    if beta == 0:
        yf = ly * j / ny
    else:
        yf = 0.5 * ly * (1 + np.tanh(beta * (2 * j / ny - 1)) / np.tanh(beta))
    return float(np.diff(yf).min())


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_step(n_sample, beta, seed):
    """Seconds for one full step of the oracle (C/OpenMP CG) at n_sample^3."""
    import oracle
    from oracle import OP_P, OP_U, OP_V, OP_W
    g = oracle.Grid(n_sample, n_sample, n_sample, beta=beta)
    c = 0.125 * float(g.dyc.min()) ** 2
    u, v, w = make_inputs(n_sample, beta, seed)
    t0 = time.perf_counter()
    us, _ = oracle.solve(g, OP_U, u, c=c)
    vs, _ = oracle.solve(g, OP_V, v, c=c)
    ws, _ = oracle.solve(g, OP_W, w, c=c)
    b = oracle.divergence(g, us, vs, ws)
    phi, _ = oracle.solve(g, OP_P, b)
    gu, gv, gw = oracle.gradient(g, phi)
    us -= gu; vs -= gv; ws -= gw
    return time.perf_counter() - t0


def cpu_helmholtz_headline(n, beta, u, v, w):
    """Seconds for the headline step's three Helmholtz solves by the oracle
    at the headline size itself (same inputs, same c)."""
    import oracle
    from oracle import OP_U, OP_V, OP_W
    g = oracle.Grid(n, n, n, beta=beta)
    c = 0.125 * float(g.dyc.min()) ** 2
    t0 = time.perf_counter()
    for op, f in ((OP_U, u), (OP_V, v), (OP_W, w)):
        oracle.solve(g, op, f, c=c)
    return time.perf_counter() - t0


def cpu_baseline(n_sample, beta, seed, n_single=64, headline=None):
    """The oracle on the same step at a reduced grid, on all host threads,
    and on one thread at a smaller grid; with headline = (n, u, v, w) also
    the step's three Helmholtz solves at the headline size."""
    import oracle
    dt = cpu_step(n_sample, beta, seed)
    head = None
    if headline is not None:
        nh, u, v, w = headline
        dth = cpu_helmholtz_headline(nh, beta, u, v, w)
        head = {"value": 3 * nh ** 3 / dth / 1e6, "unit": "Mcell-solves/s",
                "sample": f"the three Helmholtz solves of the {nh}^3 step itself (same inputs and c), "
                          f"{dth:.1f} s; the step's Poisson solve at {nh}^3 (CG, thousands of "
                          f"iterations) is left out to bound the run"}
    threads = oracle.num_threads()
    oracle.set_num_threads(1)
    try:
        dt1 = cpu_step(n_single, beta, seed)
    finally:
        oracle.set_num_threads(threads)
    return {"value": 4 * n_sample ** 3 / dt / 1e6, "unit": "Mcell-solves/s",
            "cores": threads, "kind": "oracle",
            "sample": f"one full step (3 Helmholtz + divergence + Poisson + correction) of the "
                      f"same workload at {n_sample}^3 (beta={beta}, same c rule), "
                      f"{dt:.1f} s; the CG iteration count grows with the grid, so this "
                      f"overstates the oracle's rate at 256^3",
            "single_thread": {"value": 4 * n_single ** 3 / dt1 / 1e6, "unit": "Mcell-solves/s",
                              "sample": f"the same step at {n_single}^3 on one thread, {dt1:.1f} s"},
            "headline_size_helmholtz": head,
            "cpu_model": cpu_model(), "nproc": os.cpu_count()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--beta", type=float, default=2.0)
    ap.add_argument("--path", choices=["refined", "fp64", "both"], default="both")
    ap.add_argument("--cpu-sample", type=int, default=160)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra-configs", action="store_true",
                    help="skip the shortened 512x384x384, 64-job batch and serving runs that the "
                         "default run appends under 'configs'")
    ap.add_argument("--config", choices=["c2", "c3", "batch", "serve", "rk3", "small_grids"], default="c2",
                    help="c2: 256^3 step (default); c3: 512x384x384 refined step with a forcing "
                         "shell; batch: 64 mixed-size jobs as one graph; serve: arrival-rate sweep; "
                         "rk3: full Runge-Kutta step with immersed markers at --n^3; small_grids: 128 "
                         "FP64 jobs of 32^3-64^3 as graph lanes and as multi-grid stage launches")
    ap.add_argument("--count", type=int, default=2000, help="serve: requests per rate")
    ap.add_argument("--rates", type=str, default="100,200,500,1000,2000,5000")
    ap.add_argument("--geometries", type=int, default=0,
                    help="serve: draw requests from a pool of this many (n, beta) grids so plans "
                         "are reused (0: every request on a grid of its own)")
    ap.add_argument("--passes", type=int, default=2,
                    help="refinement pass cap of the refined path (0: library default, up to 3 for "
                         "the pressure problem); the 256^3 workload converges in 2, and a cap "
                         "above that only adds launches whose kernels return at once")
    ap.add_argument("--tiles", type=str, default="",
                    help="FP64 transform tile choices 'X,Z' to use instead of autotuning (keeps "
                         "the tuner's trial launches out of counter runs)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES bytes (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this solver is single-GPU "
              "(multi-GPU sharding is a design note, not built)", file=sys.stderr)
        sys.exit(2)

    import torch
    if args.copy_calibration:
        return copy_calibration(args.copy_calibration)
    from paper_2406_19920_amd import ibsolve as ibs

    if args.config == "batch":
        return bench_batch(args)
    if args.config == "serve":
        return bench_serve(args)
    if args.config == "c3":
        return bench_c3(args)
    if args.config == "rk3":
        return bench_rk3(args)
    if args.config == "small_grids":
        from paper_2406_19920_amd import synth
        r = run_batch_modes(args.steps, args.warmup,
                            synth.batch_specs(128, seed=5, sizes=((32, 32, 32), (48, 32, 48), (64, 64, 64))),
                            "128 jobs of 32^3, 48x32x48 and 64^3 (beta ~ U[0,3]), Poisson + 3 Helmholtz "
                            "each, FP64")
        best = r[r["faster"]]
        print(json.dumps({"metric": "Mcell-solves/s, 128 small FP64 jobs (Poisson + 3 Helmholtz)",
                          "value": best["value"], "unit": "Mcell-solves/s", "n_gpus": 1,
                          "steps": args.steps, "warmup": args.warmup, "ms_per_step": best["ms_per_launch"],
                          "higher_is_better": True, "vs_baseline": None, "dtype": "f64",
                          "data": "synthetic", "config": {"workload": r["workload"]}, "forms": r}))
        return

    n, beta = args.n, args.beta
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    log(f"inputs {n}^3 beta={beta}")
    u, v, w = make_inputs(n, beta, seed=2)
    c = 0.125 * h_min(n, beta) ** 2
    ru, rv, rw = (torch.from_numpy(a).to(dev) for a in (u, v, w))
    stream = torch.cuda.current_stream(dev)
    cells = n ** 3

    def run_path(precision):
        kw = {} if precision == ibs.IBS_FP64 else {"max_iter": args.passes}
        S = ibs.Solver(n, n, n, beta=beta, precision=precision, **kw)
        # measured tile shapes for this grid (set-up, outside the timed region)
        tiles = None
        if precision == ibs.IBS_FP64:
            if args.tiles:
                tiles = [int(t) for t in args.tiles.split(",")]
                ibs.ibs_plan_set_tiles(S.plan, tiles)
            else:
                tiles = S.autotune()
        xu, xv, xw = S.empty(1), S.empty(2), S.empty(3)
        b = S.empty(0)
        phi = S.empty(0)

        def step():
            # reports: Helmholtz components in info slots 1..3, Poisson in 0
            S.helmholtz([0, 1, 2], [c, c, c], [ru, rv, rw], [xu, xv, xw], info_slot=1)
            S.divergence(xu, xv, xw, 1.0, b)
            S.poisson(b, phi)
            S.correct(phi, xu, xv, xw, 1.0)

        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        evs[0].record(stream)
        for k in range(args.steps):
            step()
            evs[k + 1].record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        per = np.array([evs[k].elapsed_time(evs[k + 1]) for k in range(args.steps)])
        ms = wall * 1e3 / args.steps
        infos = [S.read_info(q) for q in (1, 2, 3)]
        # live per-kernel timing (HIP events on the launch stream) over the
        # same number of steps
        ibs.ibs_profile(S.plan, True)
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        kern = {}
        for kid, name in enumerate(ibs.PROFILE_KERNELS):
            r = ibs.ibs_profile_read(S.plan, kid)
            if r["launches"]:
                kern[name] = r
        ibs.ibs_profile(S.plan, False)
        pinfo = S.read_info(0)
        S.close()
        return dict(ms=ms, per=per, kern=kern, hinfo=infos, pinfo=pinfo, tiles=tiles)

    def roofline(kern, steps):
        from paper_2406_19920_amd import pmc
        dom_name = max(kern, key=lambda k: kern[k]["ms"])
        d = kern[dom_name]
        avg_ms = d["ms"] / d["launches"]
        traffic = pmc.traffic_for(dom_name, TRAFFIC_FILE) if n == 256 and beta == 2.0 else None
        if dom_name in ("xgemm_f64", "zgemm_f64"):
            achieved = d["flops"] / d["launches"] / (avg_ms * 1e-3) / 1e12
            roof = {"bound": "mfma", "achieved": achieved, "peak": PEAK["fp64_tflops"],
                    "unit": "TFLOP/s"}
        else:
            achieved = d["bytes"] / d["launches"] / (avg_ms * 1e-3) / 1e9
            roof = {"bound": "hbm", "achieved": achieved, "peak": PEAK["hbm_gbs"], "unit": "GB/s"}
        roof["frac"] = roof["achieved"] / roof["peak"]
        roof["traffic"] = traffic
        roof["traffic_unit"] = "bytes per launch (HBM, rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)"
        roof["algorithmic_bytes_per_launch"] = d["bytes"] / d["launches"]
        roof["kernel"] = dom_name
        roof["avg_launch_ms"] = avg_ms
        # whole step: sum over classes of max(flops / peak, bytes / HBM peak),
        # over the measured kernel time of a step
        roof_ms = sum(max(r["flops"] / (CLASS_PEAK.get(k, PEAK["fp64_tflops"]) * 1e12),
                          r["bytes"] / (PEAK["hbm_gbs"] * 1e9)) * 1e3 for k, r in kern.items()) / steps
        kern_ms = sum(r["ms"] for r in kern.values()) / steps
        roof["step_roofline"] = {"roofline_ms": roof_ms, "kernel_ms": kern_ms, "frac": roof_ms / kern_ms}
        breakdown = {k: {"ms_per_step": r["ms"] / steps,
                         "launches_per_step": r["launches"] / steps,
                         "tflops": r["flops"] / (r["ms"] * 1e-3) / 1e12 if r["ms"] else None,
                         "gbs": r["bytes"] / (r["ms"] * 1e-3) / 1e9 if r["ms"] else None}
                     for k, r in kern.items()}
        return roof, breakdown

    results = {}
    paths = ["refined", "fp64"] if args.path == "both" else [args.path]
    for path in paths:
        log(f"path {path}")
        prec = ibs.IBS_REFINED_BF16X3 if path == "refined" else ibs.IBS_FP64
        r = run_path(prec)
        roof, brk = roofline(r["kern"], args.steps)
        results[path] = dict(
            value=4 * cells / (r["ms"] * 1e-3) / 1e6, ms_per_step=r["ms"],
            latency_ms={"p50": float(np.percentile(r["per"], 50)),
                        "p99": float(np.percentile(r["per"], 99))},
            roofline=roof, kernels=brk, tiles=r["tiles"],
            passes={"helmholtz": max(i.iters for i in r["hinfo"]), "poisson": r["pinfo"].iters},
            predicted_rel_err={"helmholtz": max(i.rel_residual for i in r["hinfo"]),
                               "poisson": r["pinfo"].rel_residual} if path == "refined" else None,
            status=[i.status for i in r["hinfo"]] + [r["pinfo"].status],
            pass_cap=None if path == "fp64" else args.passes)
        if any(results[path]["status"]):
            log(f"WARNING: path {path} status {results[path]['status']} (non-zero: not converged)")

    # the other configurations, shortened, in the same run (their own
    # --config modes run them in full)
    configs = None
    if not args.no_extra_configs and n == 256 and beta == 2.0:
        from paper_2406_19920_amd import synth
        configs = {}
        log("config c3")
        c3, c3w = run_c3(5, 1)
        configs["c3"] = {"workload": c3w, "steps": 5, "warmup": 1,
                         "refined": {k: c3["refined"][k] for k in ("value", "ms_per_step", "status", "passes")},
                         "fp64": {k: c3["fp64"][k] for k in ("value", "ms_per_step", "status", "passes")},
                         "unit": "Mcell-solves/s"}
        log("config 3p")
        r3, w3 = run_3p(10, 2)
        configs["triply_periodic"] = {"workload": w3, "steps": 10, "warmup": 2,
                                      "unit": "Mcell-solves/s", **r3}
        log("config xw")
        rx, wx = run_xw(10, 2)
        configs["x_walls"] = {"workload": wx, "steps": 10, "warmup": 2, "unit": "Mcell-solves/s", **rx}
        log("config duct")
        rd, wd = run_xw(10, 2, walls_z=True)
        configs["duct"] = {"workload": wd, "steps": 10, "warmup": 2, "unit": "Mcell-solves/s", **rd}
        log("config stretched duct")
        rs, ws = run_xw(10, 2, walls_z=True, stretch_xz=1.5)
        configs["stretched_duct"] = {"workload": ws, "steps": 10, "warmup": 2, "unit": "Mcell-solves/s", **rs}
        log("config rk3")
        rr, wr = run_rk3(5, 1)
        configs["rk3_step"] = {"workload": wr, "steps": 5, "warmup": 1,
                               "unit": "Mcell-steps/s (cells x full RK3 steps per second)", **rr}
        log("config c4")
        configs["c4"] = run_batch(5, 1)
        configs["c4_fp64_forms"] = run_batch_modes(
            5, 1, synth.batch_specs(64, seed=4),
            "the 64 mixed-size jobs (64^3 to 192x256x192), FP64: graph lanes vs multi-grid stage launches")
        configs["small_grids"] = run_batch_modes(
            10, 2, synth.batch_specs(128, seed=5, sizes=((32, 32, 32), (48, 32, 48), (64, 64, 64))),
            "128 jobs of 32^3, 48x32x48 and 64^3 (beta ~ U[0,3]), Poisson + 3 Helmholtz each, FP64: "
            "graph lanes vs multi-grid stage launches")
        log("config c5")
        rows, nwarm, w5 = run_serve([200.0, 1000.0, 5000.0], 300)
        configs["c5"] = {"workload": w5, "unit": "Mcell-solves/s", "sweep": rows}

    cpu = None
    if not args.no_cpu_baseline:
        log(f"cpu baseline: oracle at {args.cpu_sample}^3")
        cpu = cpu_baseline(args.cpu_sample, beta, seed=2, headline=(n, u, v, w))

    head = results[paths[0]]
    out = {
        "metric": "Mcell-solves/s at 256^3: 3 Helmholtz + 1 Poisson solve per step "
                  "(refined mixed precision to 1e-10; FP64 path alongside); p50/p99 step latency",
        "value": head["value"], "unit": "Mcell-solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": head["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": ("bf16x3 MFMA, f32 accumulate, f64 residual/iterate" if paths[0] == "refined"
                  else "f64"),
        "data": "synthetic",
        "config": {"workload": f"fractional-step solves {n}^3, tanh beta={beta}, periodic x/z, "
                               f"Dirichlet/Neumann walls, c={c:.4e}",
                   "path": paths[0], "grid": [n, n, n]},
        "latency_ms": head["latency_ms"],
        "roofline": head["roofline"],
        "paths": results,
        "cpu_baseline": cpu,
        "configs": configs,
    }
    print(json.dumps(out), flush=True)


def copy_calibration(nbytes):
    """A plain device-to-device copy of nbytes, five times: the reference
    reading for the HBM byte counters."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": src.numel() * 4, "repeats": 5}), flush=True)


def run_batch(steps, warmup, njobs=64):
    """64 independent refined Poisson + 3 Helmholtz jobs of mixed sizes,
    recorded once into one HIP graph and replayed, with the schedule (lane
    count, policy) picked by the library's schedule autotuner at set-up;
    returns a summary."""
    import torch
    from paper_2406_19920_amd import batch, ibsolve as ibs, synth
    specs = synth.batch_specs(njobs, seed=4)
    log("building batch of", len(specs), "jobs")
    B = batch.Batch(specs, precision=ibs.IBS_REFINED_BF16X3, nlanes="auto")
    lanes, policy, tuned_ms = B.schedule
    log("schedule", B.schedule)
    for _ in range(warmup):
        B.launch()
    torch.cuda.synchronize()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    t0 = time.perf_counter()
    evs[0].record()
    for k in range(steps):
        B.launch()
        evs[k + 1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = np.array([evs[k].elapsed_time(evs[k + 1]) for k in range(steps)])
    ms = wall * 1e3 / steps
    status = [j.solver.read_info(q).status for j in B.jobs for q in (0, 1, 2, 3)]
    out = {"value": B.cell_solves / (ms * 1e-3) / 1e6, "unit": "Mcell-solves/s",
           "ms_per_launch": ms, "launches": steps,
           "workload": f"{njobs} jobs, sizes uniform over 64^3, 96x128x96, 128^3, 192x256x192, "
                       "beta ~ U[0,3], seeds 1000+i, refined, one graph launch, schedule autotuned",
           "schedule": {"nlanes": lanes, "policy": ["balanced", "in_order"][policy], "tuned_ms": tuned_ms},
           "cell_solves_per_launch": B.cell_solves,
           "latency_ms": {"p50": float(np.percentile(per, 50)), "p99": float(np.percentile(per, 99))},
           "all_status_ok": all(s == 0 for s in status)}
    B.close()
    return out


def run_batch_modes(steps, warmup, specs, label):
    """The same FP64 jobs as a graph of per-grid launch sequences (schedule
    autotuned) and as a multi-grid batch (one persistent launch per stage
    over all grids): ms per replay and throughput of each, and the form the
    batch's own chooser (mode="auto") keeps."""
    import torch
    from paper_2406_19920_amd import batch, ibsolve as ibs
    out = {"workload": label, "unit": "Mcell-solves/s", "steps": steps, "warmup": warmup}
    for mode in ("graph", "multigrid"):
        log("batch", label, mode)
        B = batch.Batch(specs, precision=ibs.IBS_FP64, nlanes="auto", mode=mode)
        for _ in range(warmup):
            B.launch()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            B.launch()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        status = [j.solver.read_info(q).status for j in B.jobs for q in (0, 1, 2, 3)]
        out[mode] = {"value": B.cell_solves / (ms * 1e-3) / 1e6, "ms_per_launch": ms,
                     "kernel_launches_per_replay": 5 if mode == "multigrid" else None,
                     "all_status_ok": all(st == 0 for st in status)}
        if mode == "graph":
            out[mode]["schedule"] = {"nlanes": B.schedule[0], "policy": ["balanced", "in_order"][B.schedule[1]]}
        B.close()
    out["faster"] = min(("graph", "multigrid"), key=lambda m: out[m]["ms_per_launch"])
    return out


def bench_batch(args):
    r = run_batch(args.steps, args.warmup)
    out = {"metric": "Mcell-solves/s, 64 mixed-size refined jobs (Poisson + 3 Helmholtz) as one graph",
           "value": r["value"], "unit": "Mcell-solves/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": r["ms_per_launch"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "bf16x3 MFMA, f32 accumulate, f64 residual/iterate", "data": "synthetic",
           "config": {"workload": r["workload"], "cell_solves_per_launch": r["cell_solves_per_launch"],
                      "schedule": r["schedule"]},
           "latency_ms": r["latency_ms"], "all_status_ok": r["all_status_ok"]}
    print(json.dumps(out), flush=True)


def run_serve(rates, count, geometries=0):
    """Poisson-process arrivals at each rate, continuous batching over 8
    slots; one summary row per rate."""
    import torch
    from paper_2406_19920_amd import serve, synth
    ex = serve.GpuExecutor(slots=8)
    # warm-up: load every kernel once for each kind and precision
    warm = [dict(rid=i, arrival=0.0, kind=k, refined=rf, n=n, beta=1.0, seed=i)
            for i, (k, rf, n) in enumerate([(k, rf, n) for k in ("poisson", "helmholtz")
                                             for rf in (False, True) for n in (32, 128, 384)])]
    srv = serve.Server(ex, 96 << 30, 8)
    srv.run(warm)
    srv.close()
    torch.cuda.synchronize()
    rows = []
    for i, rate in enumerate(rates):
        reqs = synth.serving_requests(rate, count, seed=5 + i, geometries=geometries)
        srv = serve.Server(ex, 96 << 30, 8)
        res = srv.run(reqs)
        d = res.summary()
        d["rate"] = rate
        rows.append(d)
        srv.close()
        log(json.dumps(d))
    workload = ("Poisson-process arrivals; 50/50 Poisson or Helmholtz x3; 50/50 FP64 or refined; "
                "n log-uniform [32,384] (multiple of 16; refined requests multiple of 32); beta ~ U[0,3]; "
                + (f"(n, beta) from a pool of {geometries} grids; " if geometries
                   else "a new grid per request; ")
                + f"8 slots, 96 GiB budget; {count} requests per rate")
    return rows, len(warm), workload


def bench_serve(args):
    rates = [float(r) for r in args.rates.split(",")]
    rows, nwarm, workload = run_serve(rates, args.count, args.geometries)
    best = max(rows, key=lambda d: d["mcell_solves_per_s"])
    out = {"metric": "serving: Mcell-solves/s and p50/p99 latency vs arrival rate",
           "value": best["mcell_solves_per_s"], "unit": "Mcell-solves/s", "n_gpus": 1,
           "steps": args.count, "warmup": nwarm, "ms_per_step": None, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64 and refined (50/50)",
           "data": "synthetic",
           "config": {"workload": workload, "rates": rates},
           "sweep": rows}
    print(json.dumps(out), flush=True)


def run_c3(steps, warmup):
    """512x384x384 (x, y, z) step on both paths; RHS = N(0,1) plus a
    smoothed-delta forcing shell (radius 0.1 Lx)."""
    import torch
    from paper_2406_19920_amd import ibsolve as ibs, synth
    nx, ny, nz, beta = 512, 384, 384, 2.0
    dev = torch.device("cuda:0")
    log("inputs 512x384x384")
    u, v, w = synth.velocity(nx, ny, nz, seed=3)
    fu, fv, fw = synth.forcing_shell(nx, ny, nz, seed=3)
    u += fu; v += fv; w += fw
    v[:, 0, :] = 0; v[:, ny, :] = 0
    c = 0.125 * min(h_min(ny, beta), 1.0 / nx, 1.0 / nz) ** 2
    ru, rv, rw = (torch.from_numpy(a).to(dev) for a in (u, v, w))
    del u, v, w
    res = {}
    for path, prec in (("refined", ibs.IBS_REFINED_BF16X3), ("fp64", ibs.IBS_FP64)):
        S = ibs.Solver(nx, ny, nz, beta=beta, precision=prec)
        tiles = S.autotune() if prec == ibs.IBS_FP64 else None   # set-up, untimed
        xu, xv, xw = S.empty(1), S.empty(2), S.empty(3)
        b, phi = S.empty(0), S.empty(0)

        def step():
            # reports: Helmholtz components in info slots 1..3, Poisson in 0
            S.helmholtz([0, 1, 2], [c, c, c], [ru, rv, rw], [xu, xv, xw], info_slot=1)
            S.divergence(xu, xv, xw, 1.0, b)
            S.poisson(b, phi)
            S.correct(phi, xu, xv, xw, 1.0)

        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        status = [S.read_info(q).status for q in range(4)]
        passes = {"helmholtz": [S.read_info(q).iters for q in (1, 2, 3)], "poisson": S.read_info(0).iters}
        # live per-kernel time per step (HIP events on the launch stream)
        ibs.ibs_profile(S.plan, True)
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        kern = {}
        for kid, name in enumerate(ibs.PROFILE_KERNELS):
            r = ibs.ibs_profile_read(S.plan, kid)
            if r["launches"]:
                kern[name] = {"ms_per_step": r["ms"] / steps,
                              "gbs": r["bytes"] / (r["ms"] * 1e-3) / 1e9 if r["ms"] else None,
                              "tflops": r["flops"] / (r["ms"] * 1e-3) / 1e12 if r["ms"] else None}
        ibs.ibs_profile(S.plan, False)
        res[path] = {"value": 4 * nx * ny * nz / (ms * 1e-3) / 1e6, "ms_per_step": ms,
                     "status": status, "passes": passes, "tiles": tiles, "kernels": kern}
        S.close()
    del ru, rv, rw
    torch.cuda.empty_cache()
    return res, "512x384x384, beta=2, N(0,1) + forcing shell, c=%.4e" % c


def run_3p(steps, warmup, n=256):
    """The triply periodic branch (periodic y too, uniform grid; cyclic y
    pencils) at n^3, both paths: one step of 3 Helmholtz + divergence +
    Poisson + correction on N(0,1) low-pass filtered velocities."""
    import torch
    from paper_2406_19920_amd import ibsolve as ibs, synth
    dev = torch.device("cuda:0")
    log(f"inputs {n}^3 triply periodic")
    u, v, w = synth.filtered_velocity(n, n, n, seed=6, kmax=16.0, zero_wall_v=False)
    v = np.ascontiguousarray(v[:, :n, :])
    c = 0.125 * (1.0 / n) ** 2
    ru, rv, rw = (torch.from_numpy(a).to(dev) for a in (u, v, w))
    res = {}
    for path, prec in (("refined", ibs.IBS_REFINED_BF16X3), ("fp64", ibs.IBS_FP64)):
        kw = {"max_iter": 2} if prec != ibs.IBS_FP64 else {}
        S = ibs.Solver(n, n, n, precision=prec, bc_y_vel=ibs.IBS_PERIODIC, bc_y_p=ibs.IBS_PERIODIC, **kw)
        tiles = S.autotune() if prec == ibs.IBS_FP64 else None   # set-up, untimed
        xu, xv, xw = S.empty(1), S.empty(2), S.empty(3)
        b, phi = S.empty(0), S.empty(0)

        def step():
            S.helmholtz([0, 1, 2], [c, c, c], [ru, rv, rw], [xu, xv, xw], info_slot=1)
            S.divergence(xu, xv, xw, 1.0, b)
            S.poisson(b, phi)
            S.correct(phi, xu, xv, xw, 1.0)

        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        res[path] = {"value": 4 * n ** 3 / (ms * 1e-3) / 1e6, "ms_per_step": ms,
                     "status": [S.read_info(q).status for q in range(4)],
                     "passes": {"helmholtz": [S.read_info(q).iters for q in (1, 2, 3)],
                                "poisson": S.read_info(0).iters},
                     "predicted_rel_err": ([S.read_info(q).rel_residual for q in range(4)]
                                           if prec != ibs.IBS_FP64 else None),
                     "tiles": tiles}
        S.close()
    return res, f"{n}^3 uniform, periodic in x, y and z, N(0,1) filtered to k <= 16, c = {c:.4e}"


def run_xw(steps, warmup, n=256, beta=2.0, walls_z=False, stretch_xz=0.0):
    """Walls in x (Dirichlet velocity, Neumann pressure at x = 0 and x = lx;
    unfolded cosine/sine transforms in x), and in z too when walls_z (a
    duct), at n^3 with tanh-stretched walls in y, both paths: one step of 3
    Helmholtz + divergence + Poisson + correction on N(0,1) velocities.
    stretch_xz > 0 (with walls_z): x and z tanh-stretched too, with that
    beta (the generalised eigenbases)."""
    import torch
    from paper_2406_19920_amd import ibsolve as ibs
    dev = torch.device("cuda:0")
    log(f"inputs {n}^3 walls in x" + (" and z" if walls_z else ""))
    u, v, w = make_inputs(n, beta, seed=12)
    u[:, :, 0] = 0.0
    if walls_z:
        w[0] = 0.0
    kwz = {"bc_z": ibs.IBS_DIRICHLET} if walls_z else {}
    c = 0.125 * h_min(n, beta) ** 2
    if stretch_xz > 0:
        j = np.arange(n + 1)
        f = 0.5 * (1 + np.tanh(stretch_xz * (2 * j / n - 1)) / np.tanh(stretch_xz))
        kwz.update(x_faces=f, z_faces=f)
        c = 0.125 * min(h_min(n, beta), float(np.diff(f).min())) ** 2
    ru, rv, rw = (torch.from_numpy(a).to(dev) for a in (u, v, w))
    res = {}
    for path, prec in (("refined", ibs.IBS_REFINED_BF16X3), ("fp64", ibs.IBS_FP64)):
        kw = {"max_iter": 2} if prec != ibs.IBS_FP64 else {}
        S = ibs.Solver(n, n, n, beta=beta, precision=prec, bc_x=ibs.IBS_DIRICHLET, **kw, **kwz)
        tiles = S.autotune() if prec == ibs.IBS_FP64 else None   # set-up, untimed
        xu, xv, xw = S.empty(1), S.empty(2), S.empty(3)
        b, phi = S.empty(0), S.empty(0)

        def step():
            S.helmholtz([0, 1, 2], [c, c, c], [ru, rv, rw], [xu, xv, xw], info_slot=1)
            S.divergence(xu, xv, xw, 1.0, b)
            S.poisson(b, phi)
            S.correct(phi, xu, xv, xw, 1.0)

        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        res[path] = {"value": 4 * n ** 3 / (ms * 1e-3) / 1e6, "ms_per_step": ms,
                     "status": [S.read_info(q).status for q in range(4)],
                     "passes": {"helmholtz": [S.read_info(q).iters for q in (1, 2, 3)],
                                "poisson": S.read_info(0).iters},
                     "tiles": tiles}
        S.close()
    walls = "walls in x and z (uniform) and y" if walls_z else "walls in x (uniform) and y"
    if stretch_xz > 0:
        walls = f"walls in x and z (tanh beta={stretch_xz}) and y"
    return res, (f"{n}^3, {walls} (tanh beta={beta})" + ("" if walls_z else ", periodic z")
                 + f", N(0,1) rhs, c = {c:.4e}")


def run_rk3(steps, warmup, n=256):
    """A full three-stage Runge-Kutta step (each stage: explicit estimate,
    immersed-boundary forcing, 3 Helmholtz solves, divergence, Poisson,
    projection and pressure update) at n^3 on a uniform wall-bounded grid,
    with a sphere of markers (radius 0.15, one marker per h^2 of surface),
    both paths.  Velocities: N(0,1) low-pass filtered to k <= 16; dt from a
    convective CFL of 0.2; Re = 1000."""
    import torch
    from paper_2406_19920_amd import ibsolve as ibs, synth
    dev = torch.device("cuda:0")
    log(f"inputs {n}^3 RK3 step with markers")
    u0, v0, w0 = synth.filtered_velocity(n, n, n, seed=8, kmax=16.0)
    p0 = synth.scalar(n, n, n, seed=9)
    h = 1.0 / n
    radius = 0.15
    nm = int(4.0 * np.pi * radius * radius / (h * h))
    X = synth.sphere_markers(nm, radius)
    rng = np.random.default_rng(10)
    UD = 0.1 * rng.standard_normal((nm, 3))
    umax = max(np.abs(a).max() for a in (u0, v0, w0))
    dt, re = 0.2 * h / umax, 1000.0
    rk3 = [(4 / 15, 4 / 15, 8 / 15, 0.0), (1 / 15, 1 / 15, 5 / 12, -17 / 60),
           (1 / 6, 1 / 6, 3 / 4, -5 / 12)]
    coefs = [dict(alpha=a, beta=b, gamma=g, zeta=z, dt=dt, re=re) for a, b, g, z in rk3]
    markers, ud = (torch.from_numpy(a).to(dev) for a in (X, UD))
    dvol = torch.full((nm,), h ** 3, dtype=torch.float64, device=dev)
    force = torch.zeros((nm, 3), dtype=torch.float64, device=dev)
    res = {}
    for path, prec in (("refined", ibs.IBS_REFINED_BF16X3), ("fp64", ibs.IBS_FP64)):
        S = ibs.Solver(n, n, n, precision=prec)
        tiles = S.autotune() if prec == ibs.IBS_FP64 else None   # set-up, untimed
        u, v, w, p = (torch.from_numpy(a).to(dev) for a in (u0, v0, w0, p0))
        nu, nv, nw = (torch.zeros_like(t) for t in (u, v, w))

        def step():
            for k in coefs:
                S.rk_stage(u, v, w, p, nu, nv, nw, k, markers, ud, dvol, force)

        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        status = [S.read_info(4 + q).status for q in range(4)]
        ibs.ibs_profile(S.plan, True)
        step()
        torch.cuda.synchronize()
        kern = {}
        for kid, name in enumerate(ibs.PROFILE_KERNELS):
            r = ibs.ibs_profile_read(S.plan, kid)
            if r["launches"]:
                kern[name] = {"ms_per_step": r["ms"], "launches": r["launches"],
                              "gbs": r["bytes"] / (r["ms"] * 1e-3) / 1e9 if r["ms"] else None}
        ibs.ibs_profile(S.plan, False)
        res[path] = {"value": n ** 3 / (ms * 1e-3) / 1e6, "ms_per_step": ms, "status": status,
                     "finite": bool(torch.isfinite(u).all()), "tiles": tiles, "kernels": kern}
        S.close()
    return res, (f"{n}^3 uniform walls, RK3 (3 sub-steps), {nm} markers on a sphere r={radius}, "
                 f"dt={dt:.3e}, Re={re:g}")


def bench_c3(args):
    res, workload = run_c3(args.steps, args.warmup)
    out = {"metric": "Mcell-solves/s at 512x384x384 (refined to 1e-10; FP64 alongside)",
           "value": res["refined"]["value"], "unit": "Mcell-solves/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": res["refined"]["ms_per_step"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "bf16x3 MFMA, f32 accumulate, f64 residual/iterate", "data": "synthetic",
           "config": {"workload": workload}, "paths": res}
    print(json.dumps(out), flush=True)


def bench_rk3(args):
    res, workload = run_rk3(args.steps, args.warmup, args.n)
    out = {"metric": f"Mcell-steps/s, full RK3 step with immersed markers at {args.n}^3",
           "value": res["refined"]["value"], "unit": "Mcell-steps/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": res["refined"]["ms_per_step"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64 stencils; solves bf16x3 MFMA refined (FP64 path alongside)",
           "data": "synthetic", "config": {"workload": workload}, "paths": res}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
