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


def cpu_baseline(n_sample, beta, seed):
    """The oracle (C/OpenMP CG) on the same step at a reduced grid."""
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
    dt = time.perf_counter() - t0
    cells = n_sample ** 3
    return {"value": 4 * cells / dt / 1e6, "unit": "Mcell-solves/s",
            "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"one full step (3 Helmholtz + divergence + Poisson + correction) of the "
                      f"same workload at {n_sample}^3 (beta={beta}, same c rule), "
                      f"{dt:.1f} s; the CG iteration count grows with the grid, so this "
                      f"overstates the oracle's rate at 256^3"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--beta", type=float, default=2.0)
    ap.add_argument("--path", choices=["refined", "fp64", "both"], default="both")
    ap.add_argument("--cpu-sample", type=int, default=128)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this solver is single-GPU "
              "(multi-GPU sharding is a design note, not built)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2406_19920_amd import ibsolve as ibs

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
        S = ibs.Solver(n, n, n, beta=beta, precision=precision)
        xu, xv, xw = S.empty(1), S.empty(2), S.empty(3)
        b = S.empty(0)
        phi = S.empty(0)

        def step():
            S.helmholtz([0, 1, 2], [c, c, c], [ru, rv, rw], [xu, xv, xw])
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
        infos = [S.read_info(q) for q in range(3)]
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
        S.poisson(b, phi)
        torch.cuda.synchronize()
        pinfo = S.read_info(0)
        S.close()
        return dict(ms=ms, per=per, kern=kern, hinfo=infos, pinfo=pinfo)

    def roofline(kern, steps):
        dom_name = max(kern, key=lambda k: kern[k]["ms"])
        d = kern[dom_name]
        avg_ms = d["ms"] / d["launches"]
        if dom_name in ("xgemm_f64", "zgemm_f64"):
            achieved = d["flops"] / d["launches"] / (avg_ms * 1e-3) / 1e12
            roof = {"bound": "mfma", "achieved": achieved, "peak": PEAK["fp64_tflops"],
                    "unit": "TFLOP/s"}
        else:
            achieved = d["bytes"] / d["launches"] / (avg_ms * 1e-3) / 1e9
            roof = {"bound": "hbm", "achieved": achieved, "peak": PEAK["hbm_gbs"], "unit": "GB/s"}
        roof["frac"] = roof["achieved"] / roof["peak"]
        roof["traffic"] = None
        roof["kernel"] = dom_name
        roof["avg_launch_ms"] = avg_ms
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
            roofline=roof, kernels=brk,
            passes={"helmholtz": r["hinfo"][0].iters, "poisson": r["pinfo"].iters},
            predicted_rel_err={"helmholtz": max(i.rel_residual for i in r["hinfo"]),
                               "poisson": r["pinfo"].rel_residual} if path == "refined" else None,
            status=[i.status for i in r["hinfo"]] + [r["pinfo"].status])

    cpu = None
    if not args.no_cpu_baseline:
        log(f"cpu baseline: oracle at {args.cpu_sample}^3")
        cpu = cpu_baseline(args.cpu_sample, beta, seed=2)

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
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
