"""Batched solves of many independent grids replayed as one HIP graph.

Each job is one fractional-step solve set on its own grid: the three
Helmholtz components (one batched call) and one pressure Poisson solve.
The library records all jobs into one graph (ibs_batch_build) whose
independent branches let small grids overlap on the device; a replay is one
hipGraphLaunch.  mode="multigrid" (FP64 plans) builds the batch with
ibs_batch_build_multigrid instead: each solve stage is one persistent
launch over every grid, five launches per replay whatever the job count.  Buffers are torch allocations that live as long as the
batch.
"""
from __future__ import annotations

import numpy as np

from . import ibsolve as ibs
from . import synth


def cn_coefficient(solver) -> float:
    """Crank-Nicolson Helmholtz coefficient c = 0.5 nu dt with
    nu dt / h_min^2 = 0.25, h_min the smallest cell height of the grid."""
    yf = ibs.ibs_plan_export(solver.plan, 0)
    hmin = min(float(np.diff(yf).min()), solver.desc.lx / solver.nx, solver.desc.lz / solver.nz)
    return 0.125 * hmin * hmin


# boundary kinds a job spec may name (key "bc"; default "walls": walls in y,
# periodic x and z)
BC_KINDS = {
    "walls": {},
    "periodic_y": dict(bc_y_vel=ibs.IBS_PERIODIC, bc_y_p=ibs.IBS_PERIODIC),
    "walls_x": dict(bc_x=ibs.IBS_DIRICHLET),
}


class Job:
    def __init__(self, spec, precision, device, own_poisson_work=False):
        nx, ny, nz = spec["nx"], spec["ny"], spec["nz"]
        self.spec = spec
        self.solver = ibs.Solver(nx, ny, nz, beta=spec["beta"], precision=precision, device=device,
                                 **BC_KINDS[spec.get("bc", "walls")])
        S = self.solver
        self.c = spec.get("c", cn_coefficient(S))
        seed = spec["seed"]
        self.r = [synth.device_normal(S.shape(op), seed * 8 + op, S.device) for op in (1, 2, 3)]
        if not S.periodic_y:
            self.r[1][:, 0, :] = 0
            self.r[1][:, ny, :] = 0
        self.b = synth.device_normal(S.shape(0), seed * 8 + 5, S.device)
        self.x = [S.empty(op) for op in (1, 2, 3)]
        self.phi = S.empty(0)
        # multi-grid batches run every job side by side: the Poisson solve
        # then needs a workspace of its own
        self.work_p = None
        if own_poisson_work:
            import torch
            self.work_p = torch.empty(S.work_p, dtype=torch.uint8, device=S.device)

    @property
    def cell_solves(self) -> int:
        s = self.spec
        return 4 * s["nx"] * s["ny"] * s["nz"]

    def records(self):
        S = self.solver
        return [S.helmholtz_job([0, 1, 2], [self.c] * 3, self.r, self.x, info_slot=0),
                S.poisson_job(self.b, self.phi, info_slot=3, work=self.work_p)]

    def run_eager(self):
        S = self.solver
        S.helmholtz([0, 1, 2], [self.c] * 3, self.r, self.x, info_slot=0)
        S.poisson(self.b, self.phi)

    def outputs(self):
        return self.x + [self.phi]


class Batch:
    """All jobs of a batch, captured once; launch() replays the graph.
    nlanes="auto": the schedule (lane count and policy) is chosen by the
    library's schedule autotuner, timed on the device at set-up (the jobs
    run during tuning); self.schedule records (nlanes, policy, ms).
    mode: "graph" (per-grid launch sequences on graph lanes), "multigrid"
    (FP64: one persistent launch per stage over all grids) or "auto" (FP64:
    both timed at set-up, the faster kept; self.mode names it and
    self.timings holds both ms per replay)."""

    def __init__(self, specs, precision=ibs.IBS_REFINED_BF16X3, nlanes=8, device="cuda",
                 policy=ibs.IBS_SCHED_BALANCED, tune_reps=3, mode="graph"):
        import torch
        self.torch = torch
        if mode not in ("graph", "multigrid", "auto"):
            raise ValueError(mode)
        if mode == "auto" and precision != ibs.IBS_FP64:
            mode = "graph"                 # multi-grid batches are FP64 only
        self.mode = mode
        self.jobs = [Job(s, precision, device, own_poisson_work=mode != "graph") for s in specs]
        torch.cuda.synchronize()
        recs = []
        for j in self.jobs:
            recs.extend(j.records())
        self.schedule = None
        self.timings = None
        if mode == "multigrid":
            self.handle = ibs.ibs_batch_build_multigrid(recs)
            return
        if mode == "auto":
            # both forms timed on the device (the jobs run), the faster kept:
            # many small grids favour the multi-grid stage launches, large
            # ones the per-grid folded transforms of the graph
            stream = torch.cuda.current_stream().cuda_stream
            nl, pol, ms_graph = ibs.ibs_batch_autotune(recs, tune_reps, stream)
            mg = ibs.ibs_batch_build_multigrid(recs)
            ms_mg = self._time(mg, tune_reps)
            self.timings = {"graph": ms_graph, "multigrid": ms_mg}
            if ms_mg < ms_graph:
                self.mode, self.handle = "multigrid", mg
                return
            ibs.ibs_batch_destroy(mg)
            self.mode, self.schedule = "graph", (nl, pol, ms_graph)
            self.handle = ibs.ibs_batch_build(recs, nl, pol)
            return
        if nlanes == "auto":
            stream = torch.cuda.current_stream().cuda_stream
            nlanes, policy, ms = ibs.ibs_batch_autotune(recs, tune_reps, stream)
            self.schedule = (nlanes, policy, ms)
        self.handle = ibs.ibs_batch_build(recs, nlanes, policy)

    @property
    def cell_solves(self) -> int:
        return sum(j.cell_solves for j in self.jobs)

    def _time(self, handle, reps):
        """Best of three rounds of reps replays (ms per replay), after one
        untimed replay."""
        torch = self.torch
        s = torch.cuda.current_stream().cuda_stream
        ibs.ibs_batch_launch(handle, s)
        best = float("inf")
        for _ in range(3):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(reps):
                ibs.ibs_batch_launch(handle, s)
            b.record()
            b.synchronize()
            best = min(best, a.elapsed_time(b) / reps)
        return best

    def launch(self, stream=None):
        s = self.torch.cuda.current_stream().cuda_stream if stream is None else stream
        ibs.ibs_batch_launch(self.handle, s)

    def close(self):
        if self.handle:
            ibs.ibs_batch_destroy(self.handle)
            self.handle = None
        for j in self.jobs:
            j.solver.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
