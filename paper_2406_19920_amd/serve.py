"""Continuous-batching request loop for the solver library.

Requests (one pressure Poisson solve, or the three Helmholtz components of
one fractional step) arrive over time.  The loop admits a waiting request as
soon as a slot is free and the device memory it needs fits the HBM budget,
so requests that arrive while others are on the GPU start immediately and
overlap with them (one HIP stream and one workspace per slot).  Plans
(eigenvector tables) stay resident in an LRU cache keyed by (grid,
stretching, precision) and count against the budget; a plan's device
constants are only read, so requests on the same grid run side by side.
Fields are allocated per request and released on completion.  A request
that does not fit yet is passed over by later ones that do, at most
`max_bypass` times in a row, after which admission waits for it (no
starvation).  Completion is detected by polling per-request events; latency
runs from arrival to completion.

Failure recovery: each request writes its solve reports (ibs_solve_info)
into a small buffer of its own.  When a refined-precision request completes
with IBS_ERR_NOT_CONVERGED (the device's error estimate missed tol within
the pass cap), it goes back to the head of the queue as an FP64 request on
the same grid, and only that second solve's result is delivered (latency
still runs from the original arrival).  Any other non-zero status is
recorded as a failed request.

The scheduler talks to an executor.  GpuExecutor drives the C ABI (every
solve step runs in the library's HIP kernels); tests substitute a fake
executor to check admission and ordering on the CPU.
"""
from __future__ import annotations

import collections
import time
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np

from . import synth


def field_bytes(n: int, kind: str) -> int:
    """Device bytes of a request's fields (right-hand sides and solutions)."""
    cells = n * n * n
    if kind == "poisson":
        return 2 * 8 * cells
    return 2 * 8 * (2 * cells + n * (n + 1) * n)


NOT_CONVERGED = 5     # IBS_ERR_NOT_CONVERGED


def plan_key(req):
    return (req["n"], round(req["beta"], 12), req["refined"], req.get("max_iter", 0))


class GpuExecutor:
    """Runs requests through the C ABI on per-slot HIP streams."""

    def __init__(self, slots: int, device="cuda", nmax: int = 384):
        import torch
        from . import ibsolve
        self.torch, self.ibs = torch, ibsolve
        self.device = torch.device(device)
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(slots)]
        # one workspace per slot, sized for the largest request (a plan then
        # holds only its constants; the workspace is needed only while a
        # request runs, and a slot runs one request at a time): the larger of
        # the two precisions' Helmholtz batch of 3 components at nmax
        need = 0
        for prec in (ibsolve.IBS_FP64, ibsolve.IBS_REFINED_BF16X3):
            pl = ibsolve.solver_plan(ibsolve.make_desc(nmax, nmax, nmax, precision=prec))
            try:
                for op, nc in ((ibsolve.IBS_OP_POISSON, 1), (ibsolve.IBS_OP_HELMHOLTZ_U, 3)):
                    need = max(need, ibsolve.solver_plan_bytes(pl, op, nc)[1])
            finally:
                ibsolve.solver_plan_destroy(pl)
        self.work_bytes = need
        self.slot_work = [torch.empty(self.work_bytes, dtype=torch.uint8, device=self.device)
                          for _ in range(slots)]
        # device bytes held for the executor's lifetime (counted against the
        # serving budget)
        self.fixed_bytes = slots * need

    def prepare(self, req):
        """Host-only plan build (thread-safe; the C call releases the GIL).
        Returns (plan handle, device bytes the plan will need)."""
        ibs = self.ibs
        n = req["n"]
        prec = ibs.IBS_REFINED_BF16X3 if req["refined"] else ibs.IBS_FP64
        plan = ibs.solver_plan(ibs.make_desc(n, n, n, beta=req["beta"], precision=prec,
                                             max_iter=req.get("max_iter", 0)))
        cb, wp = ibs.solver_plan_bytes(plan, ibs.IBS_OP_POISSON)
        _, wh = ibs.solver_plan_bytes(plan, ibs.IBS_OP_HELMHOLTZ_U, 3)
        if max(wp, wh) > self.work_bytes:
            ibs.solver_plan_destroy(plan)
            raise ValueError(f"request n={n} exceeds the slot workspace")
        return plan, cb

    def discard(self, prepared):
        self.ibs.solver_plan_destroy(prepared[0])

    def make_solver(self, req, prepared):
        ibs = self.ibs
        n = req["n"]
        prec = ibs.IBS_REFINED_BF16X3 if req["refined"] else ibs.IBS_FP64
        S = ibs.Solver(n, n, n, beta=req["beta"], precision=prec, device=self.device,
                       plan=prepared[0], alloc_work=False, max_iter=req.get("max_iter", 0))
        # the constants were copied on the current stream; make them visible
        # to the slot streams before first use
        self.torch.cuda.current_stream(self.device).synchronize()
        return S

    @staticmethod
    def solver_bytes(S) -> int:
        return S.const.numel()

    @staticmethod
    def close_solver(S):
        S.close()

    def launch(self, slot, req, S):
        """Enqueue the request; returns (event, fields, outputs, cell_solves,
        report), report being the request's device buffer of solve reports."""
        from .batch import cn_coefficient
        torch = self.torch
        stream = self.streams[slot]
        n = req["n"]
        S.work, S.work_bytes = self.slot_work[slot], self.work_bytes
        with torch.cuda.stream(stream):
            info = S.new_info(3)
            if req["kind"] == "poisson":
                b = synth.device_normal(S.shape(0), req["seed"], self.device)
                phi = S.empty(0)
                S.poisson(b, phi, info=info)
                fields, outs, cells = [b, phi], [phi], n ** 3
            else:
                rs = [synth.device_normal(S.shape(op), req["seed"] * 4 + op, self.device)
                      for op in (1, 2, 3)]
                rs[1][:, 0, :] = 0
                rs[1][:, n, :] = 0
                xs = [S.empty(op) for op in (1, 2, 3)]
                c = cn_coefficient(S)
                S.helmholtz([0, 1, 2], [c, c, c], rs, xs, info=info)
                fields, outs, cells = rs + xs, xs, 3 * n ** 3
            ev = torch.cuda.Event()
            ev.record(stream)
        return ev, fields, outs, cells, (info, 1 if req["kind"] == "poisson" else 3)

    def statuses(self, report):
        """Status of each solve of a completed request."""
        info, n = report
        return [self.ibs.info_record(info[q]).status for q in range(n)]

    @staticmethod
    def fetch(outs):
        return [o.cpu() for o in outs]

    def synchronize(self):
        self.torch.cuda.synchronize(self.device)


class PlanCache:
    """LRU cache of resident plans.  A cached plan may serve several
    requests at once (each brings its slot's workspace); plans in use are
    never evicted.  Host-side plan builds for waiting requests run ahead on
    a worker pool."""

    def __init__(self, executor, capacity_bytes: int, workers: int = 4):
        self.ex = executor
        self.capacity = capacity_bytes
        self.items = collections.OrderedDict()   # key -> solver
        self.refs = collections.Counter()        # key -> requests in flight
        self.bytes = 0
        self.hits = 0
        self.misses = 0
        self.pool = ThreadPoolExecutor(workers) if workers > 0 else None
        self.futures = {}                         # key -> future of a prepared plan

    def prefetch(self, req):
        k = plan_key(req)
        if k in self.items or k in self.futures:
            return
        if self.pool is not None:
            self.futures[k] = self.pool.submit(self.ex.prepare, req)

    def _prepared(self, req):
        k = plan_key(req)
        fut = self.futures.pop(k, None)
        return fut.result() if fut is not None else self.ex.prepare(req)

    def acquire(self, req, budget_left: int):
        """(solver, bytes newly resident) or (None, 0) when it cannot be placed now."""
        k = plan_key(req)
        S = self.items.get(k)
        if S is not None:
            self.items.move_to_end(k)
            self.refs[k] += 1
            self.hits += 1
            return S, 0
        prepared = self._prepared(req)
        need = prepared[1]
        while self.bytes + need > self.capacity or need > budget_left:
            victim = next((kk for kk in self.items if self.refs[kk] == 0), None)
            if victim is None:
                self.futures[k] = _Done(prepared)     # keep it for the next attempt
                return None, 0
            old = self.items.pop(victim)
            nb = self.ex.solver_bytes(old)
            self.bytes -= nb
            budget_left += nb
            self.ex.close_solver(old)
        S = self.ex.make_solver(req, prepared)
        self.items[k] = S
        self.refs[k] += 1
        nb = self.ex.solver_bytes(S)
        self.bytes += nb
        self.misses += 1
        return S, nb

    def release(self, req):
        k = plan_key(req)
        self.refs[k] -= 1
        if self.refs[k] <= 0:
            del self.refs[k]

    def close(self):
        for S in self.items.values():
            self.ex.close_solver(S)
        self.items.clear()
        self.bytes = 0
        for fut in self.futures.values():
            self.ex.discard(fut.result())
        self.futures.clear()
        if self.pool is not None:
            self.pool.shutdown(wait=True)


class _Done:
    """An already available result with the future interface."""

    def __init__(self, v):
        self.v = v

    def result(self):
        return self.v


@dataclass
class InFlight:
    req: dict
    event: object
    fields: list
    outputs: list
    bytes: int
    admitted: float
    cells: int = 0
    report: object = None


@dataclass
class ServeResult:
    latencies: np.ndarray
    makespan: float
    cell_solves: int
    completed: int
    outputs: dict = field(default_factory=dict)
    max_inflight: int = 0
    admit_order: list = field(default_factory=list)
    peak_bytes: int = 0
    plan_hits: int = 0
    plan_misses: int = 0
    fallbacks: list = field(default_factory=list)   # rids re-run on the FP64 path
    failed: dict = field(default_factory=dict)      # rid -> statuses of a failed request

    def summary(self) -> dict:
        lat = self.latencies * 1e3
        return {"completed": self.completed, "makespan_s": self.makespan,
                "req_per_s": self.completed / self.makespan if self.makespan else 0.0,
                "mcell_solves_per_s": self.cell_solves / self.makespan / 1e6 if self.makespan else 0.0,
                "p50_ms": float(np.percentile(lat, 50)) if lat.size else None,
                "p99_ms": float(np.percentile(lat, 99)) if lat.size else None,
                "max_inflight": self.max_inflight, "peak_bytes": self.peak_bytes,
                "plan_hits": self.plan_hits, "plan_misses": self.plan_misses,
                "fallbacks": len(self.fallbacks), "failed": len(self.failed)}


class Server:
    def __init__(self, executor, hbm_budget_bytes: int, slots: int = 8, keep_outputs: bool = False,
                 clock=time.perf_counter, idle=lambda: time.sleep(20e-6), plan_workers: int = 4,
                 max_bypass: int | None = None, lookahead: int = 32):
        self.max_bypass = 2 * slots if max_bypass is None else max_bypass
        self.lookahead = lookahead
        self.ex = executor
        self.budget = int(hbm_budget_bytes)
        self.slots = slots
        self.cache = PlanCache(executor, self.budget // 2, plan_workers)
        self.keep = keep_outputs
        self.clock = clock
        self.idle = idle

    def run(self, requests) -> ServeResult:
        """Serve requests (dicts with rid, arrival, kind, refined, n, beta, seed;
        sorted by arrival).  A request that can never fit is rejected up front."""
        fixed = getattr(self.ex, "fixed_bytes", 0)
        for r in requests:
            if fixed + field_bytes(r["n"], r["kind"]) > self.budget:
                raise ValueError(f"request {r['rid']} needs more than the HBM budget")
        pending = []
        inflight = [None] * self.slots
        used = self.cache.bytes + fixed
        lat, cell_solves, outputs, order = [], 0, {}, []
        fallbacks, failed = [], {}
        nreq, nxt, done = len(requests), 0, 0
        max_inflight, peak = 0, used
        bypassed = 0     # admissions that went ahead of the current oldest request
        self.ex.synchronize()
        t0 = self.clock()
        while done < nreq:
            now = self.clock() - t0
            while nxt < nreq and requests[nxt]["arrival"] <= now:
                pending.append(requests[nxt])
                self.cache.prefetch(requests[nxt])
                nxt += 1
            progressed = False
            for s, f in enumerate(inflight):
                if f is not None and f.event.query():
                    st = self.ex.statuses(f.report)
                    used -= f.bytes
                    self.cache.release(f.req)
                    inflight[s] = None
                    progressed = True
                    if f.req["refined"] and NOT_CONVERGED in st:
                        # recover on the FP64 path, ahead of every waiting request
                        retry = dict(f.req, refined=False, max_iter=0)
                        fallbacks.append(f.req["rid"])
                        pending.insert(0, retry)
                        self.cache.prefetch(retry)
                        continue
                    lat.append(self.clock() - t0 - f.req["arrival"])
                    if any(st):
                        failed[f.req["rid"]] = st
                    else:
                        cell_solves += f.cells
                    if self.keep:
                        outputs[f.req["rid"]] = self.ex.fetch(f.outputs)
                    done += 1
            idx = 0
            while idx < min(len(pending), self.lookahead):
                s = next((i for i, f in enumerate(inflight) if f is None), None)
                if s is None:
                    break
                if idx > 0 and bypassed >= self.max_bypass:
                    break        # the oldest request has waited long enough
                req = pending[idx]
                fb = field_bytes(req["n"], req["kind"])
                S, nb = None, 0
                if used + fb <= self.budget:
                    S, nb = self.cache.acquire(req, self.budget - used - fb)
                if S is None:
                    idx += 1     # does not fit now: try a later request
                    continue
                used += nb
                del pending[idx]
                bypassed = bypassed + 1 if idx > 0 else 0
                ev, fields, outs, cells, report = self.ex.launch(s, req, S)
                inflight[s] = InFlight(req, ev, fields, outs, fb, self.clock() - t0, cells, report)
                used += fb
                order.append(req["rid"])
                progressed = True
                max_inflight = max(max_inflight, sum(f is not None for f in inflight))
                peak = max(peak, used)
            if not progressed:
                self.idle()
        makespan = self.clock() - t0
        return ServeResult(np.array(lat), makespan, cell_solves, done, outputs, max_inflight, order,
                           peak, self.cache.hits, self.cache.misses, fallbacks, failed)

    def run_alone(self, req):
        """Run one request by itself (for the alone-versus-mixed check)."""
        S, _ = self.cache.acquire(req, self.budget)
        ev, fields, outs, _, _ = self.ex.launch(0, req, S)
        self.ex.synchronize()
        self.cache.release(req)
        return self.ex.fetch(outs)

    def close(self):
        self.cache.close()


def sweep(rates, count: int, seed: int = 5, hbm_budget_gb: float = 96.0, slots: int = 8,
          nmin: int = 32, nmax: int = 384):
    """Serve `count` requests at each arrival rate; one summary per rate."""
    ex = GpuExecutor(slots)
    out = []
    for i, rate in enumerate(rates):
        reqs = synth.serving_requests(rate, count, seed + i, nmin=nmin, nmax=nmax)
        srv = Server(ex, int(hbm_budget_gb * (1 << 30)), slots)
        res = srv.run(reqs)
        d = res.summary()
        d["rate"] = rate
        out.append(d)
        srv.close()
    return out
