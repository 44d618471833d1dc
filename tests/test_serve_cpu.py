"""Serving loop scheduling on the CPU with a fake executor and a simulated
clock: admission by HBM footprint, FIFO order, overlap, plan reuse, and
host-forced failures."""
import numpy as np
import pytest

from paper_2406_19920_amd import serve, synth


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def tick(self):
        self.t += 1e-4


class FakeEvent:
    def __init__(self, clock, t_done):
        self.clock, self.t_done = clock, t_done

    def query(self):
        return self.clock() >= self.t_done


class FakeExecutor:
    """Duration proportional to the cells solved; bytes proportional to n^3."""

    def __init__(self, clock, rate_cells_per_s=1e9, fail_rid=None, diverge=(), bad=()):
        self.clock = clock
        self.diverge = set(diverge)    # rids whose refined solve reports NOT_CONVERGED
        self.bad = set(bad)            # rids that report another error on every path
        self.rate = rate_cells_per_s
        self.fail_rid = fail_rid
        self.running = []
        self.max_same_plan = 0

    def prepare(self, req):
        return ("plan", 8 * req["n"] ** 2 * 4)

    def discard(self, prepared):
        pass

    def make_solver(self, req, prepared):
        return {"key": serve.plan_key(req), "bytes": prepared[1]}

    @staticmethod
    def solver_bytes(S):
        return S["bytes"]

    @staticmethod
    def close_solver(S):
        S["closed"] = True

    def launch(self, slot, req, S):
        if req["rid"] == self.fail_rid:
            raise RuntimeError("injected executor failure")
        cells = req["n"] ** 3 * (1 if req["kind"] == "poisson" else 3)
        ev = FakeEvent(self.clock, self.clock() + cells / self.rate)
        live = [e for e in self.running if not e[0].query()]
        same = sum(1 for e in live if e[1] == S["key"]) + 1
        self.max_same_plan = max(self.max_same_plan, same)
        self.running = live + [(ev, S["key"])]
        n = 1 if req["kind"] == "poisson" else 3
        if req["rid"] in self.bad:
            st = [6] * n
        elif req["refined"] and req["rid"] in self.diverge:
            st = [0] * (n - 1) + [serve.NOT_CONVERGED]
        else:
            st = [0] * n
        self.launched = getattr(self, "launched", []) + [(req["rid"], req["refined"])]
        return ev, [], [(req["rid"], req["refined"])], cells, st

    @staticmethod
    def statuses(report):
        return report

    @staticmethod
    def fetch(outs):
        return list(outs)

    def synchronize(self):
        pass


def _server(budget=1 << 34, slots=4, **kw):
    clock = FakeClock()
    ex = FakeExecutor(clock, **kw)
    return serve.Server(ex, budget, slots, keep_outputs=True, clock=clock, idle=clock.tick,
                        plan_workers=0), ex, clock


def test_all_complete_fifo_and_overlap():
    reqs = synth.serving_requests(rate=5000, count=60, seed=3, nmin=32, nmax=128)
    srv, ex, _ = _server()
    res = srv.run(reqs)
    assert res.completed == 60 and len(res.outputs) == 60
    assert res.admit_order == sorted(res.admit_order)      # FIFO admission
    assert res.max_inflight > 1                            # continuous batching overlaps
    assert np.all(res.latencies > 0)
    s = res.summary()
    assert s["p99_ms"] >= s["p50_ms"] > 0


def test_same_grid_requests_overlap():
    """A plan's device constants are read-only: requests on one grid run
    side by side (each on its own slot workspace)."""
    reqs = [dict(rid=i, arrival=0.0, kind="helmholtz", refined=True, n=64, beta=1.0, seed=i)
            for i in range(6)]
    srv, ex, _ = _server(slots=3)
    res = srv.run(reqs)
    assert res.completed == 6
    assert ex.max_same_plan == 3
    assert res.plan_misses == 1 and res.plan_hits == 5


def test_head_of_line_bypass_bounded():
    """A request that does not fit while others run is passed over by later
    ones that fit, at most max_bypass times; then admission waits for it and
    it completes (no starvation)."""
    big = dict(rid=1, arrival=1e-6, kind="helmholtz", refined=False, n=128, beta=0.0, seed=1)
    small = [dict(rid=i, arrival=(0.0 if i == 0 else 2e-6), kind="poisson", refined=False, n=32,
                  beta=0.0, seed=i) for i in [0] + list(range(2, 12))]
    reqs = sorted([big] + small, key=lambda r: r["arrival"])
    plan_bytes = 8 * 128 ** 2 * 4 + 8 * 32 ** 2 * 4
    budget = serve.field_bytes(128, "helmholtz") + plan_bytes + serve.field_bytes(32, "poisson") // 2
    # the big request fits only when nothing else runs; solves last far
    # longer than the simulated clock's idle tick
    srv, ex, _ = _server(budget=budget, slots=4, rate_cells_per_s=1e6)
    srv.max_bypass = 3
    res = srv.run(reqs)
    assert res.completed == len(reqs)
    order = res.admit_order
    pos = order.index(1)
    assert order[0] == 0
    assert pos == 1 + 3                # later small ones went past the big one, max_bypass of them
    assert res.peak_bytes <= budget


def test_fixed_executor_bytes_count_against_budget():
    reqs = [dict(rid=0, arrival=0.0, kind="poisson", refined=False, n=32, beta=0.0, seed=0)]
    srv, ex, _ = _server(budget=serve.field_bytes(32, "poisson") + (1 << 20))
    ex.fixed_bytes = 1 << 21
    with pytest.raises(ValueError):
        srv.run(reqs)


def test_budget_limits_concurrency():
    reqs = [dict(rid=i, arrival=0.0, kind="helmholtz", refined=False, n=64, beta=0.1 * i, seed=i)
            for i in range(6)]
    one = serve.field_bytes(64, "helmholtz")
    budget = int(2.5 * one) + 2 * (8 * 64 ** 2 * 4) + (1 << 20)
    srv, _, _ = _server(budget=budget, slots=6)
    res = srv.run(reqs)
    assert res.completed == 6
    assert res.max_inflight == 2
    assert res.peak_bytes <= budget


def test_plan_reuse_and_lru():
    reqs = [dict(rid=i, arrival=0.001 * i, kind="poisson", refined=True, n=32, beta=1.0, seed=i)
            for i in range(5)]
    srv, _, _ = _server(slots=2)
    res = srv.run(reqs)
    assert res.completed == 5
    assert res.plan_misses == 1 and res.plan_hits == 4


def test_over_budget_request_rejected():
    reqs = [dict(rid=0, arrival=0.0, kind="poisson", refined=False, n=256, beta=0.0, seed=0)]
    srv, _, _ = _server(budget=1 << 20)
    with pytest.raises(ValueError):
        srv.run(reqs)


def test_injected_executor_failure_propagates():
    reqs = synth.serving_requests(rate=1000, count=8, seed=1, nmin=32, nmax=64)
    srv, _, _ = _server(fail_rid=3)
    with pytest.raises(RuntimeError, match="injected"):
        srv.run(reqs)


def test_request_generator_recipe():
    reqs = synth.serving_requests(rate=1000, count=4000, seed=9)
    arr = np.array([r["arrival"] for r in reqs])
    assert np.all(np.diff(arr) >= 0)
    assert abs(len(reqs) / arr[-1] - 1000) < 100            # Poisson rate
    ns = np.array([r["n"] for r in reqs])
    rf = np.array([r["refined"] for r in reqs])
    assert ns.min() >= 32 and ns.max() <= 384
    assert np.all(ns[rf] % 32 == 0) and np.all(ns[~rf] % 16 == 0)
    assert np.any(ns[~rf] % 32 == 16)          # FP64 requests use the finer sizes
    assert 0.45 < np.mean([r["kind"] == "poisson" for r in reqs]) < 0.55
    assert 0.45 < np.mean([r["refined"] for r in reqs]) < 0.55


def test_geometry_pool_reuses_plans():
    reqs = synth.serving_requests(rate=1000, count=400, seed=4, nmin=32, nmax=128, geometries=5)
    grids = {(r["n"], r["beta"]) for r in reqs}
    assert len(grids) <= 10                     # each pool grid, rounded per precision
    assert len({r["beta"] for r in reqs}) <= 5
    assert all(r["n"] % (32 if r["refined"] else 16) == 0 and 32 <= r["n"] <= 128
               and 0.0 <= r["beta"] <= 3.0 for r in reqs)
    # the pool depends on the seed alone, not on the rate
    other = synth.serving_requests(rate=50, count=400, seed=4, nmin=32, nmax=128, geometries=5)
    assert {(r["n"], r["beta"]) for r in other} == grids
    srv, ex, _ = _server()
    res = srv.run(reqs)
    d = res.summary()
    assert d["completed"] == 400
    # one miss per plan key at most per concurrent use; most requests hit
    assert d["plan_hits"] > 280 and d["plan_hits"] + d["plan_misses"] == 400


def test_not_converged_refined_request_falls_back_to_fp64():
    """A refined request reporting NOT_CONVERGED is re-run once on the FP64
    path, ahead of the queue; the FP64 result is the one delivered, its
    latency runs from the original arrival, and its cells count once."""
    reqs = synth.serving_requests(2000.0, 40, seed=3, nmin=32, nmax=96)
    refined = [r["rid"] for r in reqs if r["refined"]]
    fp64 = [r["rid"] for r in reqs if not r["refined"]]
    diverge = refined[:3] + fp64[:1]          # the FP64 one must not be retried
    srv, ex, _ = _server(diverge=diverge)
    res = srv.run(reqs)
    assert res.completed == len(reqs) and len(res.latencies) == len(reqs)
    assert sorted(res.fallbacks) == sorted(refined[:3])
    assert not res.failed
    for rid in refined[:3]:
        assert res.outputs[rid] == [(rid, False)]            # delivered from the FP64 re-run
        assert ex.launched.count((rid, True)) == 1 and ex.launched.count((rid, False)) == 1
    for rid in refined[3:]:
        assert res.outputs[rid] == [(rid, True)]
    cells = sum(r["n"] ** 3 * (1 if r["kind"] == "poisson" else 3) for r in reqs)
    assert res.cell_solves == cells
    assert res.summary()["fallbacks"] == 3


def test_other_errors_are_reported_not_retried():
    reqs = synth.serving_requests(500.0, 12, seed=4, nmin=32, nmax=64)
    bad = [reqs[2]["rid"], reqs[5]["rid"]]
    srv, ex, _ = _server(bad=bad)
    res = srv.run(reqs)
    assert res.completed == len(reqs)
    assert sorted(res.failed) == sorted(bad)
    assert not res.fallbacks
    assert len(ex.launched) == len(reqs)
