"""Multi-grid batches (ibs_batch_build_multigrid): every solve stage is one
persistent launch over all grids.  Each job's Poisson and Helmholtz results
match the single-grid FP64 solves of the same inputs (max norm, to
rounding: the plain transforms and the Thomas pencils order their sums
differently) and, for a sample, the oracle; replays are bitwise
reproducible; reports match; the C4-size mix runs; bad jobs are refused."""
import sys

import numpy as np
import pytest

import oracle
from oracle import OP_P, OP_U, OP_V, OP_W
from paper_2406_19920_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mods():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2406_19920_amd import batch, ibsolve
    return ibsolve, batch


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _maxrel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def _tanh_faces(n, beta):
    j = np.arange(n + 1)
    return 0.5 * (1 + np.tanh(beta * (2 * j / n - 1)) / np.tanh(beta))


class _Job:
    """One grid's Helmholtz x3 and Poisson solve with its own buffers and
    two workspaces (Helmholtz, Poisson)."""

    def __init__(self, ibs, nx, ny, nz, beta, seed, **kw):
        self.S = S = ibs.Solver(nx, ny, nz, beta=beta, precision=ibs.IBS_FP64, **kw)
        self.kw = kw
        self.beta = beta
        hmin = float(np.diff(ibs.ibs_plan_export(S.plan, 0)).min())
        self.c = 0.125 * min(hmin, 1.0 / nx, 1.0 / nz) ** 2 * 8
        self.r = [synth.device_normal(S.shape(op), seed * 8 + op, S.device) for op in (1, 2, 3)]
        self.r[1][:, 0, :] = 0
        self.r[1][:, ny, :] = 0
        self.b = synth.device_normal(S.shape(0), seed * 8 + 5, S.device) + 0.25   # nonzero mean
        self.x = [S.empty(op) for op in (1, 2, 3)]
        self.phi = S.empty(0)
        self.work_p = torch.empty(S.work_p, dtype=torch.uint8, device=S.device)
        self.info = S.new_info(4)

    def records(self, ibs):
        S = self.S
        jh = S.helmholtz_job([0, 1, 2], [self.c] * 3, self.r, self.x)
        jp = S.poisson_job(self.b, self.phi, work=self.work_p)
        jh.info = self.info[0].data_ptr()
        jp.info = self.info[3].data_ptr()
        return [jh, jp]

    def single(self):
        S = self.S
        xs = S.helmholtz([0, 1, 2], [self.c] * 3, self.r)
        phi = S.poisson(self.b)
        torch.cuda.synchronize()
        return [x.cpu().numpy() for x in xs] + [phi.cpu().numpy()], [S.read_info(q) for q in range(4)]

    def outputs(self):
        torch.cuda.synchronize()
        return [x.cpu().numpy() for x in self.x] + [self.phi.cpu().numpy()]


def _mix(ibs):
    rng = np.random.default_rng(3)
    specs = [((32, 24, 48), 1.0, {}), ((64, 40, 32), 2.0, dict(bc_x=ibs.IBS_DIRICHLET)),
             ((48, 33, 64), 1.5, dict(bc_x=ibs.IBS_DIRICHLET, bc_z=ibs.IBS_DIRICHLET,
                                       x_faces=_tanh_faces(48, 1.2), z_faces=_tanh_faces(64, 0.8))),
             ((96, 64, 96), 0.0, {}), ((16, 8, 16), 3.0, {}), ((80, 20, 48), 2.5, dict(bc_z=ibs.IBS_DIRICHLET)),
             ((128, 96, 64), 1.0, {})]
    return [_Job(ibs, *shape, beta, int(rng.integers(1, 10 ** 6)), **kw) for shape, beta, kw in specs]


def test_multigrid_matches_single_grid_and_oracle(mods):
    ibs, _ = mods
    _say("case multigrid mix")
    jobs = _mix(ibs)
    recs = [r for j in jobs for r in j.records(ibs)]
    h = ibs.ibs_batch_build_multigrid(recs)
    try:
        stream = torch.cuda.current_stream().cuda_stream
        ibs.ibs_batch_launch(h, stream)
        first = [j.outputs() for j in jobs]
        ibs.ibs_batch_launch(h, stream)
        second = [j.outputs() for j in jobs]
    finally:
        ibs.ibs_batch_destroy(h)
    for jb, a, b in zip(jobs, first, second):
        for u, v in zip(a, b):
            np.testing.assert_array_equal(u, v)   # replays are bitwise reproducible
    for k, jb in enumerate(jobs):
        single, infos = jb.single()
        errs = [_maxrel(m, s) for m, s in zip(first[k], single)]
        _say("job", k, jb.S.nx, jb.S.ny, jb.S.nz, "errs vs single-grid", errs)
        assert max(errs) < 1e-12
        got = [ibs.info_record(jb.info[q]) for q in range(4)]
        for q in range(4):
            assert got[q].status == 0 and got[q].iters == 1
        assert abs(got[3].removed_mean - infos[0].removed_mean) <= 1e-12 * abs(infos[0].removed_mean)
        assert got[3].removed_mean > 0.1            # the rhs's +0.25 shift, reported
        # the v wall rows and the x / z wall slots are zero
        assert np.all(first[k][1][:, 0, :] == 0) and np.all(first[k][1][:, -1, :] == 0)
        if "bc_x" in jb.kw:
            assert np.all(first[k][0][:, :, 0] == 0)
        if "bc_z" in jb.kw:
            assert np.all(first[k][2][0] == 0)
    # a sample against the oracle (the stretched duct and a periodic grid)
    for k in (0, 2):
        jb = jobs[k]
        S = jb.S
        g = oracle.Grid(S.nx, S.ny, S.nz, beta=jb.beta, periodic_x="bc_x" not in jb.kw,
                        periodic_z="bc_z" not in jb.kw, xf_in=jb.kw.get("x_faces"), zf_in=jb.kw.get("z_faces"))
        xo, _ = oracle.solve(g, OP_P, jb.b.cpu().numpy())
        err = _maxrel(first[k][3], xo)
        ref = oracle.solve(g, OP_V, jb.r[1].cpu().numpy(), c=jb.c)[0]
        errv = _maxrel(first[k][1], ref)
        _say("job", k, "vs oracle: poisson", err, "v", errv)
        assert err < 1e-12 and errv < 1e-12


def _rel(a, b):
    d = (a - b).ravel()
    return max(float(np.linalg.norm(d) / np.linalg.norm(b.ravel())),
               float(np.abs(d).max() / np.abs(b).max()))


def test_multigrid_c4_sizes_manufactured(mods):
    """Jobs at the mixed-size batch's own grid sizes (96x128x96, 192x256x192
    and 64^3, stretched) in one multi-grid batch: all four solves of each
    return the manufactured solutions (b = A x_true by the oracle's
    long-double stencil) to 1e-12 in l2 and max norm."""
    ibs, batch = mods
    specs = [dict(nx=96, ny=128, nz=96, beta=1.2, seed=1200),
             dict(nx=192, ny=256, nz=192, beta=2.4, seed=1201),
             dict(nx=64, ny=64, nz=64, beta=0.3, seed=1202)]
    _say("case multigrid c4 sizes manufactured")
    B = batch.Batch(specs, precision=ibs.IBS_FP64, mode="multigrid")
    try:
        truth = []
        for j in B.jobs:
            s = j.spec
            g = oracle.Grid(s["nx"], s["ny"], s["nz"], beta=s["beta"])
            xs = []
            for q, op in enumerate((OP_U, OP_V, OP_W)):
                rows = s["ny"] + 1 if op == OP_V else None
                xt = synth.manufactured(s["nx"], s["ny"], s["nz"], seed=s["seed"] + 10 * q, rows=rows)
                if op == OP_V:
                    xt[:, 0, :] = 0
                    xt[:, s["ny"], :] = 0
                r, _, _ = oracle.residual_ld(g, op, j.c, xt, np.zeros_like(xt))
                j.r[q].copy_(torch.from_numpy(-r))
                xs.append(xt)
            xp = synth.manufactured(s["nx"], s["ny"], s["nz"], seed=s["seed"] + 77)
            xp = xp - oracle.weighted_mean(g, OP_P, xp)
            r, _, _ = oracle.residual_ld(g, OP_P, 0.0, xp, np.zeros_like(xp))
            j.b.copy_(torch.from_numpy(-r))
            truth.append(xs + [xp])
        torch.cuda.synchronize()
        B.launch()
        torch.cuda.synchronize()
        for q, (j, tr) in enumerate(zip(B.jobs, truth)):
            for k, (o, t) in enumerate(zip(j.outputs(), tr)):
                err = _rel(o.cpu().numpy(), t)
                _say("job", q, j.spec["nx"], j.spec["ny"], "solve", k, "err", err)
                assert err < 1e-12
            assert all(j.solver.read_info(k).status == 0 for k in range(4))
    finally:
        B.close()


def test_multigrid_c4_mix(mods):
    """The 64-job mixed-size batch (64^3 to 192x256x192) as five launches:
    every job matches its single-grid FP64 solves on the same N(0,1)
    right-hand sides: the Helmholtz components to 1e-12 in max norm, the
    pressure to 5e-12 (on these rough right-hand sides each FP64 pressure
    solve at 192x256x192 with beta up to 3 is itself within about 1e-12 of
    the exact discrete solution, so two of them differ by up to the sum;
    the manufactured-solution test above pins each against the truth)."""
    ibs, batch = mods
    _say("case multigrid c4")
    specs = synth.batch_specs(64, seed=4)
    B = batch.Batch(specs, precision=ibs.IBS_FP64, mode="multigrid")
    try:
        B.launch()
        torch.cuda.synchronize()
        worst_h = worst_p = 0.0
        for j in B.jobs:
            got = [t.cpu().numpy() for t in j.outputs()]
            S = j.solver
            ref = [t.cpu().numpy() for t in S.helmholtz([0, 1, 2], [j.c] * 3, j.r)] + [S.poisson(j.b).cpu().numpy()]
            worst_h = max(worst_h, max(_maxrel(a, b) for a, b in zip(got[:3], ref[:3])))
            worst_p = max(worst_p, _maxrel(got[3], ref[3]))
            assert all(S.read_info(q).status == 0 for q in range(4))
        _say("c4 multigrid worst max-rel vs single-grid: helmholtz", worst_h, "poisson", worst_p)
        assert worst_h < 1e-12 and worst_p < 5e-12
    finally:
        B.close()


def test_multigrid_refuses_bad_jobs(mods):
    ibs, _ = mods
    _say("case multigrid refusals")
    S = ibs.Solver(32, 16, 32, precision=ibs.IBS_REFINED_BF16X3)
    b, x = S.empty(0), S.empty(0)
    with pytest.raises(ibs.IbsError) as e:
        ibs.ibs_batch_build_multigrid([S.poisson_job(b, x)])
    assert e.value.status == ibs.IBS_ERR_UNSUPPORTED
    P = ibs.Solver(32, 48, 32, precision=ibs.IBS_FP64, bc_y_vel=ibs.IBS_PERIODIC, bc_y_p=ibs.IBS_PERIODIC)
    with pytest.raises(ibs.IbsError) as e:
        ibs.ibs_batch_build_multigrid([P.poisson_job(P.empty(0), P.empty(0))])
    assert e.value.status == ibs.IBS_ERR_UNSUPPORTED
    F = ibs.Solver(32, 16, 32, precision=ibs.IBS_FP64)
    r = [F.empty(op) for op in (1, 2, 3)]
    xs = [F.empty(op) for op in (1, 2, 3)]
    shared = [F.helmholtz_job([0, 1, 2], [1e-3] * 3, r, xs), F.poisson_job(F.empty(0), F.empty(0))]
    with pytest.raises(ibs.IbsError) as e:
        ibs.ibs_batch_build_multigrid(shared)
    assert e.value.status == ibs.IBS_ERR_INVALID_ARG
    for s in (S, P, F):
        s.close()


def test_batch_auto_picks_a_form(mods):
    """mode="auto" times both forms on the device and keeps the faster; the
    kept batch's results match the single-grid FP64 solves."""
    ibs, batch = mods
    _say("case batch auto")
    specs = synth.batch_specs(12, seed=9, sizes=((32, 32, 32), (64, 48, 64)))
    B = batch.Batch(specs, precision=ibs.IBS_FP64, mode="auto", tune_reps=2)
    try:
        _say("auto kept", B.mode, "timings", B.timings)
        assert B.mode in ("graph", "multigrid") and set(B.timings) == {"graph", "multigrid"}
        assert B.timings[B.mode] == min(B.timings.values())
        B.launch()
        torch.cuda.synchronize()
        for j in B.jobs:
            got = [t.cpu().numpy() for t in j.outputs()]
            S = j.solver
            ref = [t.cpu().numpy() for t in S.helmholtz([0, 1, 2], [j.c] * 3, j.r)] + [S.poisson(j.b).cpu().numpy()]
            assert max(_maxrel(a, b) for a, b in zip(got, ref)) < 1e-12
    finally:
        B.close()
