"""Batched multi-grid execution replayed as one HIP graph: every result of
the batch equals the same job run alone (bitwise: fixed tiles and reduction
orders, no atomics), on every replay, with eager work between replays; one
job is also checked against the oracle."""
import sys

import numpy as np
import pytest

import oracle
from oracle import OP_P

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mods():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2406_19920_amd import batch, ibsolve
    return batch, ibsolve


SPECS = [dict(nx=32, ny=24, nz=32, beta=0.5, seed=1000),
         dict(nx=64, ny=40, nz=32, beta=2.5, seed=1001),
         dict(nx=32, ny=17, nz=64, beta=1.0, seed=1002),
         dict(nx=96, ny=33, nz=32, beta=3.0, seed=1003),
         dict(nx=32, ny=32, nz=32, beta=0.0, seed=1004)]


@pytest.mark.parametrize("refined", [True, False])
def test_batch_equals_alone(mods, refined):
    batch, ibs = mods
    prec = ibs.IBS_REFINED_BF16X3 if refined else ibs.IBS_FP64
    print("case batch refined" if refined else "case batch fp64", flush=True)
    alone = []
    for s in SPECS:
        j = batch.Job(s, prec, "cuda")
        j.run_eager()
        torch.cuda.synchronize()
        alone.append([o.cpu().numpy() for o in j.outputs()])
        j.solver.close()
    B = batch.Batch(SPECS, precision=prec, nlanes=3)
    for rep in range(3):
        for j in B.jobs:
            for o in j.outputs():
                o.fill_(float("nan"))
        B.launch()
        torch.cuda.synchronize()
        for q, (j, ref) in enumerate(zip(B.jobs, alone)):
            for o, r in zip(j.outputs(), ref):
                np.testing.assert_array_equal(o.cpu().numpy(), r, err_msg=f"job {q} replay {rep}")
        # eager work between replays
        x = torch.randn(1 << 20, device="cuda", dtype=torch.float64)
        float(x.sum())
    # one job against the oracle
    j = B.jobs[1]
    s = j.spec
    g = oracle.Grid(s["nx"], s["ny"], s["nz"], beta=s["beta"])
    xo, _ = oracle.solve(g, OP_P, j.b.cpu().numpy())
    err = np.linalg.norm(j.phi.cpu().numpy() - xo) / np.linalg.norm(xo)
    print("batch job oracle err", err, flush=True)
    assert err < (1e-10 if refined else 1e-12)
    B.close()


def test_batch_rejects_bad_job(mods):
    batch, ibs = mods
    rec = ibs.ibs_batch_job()
    rec.plan = None
    with pytest.raises(ibs.IbsError) as e:
        ibs.ibs_batch_build([rec], 2)
    assert e.value.status == ibs.IBS_ERR_INVALID_ARG


def _rel(a, b):
    d = (a - b).ravel()
    return max(float(np.linalg.norm(d) / np.linalg.norm(b.ravel())),
               float(np.abs(d).max() / np.abs(b).max()))


@pytest.mark.parametrize("refined", [True, False])
def test_batch_mixed_sizes_manufactured(mods, refined):
    """Jobs at the mixed-size batch's own grid sizes (96x128x96 and
    192x256x192, stretched), replayed as one graph: all four solves of each
    job (u, v, w Helmholtz and Poisson) return the manufactured solutions
    (x_true seeded; b = A x_true formed by the oracle's long-double stencil
    on the CPU), in l2 and max norm."""
    from oracle import OP_U, OP_V, OP_W
    from paper_2406_19920_amd import synth
    batch, ibs = mods
    prec = ibs.IBS_REFINED_BF16X3 if refined else ibs.IBS_FP64
    tol = 1e-10 if refined else 1e-12
    specs = [dict(nx=96, ny=128, nz=96, beta=1.2, seed=1100),
             dict(nx=192, ny=256, nz=192, beta=2.4, seed=1101),
             dict(nx=64, ny=64, nz=64, beta=0.3, seed=1102)]
    print("case batch mixed sizes manufactured", refined, flush=True)
    B = batch.Batch(specs, precision=prec, nlanes=3)
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
            print("job", q, j.spec["nx"], j.spec["ny"], "solve", k, "err", err, flush=True)
            assert err < tol
        for k in range(4):
            assert j.solver.read_info(k).status == 0
    B.close()


@pytest.mark.parametrize("refined", [True, False])
def test_batch_boundary_kinds(mods, refined):
    """Jobs with walls in y, periodic y and walls in x in one graph: each
    equals the same job run alone (bitwise) and all four solves match the
    oracle (l2 and max norm)."""
    from oracle import OP_U, OP_V, OP_W
    batch, ibs = mods
    prec = ibs.IBS_REFINED_BF16X3 if refined else ibs.IBS_FP64
    tol = 1e-10 if refined else 1e-12
    specs = [dict(nx=64, ny=48, nz=32, beta=0.0, seed=1200, bc="periodic_y"),
             dict(nx=64, ny=40, nz=32, beta=1.5, seed=1201, bc="walls_x"),
             dict(nx=32, ny=24, nz=64, beta=2.0, seed=1202, bc="walls"),
             dict(nx=32, ny=64, nz=32, beta=1.0, seed=1203, bc="walls_x")]
    print("case batch boundary kinds", refined, flush=True)
    B = batch.Batch(specs, precision=prec, nlanes=3)
    alone = []
    for j in B.jobs:
        j.run_eager()
        torch.cuda.synchronize()
        alone.append([o.cpu().numpy().copy() for o in j.outputs()])
    for rep in range(2):
        for j in B.jobs:
            for o in j.outputs():
                o.fill_(float("nan"))
        B.launch()
        torch.cuda.synchronize()
        for q, j in enumerate(B.jobs):
            for a, o in zip(alone[q], j.outputs()):
                np.testing.assert_array_equal(o.cpu().numpy(), a, err_msg=f"job {q} replay {rep}")
    for q, j in enumerate(B.jobs):
        s = j.spec
        g = oracle.Grid(s["nx"], s["ny"], s["nz"], beta=s["beta"], periodic_y=s["bc"] == "periodic_y",
                        periodic_x=s["bc"] != "walls_x")
        outs = j.outputs()
        for k, op in enumerate((OP_U, OP_V, OP_W)):
            ref, _ = oracle.solve(g, op, j.r[k].cpu().numpy(), c=j.c)
            err = _rel(outs[k].cpu().numpy(), ref)
            print("job", q, s["bc"], "comp", k, "err", err, flush=True)
            assert err < tol
        ref, _ = oracle.solve(g, OP_P, j.b.cpu().numpy())
        err = _rel(outs[3].cpu().numpy(), ref)
        print("job", q, s["bc"], "poisson err", err, flush=True)
        assert err < tol
        for k in range(4):
            assert j.solver.read_info(k).status == 0
    B.close()


def test_schedule_autotuner(mods):
    """The schedule autotuner returns a valid (lanes, policy) and a batch
    built with it reproduces every job bitwise (each job's launches run in
    the same order on its own workspace, whatever the schedule)."""
    batch, ibs = mods
    print("case batch schedule autotuner", flush=True)
    B0 = batch.Batch(SPECS, precision=ibs.IBS_REFINED_BF16X3, nlanes=1)
    B0.launch()
    torch.cuda.synchronize()
    ref = [[o.cpu().numpy().copy() for o in j.outputs()] for j in B0.jobs]
    B0.close()
    B = batch.Batch(SPECS, precision=ibs.IBS_REFINED_BF16X3, nlanes="auto")
    nl, pol, ms = B.schedule
    print("schedule", B.schedule, flush=True)
    assert 1 <= nl <= len(SPECS) and pol in (ibs.IBS_SCHED_BALANCED, ibs.IBS_SCHED_IN_ORDER) and ms > 0
    for j in B.jobs:
        for o in j.outputs():
            o.fill_(float("nan"))
    B.launch()
    torch.cuda.synchronize()
    for q, j in enumerate(B.jobs):
        for a, o in zip(ref[q], j.outputs()):
            np.testing.assert_array_equal(o.cpu().numpy(), a)
    # both policies at the largest lane count give the same results too
    for policy in (ibs.IBS_SCHED_BALANCED, ibs.IBS_SCHED_IN_ORDER):
        B2 = batch.Batch(SPECS, precision=ibs.IBS_REFINED_BF16X3, nlanes=len(SPECS), policy=policy)
        B2.launch()
        torch.cuda.synchronize()
        for q, j in enumerate(B2.jobs):
            for a, o in zip(ref[q], j.outputs()):
                np.testing.assert_array_equal(o.cpu().numpy(), a)
        B2.close()
    B.close()
