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
