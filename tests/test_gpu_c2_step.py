"""The benchmark's own 256^3 step, in the launch configuration bench.py
times (refined, two passes; FP64 beside it), checked against the oracle:
the three Helmholtz solutions element by element (the oracle solves them at
full size in seconds), and for the pressure, whose oracle solve at 256^3
takes minutes, the properties that hold at any size: the divergence of the
GPU's u* equals the oracle's, the oracle's long-double residual of the GPU's
phi is at the level the tolerance implies, phi has zero weighted mean, the
correction equals u* - G phi with the oracle's gradient, and the corrected
field is divergence-free."""
import sys

import numpy as np
import pytest

import bench
import oracle
from oracle import OP_P, OP_U, OP_V, OP_W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _rel(a, b):
    d = (a - b).ravel()
    return max(float(np.linalg.norm(d) / np.linalg.norm(b.ravel())),
               float(np.abs(d).max() / np.abs(b).max()))


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("refined", [True, False])
def test_c2_bench_step_vs_oracle(refined):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2406_19920_amd import ibsolve as ibs
    n, beta = 256, 2.0
    _say("case c2 bench step", "refined" if refined else "fp64")
    u, v, w = bench.make_inputs(n, beta, seed=2)
    c = 0.125 * bench.h_min(n, beta) ** 2
    kw = {"max_iter": 2} if refined else {}
    S = ibs.Solver(n, n, n, beta=beta, precision=ibs.IBS_REFINED_BF16X3 if refined else ibs.IBS_FP64, **kw)
    ru, rv, rw = (torch.from_numpy(a).cuda() for a in (u, v, w))
    xu, xv, xw = S.empty(1), S.empty(2), S.empty(3)
    b, phi = S.empty(0), S.empty(0)
    S.helmholtz([0, 1, 2], [c, c, c], [ru, rv, rw], [xu, xv, xw], info_slot=1)
    S.divergence(xu, xv, xw, 1.0, b)
    S.poisson(b, phi)
    torch.cuda.synchronize()
    us = [t.cpu().numpy() for t in (xu, xv, xw)]
    bg, pg = b.cpu().numpy(), phi.cpu().numpy()
    S.correct(phi, xu, xv, xw, 1.0)
    torch.cuda.synchronize()
    un = [t.cpu().numpy() for t in (xu, xv, xw)]
    for q in range(4):
        assert S.read_info(q).status == 0
    tol = 1e-10 if refined else 1e-12
    g = oracle.Grid(n, n, n, beta=beta)
    # Helmholtz, element by element
    for q, (op, f) in enumerate(zip((OP_U, OP_V, OP_W), (u, v, w))):
        ref, _ = oracle.solve(g, op, f, c=c)
        err = _rel(us[q], ref)
        _say("helmholtz", q, "err", err)
        assert err < tol
    # the divergence of the GPU's u*
    bo = oracle.divergence(g, *us)
    assert np.abs(bg - bo).max() <= 1e-14 * np.abs(bo).max()
    # pressure: residual of the GPU's phi (the weighted mean of b removed,
    # as the solve does), zero weighted mean
    bc = bo - oracle.weighted_mean(g, OP_P, bo)
    r, rn, bn = oracle.residual_ld(g, OP_P, 0.0, pg, bc)
    _say("poisson residual", rn / bn, "mean", oracle.weighted_mean(g, OP_P, pg))
    assert rn / bn < (1e-8 if refined else 1e-11)
    assert abs(oracle.weighted_mean(g, OP_P, pg)) < 1e-12 * np.abs(pg).max()
    # projection: u^n = u* - G phi, divergence-free
    gu, gv, gw = oracle.gradient(g, pg)
    for got, ref in zip(un, (us[0] - gu, us[1] - gv, us[2] - gw)):
        assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()
    d1 = oracle.divergence(g, *un)
    _say("divergence after projection", np.abs(d1).max() / np.abs(bo).max())
    assert np.abs(d1).max() <= (1e-8 if refined else 1e-11) * np.abs(bo).max()
