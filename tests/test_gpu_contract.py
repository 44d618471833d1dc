"""GPU checks of the C ABI's contracts: the one-pass report, the strict
compatibility check (FP64, on b itself) on both paths, concurrent solves on
one plan with separate workspaces, and the residual's workspace."""
import sys

import numpy as np
import pytest

import oracle
from oracle import OP_P
from paper_2406_19920_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ibs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2406_19920_amd import ibsolve
    return ibsolve


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _rel(a, b):
    d = (a - b).ravel()
    return max(float(np.linalg.norm(d) / np.linalg.norm(b.ravel())),
               float(np.abs(d).max() / np.abs(b).max()))


def test_refined_one_pass_reports_not_converged(ibs):
    """A single refined pass measures no correction: the report is
    NOT_CONVERGED with NaN estimates, whatever the tolerance, for both
    solve kinds."""
    n = 32
    _say("case one pass")
    b = synth.scalar(n, n, n, 3)
    for tol in (1e-10, 1e-3):
        S = ibs.Solver(n, n, n, beta=1.0, precision=ibs.IBS_REFINED_BF16X3, max_iter=1, tol=tol)
        S.poisson(_dev(b))
        inf = S.read_info()
        assert inf.status == ibs.IBS_ERR_NOT_CONVERGED and inf.iters == 1
        assert np.isnan(inf.rel_residual) and np.isnan(inf.rel_correction)
        u, v, w = synth.velocity(n, n, n, seed=4)
        S.helmholtz([0, 1, 2], [1e-3] * 3, [_dev(u), _dev(v), _dev(w)])
        for q in range(3):
            inf = S.read_info(q)
            assert inf.status == ibs.IBS_ERR_NOT_CONVERGED and inf.iters == 1
            assert np.isnan(inf.rel_residual)
        S.close()


@pytest.mark.parametrize("refined", [False, True])
def test_strict_compat(ibs, refined):
    """strict_compat: the divergence of a velocity field with no wall flux is
    compatible (status OK); the same rhs plus a constant is flagged
    INCOMPATIBLE_RHS, and the solve still returns the projected solution."""
    nx, ny, nz = 64, 48, 32
    _say("case strict compat", refined)
    g = oracle.Grid(nx, ny, nz, beta=2.0)
    u, v, w = synth.velocity(nx, ny, nz, seed=8)
    v[:, 0, :] = 0
    v[:, ny, :] = 0
    b = oracle.divergence(g, u, v, w)
    prec = ibs.IBS_REFINED_BF16X3 if refined else ibs.IBS_FP64
    tol = 1e-10 if refined else 1e-12
    S = ibs.Solver(nx, ny, nz, beta=2.0, precision=prec, strict_compat=1)
    xo, _ = oracle.solve(g, OP_P, b)
    xg = _host(S.poisson(_dev(b)))
    inf = S.read_info()
    _say("compatible: status", inf.status, "err", _rel(xg, xo))
    assert inf.status == ibs.IBS_OK
    assert _rel(xg, xo) < tol
    bs = b + 0.25 * np.abs(b).max()
    xg = _host(S.poisson(_dev(bs)))
    inf = S.read_info()
    _say("shifted: status", inf.status, "removed", inf.removed_mean)
    assert inf.status == ibs.IBS_ERR_INCOMPATIBLE_RHS
    assert _rel(xg, xo) < tol
    # without the flag the shifted rhs is projected silently
    S2 = ibs.Solver(nx, ny, nz, beta=2.0, precision=prec)
    xg = _host(S2.poisson(_dev(bs)))
    assert S2.read_info().status == ibs.IBS_OK
    assert _rel(xg, xo) < tol


@pytest.mark.parametrize("refined", [False, True])
def test_concurrent_solves_share_one_plan(ibs, refined):
    """The plan's device constants are read-only: solves on one plan on two
    streams with two workspaces run side by side and give the bits each
    gives alone."""
    nx, ny, nz = 96, 40, 64
    _say("case concurrent", refined)
    prec = ibs.IBS_REFINED_BF16X3 if refined else ibs.IBS_FP64
    S = ibs.Solver(nx, ny, nz, beta=1.5, precision=prec)
    bs = [_dev(synth.scalar(nx, ny, nz, 30 + q)) for q in range(4)]
    alone = [_host(S.poisson(b)).copy() for b in bs]
    works = [torch.empty(S.work_bytes, dtype=torch.uint8, device="cuda") for _ in range(2)]
    infos = torch.zeros((2, 8), dtype=torch.float64, device="cuda")
    streams = [torch.cuda.Stream() for _ in range(2)]
    outs = [S.empty() for _ in bs]
    torch.cuda.synchronize()
    for rep in range(2):
        for q, b in enumerate(bs):
            lane = q % 2
            with torch.cuda.stream(streams[lane]):
                ibs.solve_poisson(S.plan, b.data_ptr(), outs[q].data_ptr(), works[lane].data_ptr(),
                                  S.work_bytes, infos[lane].data_ptr(),
                                  streams[lane].cuda_stream)
        torch.cuda.synchronize()
        for q in range(len(bs)):
            np.testing.assert_array_equal(_host(outs[q]), alone[q], err_msg=f"rhs {q} rep {rep}")


def test_residual_needs_workspace_for_norms(ibs):
    nx, ny, nz = 32, 24, 16
    S = ibs.Solver(nx, ny, nz, beta=1.0)
    x = _dev(synth.scalar(nx, ny, nz, 1))
    b = _dev(synth.scalar(nx, ny, nz, 2))
    r = S.empty()
    with pytest.raises(ibs.IbsError) as e:
        ibs.residual(S.plan, 0, 0.0, x.data_ptr(), b.data_ptr(), r.data_ptr(),
                     torch.zeros(2, dtype=torch.float64, device="cuda").data_ptr(), None, 0,
                     S.stream())
    assert e.value.status == ibs.IBS_ERR_INVALID_ARG
    # without norms no workspace is read
    ibs.residual(S.plan, 0, 0.0, x.data_ptr(), b.data_ptr(), r.data_ptr(), None, None, 0,
                 S.stream())
    r2, n2 = S.residual(0, 0.0, x, b, norms=True)
    np.testing.assert_array_equal(_host(r), _host(r2))
    assert np.isclose(np.sqrt(_host(n2)[0]), np.linalg.norm(_host(r2)), rtol=1e-13)
