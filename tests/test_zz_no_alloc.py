"""The allocation-free Poisson entry point (library-held scratch instead of
a workspace argument): through the C ABI, two calls in a row, the second on
a smaller grid, each bitwise equal to solve_poisson() on the same input with
a caller workspace; oversize grids are refused before anything runs."""
import numpy as np
import pytest

import oracle
from oracle import OP_P
from paper_2406_19920_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("refined", [False, True])
def test_noalloc_matches_workspace_entry(refined):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2406_19920_amd import ibsolve as ibs
    prec = ibs.IBS_REFINED_BF16X3 if refined else ibs.IBS_FP64
    print("case noalloc", "refined" if refined else "fp64", flush=True)
    # second call smaller than the first, and both within the scratch
    for (nx, ny, nz), beta, seed in (((128, 96, 128), 2.0, 3), ((64, 40, 32), 1.0, 4)):
        S = ibs.Solver(nx, ny, nz, beta=beta, precision=prec)
        assert S.work_p <= ibs.IBS_NOALLOC_SCRATCH_BYTES
        b = synth.scalar(nx, ny, nz, seed)
        bd = torch.from_numpy(b).to("cuda")
        ref = S.poisson(bd)
        info_ref = S.read_info(0)
        phi = torch.full_like(bd, float("nan"))
        info = torch.zeros(8, dtype=torch.float64, device="cuda")
        ibs.solve_poisson_noalloc(S.plan, bd.data_ptr(), phi.data_ptr(), info.data_ptr(), S.stream())
        torch.cuda.synchronize()
        np.testing.assert_array_equal(phi.cpu().numpy(), ref.cpu().numpy())
        raw = info.cpu().numpy().tobytes()[:ibs.INFO_BYTES]
        inf = ibs.ibs_solve_info.from_buffer_copy(raw)
        assert inf.status == info_ref.status == 0 and inf.iters == info_ref.iters
        # and against the oracle, in l2 and max norm
        g = oracle.Grid(nx, ny, nz, beta=beta)
        xo, _ = oracle.solve(g, OP_P, b)
        got = phi.cpu().numpy()
        d = (got - xo).ravel()
        err = max(np.linalg.norm(d) / np.linalg.norm(xo), np.abs(d).max() / np.abs(xo).max())
        print("grid", (nx, ny, nz), "err", err, flush=True)
        assert err < (1e-10 if refined else 1e-12)
        S.close()


@pytest.mark.parametrize("refined", [False, True])
def test_noalloc_boundary_kinds(refined):
    """Periodic y and walls in x through the allocation-free entry point:
    bitwise equal to solve_poisson() with a workspace, two calls in a row
    (the second smaller)."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2406_19920_amd import ibsolve as ibs
    prec = ibs.IBS_REFINED_BF16X3 if refined else ibs.IBS_FP64
    print("case noalloc boundary kinds", "refined" if refined else "fp64", flush=True)
    cases = (((96, 64, 64), dict(bc_y_vel=ibs.IBS_PERIODIC, bc_y_p=ibs.IBS_PERIODIC), 5),
             ((64, 40, 32), dict(bc_x=ibs.IBS_DIRICHLET, beta=1.5), 6))
    for (nx, ny, nz), kw, seed in cases:
        S = ibs.Solver(nx, ny, nz, precision=prec, **kw)
        assert S.work_p <= ibs.IBS_NOALLOC_SCRATCH_BYTES
        bd = torch.from_numpy(synth.scalar(nx, ny, nz, seed)).to("cuda")
        ref = S.poisson(bd)
        phi = torch.full_like(bd, float("nan"))
        info = torch.zeros(8, dtype=torch.float64, device="cuda")
        ibs.solve_poisson_noalloc(S.plan, bd.data_ptr(), phi.data_ptr(), info.data_ptr(), S.stream())
        torch.cuda.synchronize()
        np.testing.assert_array_equal(phi.cpu().numpy(), ref.cpu().numpy())
        inf = ibs.ibs_solve_info.from_buffer_copy(info.cpu().numpy().tobytes()[:ibs.INFO_BYTES])
        assert inf.status == 0
        S.close()


def test_noalloc_refuses_oversize_grid():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2406_19920_amd import ibsolve as ibs
    S = ibs.Solver(256, 256, 256, precision=ibs.IBS_FP64)
    assert S.work_p > ibs.IBS_NOALLOC_SCRATCH_BYTES
    b = S.empty()
    with pytest.raises(ibs.IbsError) as e:
        ibs.solve_poisson_noalloc(S.plan, b.data_ptr(), b.data_ptr(), None, S.stream())
    assert e.value.status == ibs.IBS_ERR_WORKSPACE_TOO_SMALL
    S.close()
