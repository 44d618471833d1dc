"""The refined path scales its FP32 residuals by a power of two taken from
the first pass (no FP32 or bfloat16 value of a correction pass leaves their
exponent range, whatever the rhs's magnitude): right-hand sides from 1e-30
to 1e30 all converge to the FP64 path's result within tol, and no solve
reports success while missing it (a capped solve may report NOT_CONVERGED
at the extremes, never a wrong answer with status 0)."""
import sys

import numpy as np
import pytest

from paper_2406_19920_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ibs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2406_19920_amd import ibsolve
    return ibsolve


def _maxrel(a, b):
    return float((a - b).abs().max() / b.abs().max())


@pytest.mark.parametrize("bc", ["walls", "periodic_y"])
def test_refined_rhs_magnitudes(ibs, bc):
    n = 64
    kw = dict(beta=1.5)
    if bc == "periodic_y":
        kw.update(bc_y_vel=ibs.IBS_PERIODIC, bc_y_p=ibs.IBS_PERIODIC)
    R = ibs.Solver(n, n, n, precision=ibs.IBS_REFINED_BF16X3, **kw)
    F = ibs.Solver(n, n, n, precision=ibs.IBS_FP64, **kw)
    b0 = synth.device_normal((n, n, n), 3, "cuda")
    f0 = [synth.device_normal(R.shape(op), 10 + op, "cuda") for op in (1, 2, 3)]
    if bc == "walls":
        f0[1][:, 0, :] = 0
        f0[1][:, n, :] = 0
    c = 1e-4
    for sc in (1e-36, 1e-30, 1e-20, 1e-10, 1.0, 1e10, 1e20, 1e30, 1e35):
        print("case scale", sc, bc, flush=True)
        b = b0 * sc
        xr = R.poisson(b)
        ir = R.read_info()
        xf = F.poisson(b)
        fs = [f * sc for f in f0]
        hr = R.helmholtz([0, 1, 2], [c] * 3, fs)
        st = [R.read_info(q).status for q in range(3)]
        hf = F.helmholtz([0, 1, 2], [c] * 3, fs)
        torch.cuda.synchronize()
        ep = _maxrel(xr, xf)
        eh = [_maxrel(a, b_) for a, b_ in zip(hr, hf)]
        print(f"  poisson err {ep:.2e} status {ir.status} passes {ir.iters}; helmholtz {max(eh):.2e} {st}",
              flush=True)
        sys.stdout.flush()
        # never a wrong answer reported as converged
        assert ir.status in (0, ibs.IBS_ERR_NOT_CONVERGED)
        if ir.status == 0:
            assert ep < 1e-10
        for q in range(3):
            assert st[q] in (0, ibs.IBS_ERR_NOT_CONVERGED)
            if st[q] == 0:
                assert eh[q] < 1e-10
        # inside the FP32 exponent range with room to spare, every solve converges
        if 1e-30 <= sc <= 1e30:
            assert ir.status == 0 and all(s == 0 for s in st)
    R.close()
    F.close()


@pytest.mark.parametrize("n,beta", [(64, 4.0), (64, 7.0), (128, 4.0), (128, 7.0)])
def test_strong_stretching_manufactured(ibs, n, beta):
    """Strongly stretched walls, up to cells of 2e-7 of the height: both
    paths return the manufactured pressure (b = L_p x_true by the oracle's
    long-double stencil) to tol (refined) and to 1e-10 (FP64: its rounding
    grows with the condition number, 1e-10 of the solution at beta = 7),
    and a refined solve that stops reports success only when it met tol."""
    import oracle
    from oracle import OP_P
    print("case stretching", n, beta, flush=True)
    g = oracle.Grid(n, n, n, beta=beta)
    xt = synth.manufactured(n, n, n, seed=7)
    xt = xt - oracle.weighted_mean(g, OP_P, xt)
    r, _, _ = oracle.residual_ld(g, OP_P, 0.0, xt, np.zeros_like(xt))
    b = torch.from_numpy(-r).cuda()
    for prec, tol in ((ibs.IBS_REFINED_BF16X3, 1e-10), (ibs.IBS_FP64, 1e-10)):
        S = ibs.Solver(n, n, n, beta=beta, precision=prec)
        x = S.poisson(b).cpu().numpy()
        inf = S.read_info()
        d = x - xt
        err = max(np.linalg.norm(d) / np.linalg.norm(xt), np.abs(d).max() / np.abs(xt).max())
        print(f"  precision {prec}: err {err:.2e} status {inf.status} passes {inf.iters}", flush=True)
        assert inf.status == 0 and err < tol
        S.close()


def test_too_strong_stretching_refused(ibs):
    """Cells below 1e-7 of the height (beta = 10 at 64 cells: 1.8e-9) are
    refused at plan time on both paths."""
    for prec in (ibs.IBS_FP64, ibs.IBS_REFINED_BF16X3):
        with pytest.raises(ibs.IbsError) as e:
            ibs.solver_plan(ibs.make_desc(64, 64, 64, beta=10.0, precision=prec))
        assert e.value.status == ibs.IBS_ERR_UNSUPPORTED


def test_refined_nan_rhs_reports_failure(ibs):
    """A NaN in the right-hand side never comes back as a converged solve."""
    n = 32
    R = ibs.Solver(n, n, n, beta=1.0, precision=ibs.IBS_REFINED_BF16X3)
    print("case nan rhs", flush=True)
    b = synth.device_normal((n, n, n), 6, "cuda")
    b[3, 4, 5] = float("nan")
    R.poisson(b)
    torch.cuda.synchronize()
    assert R.read_info().status != 0
    R.close()
