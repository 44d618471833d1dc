"""GPU parity of inhomogeneous wall data (Section 2.3.3, subroutine BC2.2;
Appendix B's boundary terms): ibs_wall_data() then the homogeneous solve,
against the oracle's solve with the data in its flux form, on stretched
grids with seeded random data, both precisions, in l2 and max norm; and the
exact profiles (phi = y^2/2 with Neumann data on a uniform grid; u = y,
v = y with Dirichlet data on a stretched grid) recovered to round-off."""
import sys

import numpy as np
import pytest

import oracle
from oracle import OP_P, OP_U, OP_V, OP_W
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


def _rel(a, b):
    d = (a - b).ravel()
    return max(float(np.linalg.norm(d) / np.linalg.norm(b.ravel())),
               float(np.abs(d).max() / np.abs(b).max()))


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("refined", [False, True])
@pytest.mark.parametrize("shape,beta", [((64, 48, 32), 2.0), ((96, 33, 64), 1.0)])
def test_wall_data_vs_oracle(ibs, refined, shape, beta):
    nx, ny, nz = shape
    _say("case wall data", shape, beta, "refined" if refined else "fp64")
    g = oracle.Grid(nx, ny, nz, beta=beta)
    prec = ibs.IBS_REFINED_BF16X3 if refined else ibs.IBS_FP64
    tol = 1e-10 if refined else 1e-12
    S = ibs.Solver(nx, ny, nz, beta=beta, precision=prec)
    c = 0.125 * min(float(g.dyc.min()), 1.0 / nx) ** 2 * 50
    rng = np.random.default_rng(17)
    for op in (OP_P, OP_U, OP_V, OP_W):
        lo = rng.standard_normal(oracle.wall_shape(g))
        hi = rng.standard_normal(oracle.wall_shape(g))
        b = synth.scalar(nx, ny, nz, 40 + op, rows=ny + 1 if op == OP_V else None)
        cc = 0.0 if op == OP_P else c
        xo, _ = oracle.solve_bc(g, op, b, lo, hi, c=cc)
        rhs = _dev(b)
        S.wall_data(op, rhs, _dev(lo), _dev(hi), c=cc)
        if op == OP_P:
            xg = _host(S.poisson(rhs))
        else:
            (x,) = S.helmholtz([op - 1], [cc], [rhs])
            xg = _host(x)
            if op == OP_V:
                xg[:, 0, :] = lo
                xg[:, ny, :] = hi
        err = _rel(xg, xo)
        _say("op", op, "err", err, "status", S.read_info().status)
        assert err < tol


@pytest.mark.parametrize("refined", [False, True])
def test_wall_data_exact_profiles(ibs, refined):
    nx, ny, nz = 64, 40, 32
    prec = ibs.IBS_REFINED_BF16X3 if refined else ibs.IBS_FP64
    _say("case wall data exact profiles", "refined" if refined else "fp64")
    # Neumann data dphi/dy = y on a uniform grid: phi = y^2/2 solves L_p phi = 1
    g = oracle.Grid(nx, ny, nz)
    S = ibs.Solver(nx, ny, nz, precision=prec)
    phi = np.broadcast_to((g.yc ** 2 / 2)[None, :, None], g.shape(OP_P)).copy()
    phi -= oracle.weighted_mean(g, OP_P, phi)
    rhs = _dev(np.ones(g.shape(OP_P)))
    S.wall_data(OP_P, rhs, None, _dev(np.ones(oracle.wall_shape(g))))
    err = _rel(_host(S.poisson(rhs)), phi)
    _say("poisson y^2/2 err", err)
    assert err < 1e-10
    # Dirichlet data g = y on a stretched grid: u = y (cell centres), v = y
    # (faces) satisfy (I - cL) f = f
    gs = oracle.Grid(nx, ny, nz, beta=2.0)
    S2 = ibs.Solver(nx, ny, nz, beta=2.0, precision=prec)
    c = 1e-4
    for op, prof in ((OP_U, gs.yc), (OP_V, gs.yf), (OP_W, gs.yc)):
        f = np.broadcast_to(prof[None, :, None], gs.shape(op)).copy()
        rhs = _dev(f)
        S2.wall_data(op, rhs, None, _dev(np.ones(oracle.wall_shape(gs))), c=c)
        (x,) = S2.helmholtz([op - 1], [c], [rhs])
        xg = _host(x)
        if op == OP_V:
            xg[:, ny, :] = 1.0
        err = _rel(xg, f)
        _say("op", op, "linear profile err", err)
        assert err < 1e-10
