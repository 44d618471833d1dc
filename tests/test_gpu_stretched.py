"""GPU parity on stretched wall-bounded x and z (the generalised eigenbases of
the flux-form operators), against the oracle, both precisions, in l2 and max
norm: solves on several shapes (x, z or both stretched; randomly graded and
tanh faces; periodic y), manufactured solutions in a 192 x 128 x 192
stretched duct, the stencils over the local widths, and the strict
compatibility check with the stretched volume weights."""
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


def _random_faces(n, length, seed):
    w = np.random.default_rng(seed).uniform(0.5, 2.0, n)
    f = np.concatenate([[0.0], np.cumsum(w)])
    return f * (length / f[-1])


def _tanh_faces(n, length, beta):
    j = np.arange(n + 1)
    return 0.5 * length * (1 + np.tanh(beta * (2 * j / n - 1)) / np.tanh(beta))


def _setup(ibs, nx, ny, nz, beta, sx, sz, refined, py=False, wx=True, wz=True):
    """(oracle grid, solver) with x / z stretched as asked (random faces in
    x, tanh faces in z) and walls along every stretched axis."""
    xf = _random_faces(nx, 1.1, nx) if sx else None
    zf = _tanh_faces(nz, 0.9, 1.3) if sz else None
    wx, wz = wx or sx, wz or sz
    kw = dict(beta=beta)
    if py:
        kw.update(bc_y_vel=ibs.IBS_PERIODIC, bc_y_p=ibs.IBS_PERIODIC)
    if wx:
        kw["bc_x"] = ibs.IBS_DIRICHLET
    if wz:
        kw["bc_z"] = ibs.IBS_DIRICHLET
    prec = ibs.IBS_REFINED_BF16X3 if refined else ibs.IBS_FP64
    S = ibs.Solver(nx, ny, nz, precision=prec, x_faces=xf, z_faces=zf, lx=1.1, lz=0.9, **kw)
    g = oracle.Grid(nx, ny, nz, lx=1.1, lz=0.9, beta=beta, periodic_y=py, periodic_x=not wx,
                    periodic_z=not wz, xf_in=xf, zf_in=zf)
    return g, S


# (shape, beta, stretched x, stretched z, periodic y, refined)
CASES = [(s, b, sx, sz, py, rf) for (s, b, sx, sz, py) in (((64, 48, 32), 1.5, True, False, False),
                                                           ((32, 40, 64), 2.0, False, True, False),
                                                           ((64, 32, 64), 1.0, True, True, False),
                                                           ((64, 48, 64), 0.0, True, True, True))
         for rf in (False, True)] + [((48, 20, 80), 1.0, True, True, False, False),
                                     ((16, 33, 48), 0.5, False, True, False, False)]


@pytest.mark.parametrize("shape,beta,sx,sz,py,refined", CASES)
def test_stretched_vs_oracle(ibs, shape, beta, sx, sz, py, refined):
    nx, ny, nz = shape
    _say("case stretched", shape, beta, "sx" if sx else "", "sz" if sz else "", "py" if py else "",
         "refined" if refined else "fp64")
    tol = 1e-10 if refined else 1e-12
    g, S = _setup(ibs, nx, ny, nz, beta, sx, sz, refined, py)
    b = synth.scalar(nx, ny, nz, 75)
    xo, info = oracle.solve(g, OP_P, b)
    err = _rel(_host(S.poisson(_dev(b))), xo)
    inf = S.read_info()
    _say("poisson err", err, "passes", inf.iters, "status", inf.status)
    assert err < tol and inf.status == 0
    hmin = min(float(g.dyc.min()), float(g.dxc.min()), float(g.dzc.min()))
    c = 0.125 * hmin ** 2 * 20
    fs = [synth.scalar(nx, ny, nz, 76 + q, rows=ny + 1 if (q == 1 and not py) else None) for q in range(3)]
    if not py:
        fs[1][:, 0, :] = 0
        fs[1][:, ny, :] = 0
    refs = [oracle.solve(g, op, f, c=c)[0] for op, f in zip((OP_U, OP_V, OP_W), fs)]
    xs = S.helmholtz([0, 1, 2], [c] * 3, [_dev(f) for f in fs])
    for q, (x, ref) in enumerate(zip(xs, refs)):
        got = _host(x)
        err = _rel(got, ref)
        _say("comp", q, "err", err, "status", S.read_info(q).status)
        assert err < tol and S.read_info(q).status == 0
        if q == 0:
            assert np.all(got[:, :, 0] == 0)
        if q == 2:
            assert np.all(got[0] == 0)


@pytest.mark.parametrize("refined", [False, True])
def test_stretched_duct_manufactured(ibs, refined):
    """A 192 x 128 x 192 duct stretched in x, y and z: manufactured
    solutions for the pressure and all three components."""
    nx, ny, nz = 192, 128, 192
    _say("case stretched duct manufactured", refined)
    g, S = _setup(ibs, nx, ny, nz, 2.0, True, True, refined)
    tol = 1e-10 if refined else 1e-12
    xt = synth.manufactured(nx, ny, nz, seed=101)
    xt = xt - oracle.weighted_mean(g, OP_P, xt)
    r, _, _ = oracle.residual_ld(g, OP_P, 0.0, xt, np.zeros_like(xt))
    err = _rel(_host(S.poisson(_dev(-r))), xt)
    _say("poisson err", err, "passes", S.read_info().iters)
    assert err < tol and S.read_info().status == 0
    c = 0.125 * min(float(g.dyc.min()), float(g.dxc.min()), float(g.dzc.min())) ** 2 * 4
    xts, rhs = [], []
    for q, op in enumerate((OP_U, OP_V, OP_W)):
        t = synth.manufactured(nx, ny, nz, seed=102 + q, rows=ny + 1 if op == OP_V else None)
        if op == OP_V:
            t[:, 0, :] = 0
            t[:, ny, :] = 0
        if op == OP_U:
            t[:, :, 0] = 0
        if op == OP_W:
            t[0] = 0
        rr, _, _ = oracle.residual_ld(g, op, c, t, np.zeros_like(t))
        xts.append(t)
        rhs.append(-rr)
    xs = S.helmholtz([0, 1, 2], [c] * 3, [_dev(f) for f in rhs])
    for q in range(3):
        err = _rel(_host(xs[q]), xts[q])
        _say("helmholtz", q, "err", err, "passes", S.read_info(q).iters)
        assert err < tol and S.read_info(q).status == 0


@pytest.mark.parametrize("sx,sz", [(True, False), (False, True), (True, True)])
def test_stretched_stencils_and_projection(ibs, sx, sz):
    nx, ny, nz = 64, 40, 48
    _say("case stretched stencils", sx, sz)
    g, S = _setup(ibs, nx, ny, nz, 1.0, sx, sz, False)
    u, w = synth.scalar(nx, ny, nz, 131), synth.scalar(nx, ny, nz, 133)
    v = synth.scalar(nx, ny, nz, 132, rows=ny + 1)
    v[:, 0, :] = 0
    v[:, ny, :] = 0
    w[0] = 3.0                   # the wall planes: ignored by the divergence
    u[:, :, 0] = 4.0
    ud, vd, wd = _dev(u), _dev(v), _dev(w)
    b = S.divergence(ud, vd, wd, scale=2.0)
    bo = oracle.divergence(g, u, v, w, scale=2.0)
    assert np.abs(_host(b) - bo).max() < 1e-14 * np.abs(bo).max()
    phi = S.poisson(b)
    S.correct(phi, ud, vd, wd, 0.5)
    gu, gv, gw = oracle.gradient(g, _host(phi))
    w[0] = 0.0
    u[:, :, 0] = 0.0
    for got, ref in ((ud, u - 0.5 * gu), (vd, v - 0.5 * gv), (wd, w - 0.5 * gw)):
        assert np.abs(_host(got) - ref).max() < 1e-13 * np.abs(ref).max()
    d1 = _host(S.divergence(ud, vd, wd))
    assert np.abs(d1).max() < 1e-12 * np.abs(bo).max() / 2.0
    for op in (0, 1, 2, 3):
        c = 0.0 if op == 0 else 1e-3
        x = synth.scalar(nx, ny, nz, 140 + op, rows=ny + 1 if op == 2 else None)
        if op == 3:
            x[0] = 0.0
        if op == 1:
            x[:, :, 0] = 0.0
        bb = synth.scalar(nx, ny, nz, 150 + op, rows=ny + 1 if op == 2 else None)
        r, n2 = S.residual(op, c, _dev(x), _dev(bb), norms=True)
        ref, rn, _ = oracle.residual_ld(g, op, c, x, bb)
        got = _host(r)
        assert np.abs(got - ref).max() < 1e-12 * np.abs(ref).max(), op
        assert abs(np.sqrt(_host(n2)[0]) - rn) < 1e-12 * rn


@pytest.mark.parametrize("refined", [False, True])
def test_stretched_strict_compat(ibs, refined):
    """The compatibility check weighs b by the stretched control volumes: the
    divergence of a field with no wall flux is compatible (its volume-
    weighted mean vanishes to rounding although its plain mean does not),
    and the same b shifted by a constant is flagged."""
    nx, ny, nz = 64, 32, 64
    _say("case stretched compat", refined)
    xf = _random_faces(nx, 1.1, 7)
    zf = _tanh_faces(nz, 0.9, 1.6)
    prec = ibs.IBS_REFINED_BF16X3 if refined else ibs.IBS_FP64
    S = ibs.Solver(nx, ny, nz, beta=1.0, precision=prec, bc_x=ibs.IBS_DIRICHLET, bc_z=ibs.IBS_DIRICHLET,
                   x_faces=xf, z_faces=zf, strict_compat=1)
    g = oracle.Grid(nx, ny, nz, lx=1.1, lz=0.9, beta=1.0, periodic_x=False, periodic_z=False,
                    xf_in=xf, zf_in=zf)
    u, v, w = synth.velocity(nx, ny, nz, seed=8)
    v[:, 0, :] = 0
    v[:, ny, :] = 0
    u[:, :, 0] = 0
    w[0] = 0
    b = oracle.divergence(g, u, v, w)
    assert abs(b.mean()) > 1e-6 * np.abs(b).std()     # the plain mean is not zero
    S.poisson(_dev(b))
    assert S.read_info().status == 0
    S.poisson(_dev(b + 0.01 * np.abs(b).std()))
    assert S.read_info().status == ibs.IBS_ERR_INCOMPATIBLE_RHS
