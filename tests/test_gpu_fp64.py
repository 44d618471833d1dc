"""GPU parity of the FP64 path against the oracle (through the C ABI).

Tolerance: 1e-12 relative, both in l2 over all unknowns and in max norm
(max|x - x_ref| / max|x_ref|), after fixing the Poisson null mode to zero
weighted mean on both sides.
"""
import sys

import numpy as np
import pytest

import oracle
from oracle import OP_P, OP_U, OP_V, OP_W
from paper_2406_19920_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-12


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
    """Larger of the relative l2 error over all unknowns and the relative
    max-norm error max|a - b| / max|b| (both must meet the tolerance)."""
    d = (a - b).ravel()
    l2 = float(np.linalg.norm(d) / np.linalg.norm(b.ravel()))
    linf = float(np.abs(d).max() / np.abs(b).max())
    return max(l2, linf)


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_c1_poisson_64cube(ibs):
    """64^3 uniform grid, RHS = divergence of seeded N(0,1) face velocities
    (wall v included, so the mean must be removed), one FP64 solve."""
    n = 64
    _say("case c1 poisson 64^3")
    g = oracle.Grid(n, n, n)
    u, v, w = synth.velocity(n, n, n, seed=1)
    b = oracle.divergence(g, u, v, w)
    xo, info = oracle.solve(g, OP_P, b)
    S = ibs.Solver(n, n, n)
    bd = S.divergence(_dev(u), _dev(v), _dev(w))
    bg = _host(bd)
    assert _rel(bg, b) < 1e-14
    phi = S.poisson(bd)
    xg = _host(phi)
    err = _rel(xg, xo)
    _say("c1 rel err", err)
    assert err < TOL
    inf = S.read_info()
    assert inf.status == 0 and inf.iters == 1
    assert abs(inf.removed_mean - info.removed_mean) < 1e-12 * np.abs(b).max()
    assert abs(oracle.weighted_mean(g, OP_P, xg)) < 1e-14 * np.abs(xg).max()


@pytest.mark.parametrize("shape,beta", [((32, 40, 48), 2.0), ((96, 7, 16), 0.0),
                                        ((16, 33, 16), 3.0), ((48, 2, 32), 1.0)])
def test_poisson_shapes(ibs, shape, beta):
    nx, ny, nz = shape
    _say("case poisson", shape, beta)
    g = oracle.Grid(nx, ny, nz, beta=beta)
    b = synth.scalar(nx, ny, nz, seed=5)
    xo, _ = oracle.solve(g, OP_P, b)
    S = ibs.Solver(nx, ny, nz, beta=beta)
    xg = _host(S.poisson(_dev(b)))
    err = _rel(xg, xo)
    _say("rel err", err)
    assert err < TOL


@pytest.mark.parametrize("shape,beta,c", [((32, 40, 48), 2.0, 1e-3), ((64, 24, 16), 0.0, 3e-2),
                                          ((16, 17, 32), 3.0, 4.2e-8)])
def test_helmholtz_batch(ibs, shape, beta, c):
    nx, ny, nz = shape
    _say("case helmholtz", shape, beta, c)
    g = oracle.Grid(nx, ny, nz, beta=beta)
    u, v, w = synth.velocity(nx, ny, nz, seed=7)
    refs = []
    for op, f in ((OP_U, u), (OP_V, v), (OP_W, w)):
        refs.append(oracle.solve(g, op, f, c=c)[0])
    S = ibs.Solver(nx, ny, nz, beta=beta)
    xs = S.helmholtz([0, 1, 2], [c, c, c], [_dev(u), _dev(v), _dev(w)])
    for q, (x, ref) in enumerate(zip(xs, refs)):
        xg = _host(x)
        err = _rel(xg, ref)
        _say("comp", q, "rel err", err)
        assert err < TOL
        if q == 1:
            assert np.all(xg[:, 0, :] == 0) and np.all(xg[:, ny, :] == 0)
        assert S.read_info(q).status == 0


def test_helmholtz_in_place_and_single(ibs):
    nx, ny, nz = 32, 20, 16
    g = oracle.Grid(nx, ny, nz, beta=1.0)
    v = synth.scalar(nx, ny, nz, 3, rows=ny + 1)
    ref, _ = oracle.solve(g, OP_V, v, c=5e-3)
    S = ibs.Solver(nx, ny, nz, beta=1.0)
    t = _dev(v)
    S.helmholtz([1], [5e-3], [t], [t])
    assert _rel(_host(t), ref) < TOL


def test_residual_kernel(ibs):
    nx, ny, nz = 32, 24, 16
    g = oracle.Grid(nx, ny, nz, beta=2.0)
    S = ibs.Solver(nx, ny, nz, beta=2.0)
    for op in (OP_P, OP_U, OP_V, OP_W):
        rows = ny + 1 if op == OP_V else None
        x = synth.scalar(nx, ny, nz, 1, rows=rows)
        b = synth.scalar(nx, ny, nz, 2, rows=rows)
        c = 0.0 if op == OP_P else 1e-3
        r_ref, rn, bn = oracle.residual_ld(g, op, c, x, b)
        r, n2 = S.residual(op, c, _dev(x), _dev(b), norms=True)
        rg = _host(r)
        scale = np.abs(r_ref).max()
        assert np.abs(rg - r_ref).max() < 1e-13 * scale
        n2 = _host(n2)
        assert abs(np.sqrt(n2[0]) - rn) < 1e-12 * rn
        assert abs(np.sqrt(n2[1]) - bn) < 1e-12 * bn


def test_projection_divergence_free(ibs):
    """Solve, then correct: the corrected velocity is discretely
    divergence-free to round-off (eq. g)."""
    nx, ny, nz = 64, 48, 32
    u, v, w = synth.velocity(nx, ny, nz, seed=4)
    v[:, 0, :] = 0
    v[:, ny, :] = 0
    S = ibs.Solver(nx, ny, nz, beta=2.0)
    ud, vd, wd = _dev(u), _dev(v), _dev(w)
    dt = 0.37
    b = S.divergence(ud, vd, wd, scale=1.0 / dt)
    phi = S.poisson(b)
    p = torch.zeros_like(b)
    S.correct(phi, ud, vd, wd, dt, p=p, lap_phi=b, cp=0.0)
    d1 = _host(S.divergence(ud, vd, wd))
    d0 = _host(b) * dt
    assert np.abs(d1).max() < 1e-12 * np.abs(d0).max()
    np.testing.assert_array_equal(_host(p), _host(phi))
    assert np.all(_host(vd)[:, 0, :] == 0)


@pytest.mark.parametrize("shape", [(48, 7, 16), (16, 33, 48), (1024, 3, 16), (80, 5, 48), (256, 2, 272)])
def test_stencils_shapes(ibs, shape):
    """Divergence (kernel E2) and projection plus pressure update (eq. g, h)
    against the oracle's divergence and gradient on shapes whose row blocks
    and z chunks are ragged (nx/4 not a power of two, ny+1 rows not a
    multiple of the rows per block, one row per block at nx = 1024)."""
    nx, ny, nz = shape
    _say("case stencils", shape)
    g = oracle.Grid(nx, ny, nz, beta=1.5)
    u, v, w = synth.velocity(nx, ny, nz, seed=11)
    phi = synth.scalar(nx, ny, nz, 12)
    p0 = synth.scalar(nx, ny, nz, 13)
    lap = synth.scalar(nx, ny, nz, 14)
    S = ibs.Solver(nx, ny, nz, beta=1.5)
    b = _host(S.divergence(_dev(u), _dev(v), _dev(w), scale=0.7))
    bo = oracle.divergence(g, u, v, w, scale=0.7)
    assert np.abs(b - bo).max() < 1e-14 * np.abs(bo).max()
    gs, cp = 0.3, 0.05
    ud, vd, wd, pd = _dev(u), _dev(v), _dev(w), _dev(p0)
    S.correct(_dev(phi), ud, vd, wd, gs, p=pd, lap_phi=_dev(lap), cp=cp)
    gu, gv, gw = oracle.gradient(g, phi)
    for got, ref in ((ud, u - gs * gu), (wd, w - gs * gw), (pd, p0 + phi - cp * lap)):
        ref_s = np.abs(ref).max()
        assert np.abs(_host(got) - ref).max() < 1e-14 * ref_s
    vref = v - gs * gv
    vref[:, 0, :] = 0
    vref[:, ny, :] = 0
    assert np.abs(_host(vd) - vref).max() < 1e-14 * np.abs(vref).max()
    vg = _host(vd)
    assert np.all(vg[:, 0, :] == 0) and np.all(vg[:, ny, :] == 0)
    # without the pressure update u, v, w are corrected the same way
    ud2 = _dev(u)
    S.correct(_dev(phi), ud2, _dev(v), _dev(w), gs)
    np.testing.assert_array_equal(_host(ud2), _host(ud))


def test_deterministic_bitwise(ibs):
    n = 48
    b = synth.scalar(n, n, n, 9)
    S = ibs.Solver(n, n, n, beta=1.5)
    x1 = _host(S.poisson(_dev(b)))
    x2 = _host(S.poisson(_dev(b)))
    np.testing.assert_array_equal(x1, x2)


def _eig_mode(nx, ny, nz, a, b, cz):
    i, j, k = np.arange(nx), np.arange(ny), np.arange(nz)
    return (np.cos(2 * np.pi * cz * k / nz)[:, None, None]
            * np.cos(np.pi * b * (j + 0.5) / ny)[None, :, None]
            * np.sin(2 * np.pi * a * i / nx)[None, None, :])


def test_c2_size_poisson_eigenmode_256(ibs):
    """256^3 uniform: an exact discrete eigenmode is recovered (the pin needs
    no oracle run and holds at any size)."""
    n = 256
    _say("case eigenmode 256^3")
    m = _eig_mode(n, n, n, 5, 3, 7)
    h = 1.0 / n
    lam = -(4 / h ** 2) * (np.sin(np.pi * 5 / n) ** 2 + np.sin(np.pi * 7 / n) ** 2
                           + np.sin(np.pi * 3 / (2 * n)) ** 2)
    S = ibs.Solver(n, n, n)
    xg = _host(S.poisson(_dev(lam * m)))
    err = _rel(xg, m)
    _say("rel err", err)
    assert err < TOL


def test_c2_size_manufactured_256(ibs):
    """256^3, beta = 2: manufactured solutions.  x_true is seeded (smooth +
    noise); the oracle forms b = A x_true (long-double flux form) on the CPU;
    the GPU solve must return x_true (Poisson: up to the null mode)."""
    n = 256
    _say("case manufactured 256^3")
    g = oracle.Grid(n, n, n, beta=2.0)
    S = ibs.Solver(n, n, n, beta=2.0)
    c = 0.125 * float(g.dyc.min()) ** 2
    xt = synth.manufactured(n, n, n, seed=2)
    xt = xt - oracle.weighted_mean(g, OP_P, xt)
    r, _, _ = oracle.residual_ld(g, OP_P, 0.0, xt, np.zeros_like(xt))
    xg = _host(S.poisson(_dev(-r)))
    err = _rel(xg, xt)
    _say("poisson rel err", err)
    assert err < TOL
    for op, comp in ((OP_U, 0), (OP_V, 1)):
        rows = n + 1 if op == OP_V else None
        xt = synth.manufactured(n, n, n, seed=3 + comp, rows=rows)
        if op == OP_V:
            xt[:, 0, :] = 0
            xt[:, n, :] = 0
        r, _, _ = oracle.residual_ld(g, op, c, xt, np.zeros_like(xt))
        (xg,) = S.helmholtz([comp], [c], [_dev(-r)])
        err = _rel(_host(xg), xt)
        _say("helmholtz", comp, "rel err", err)
        assert err < TOL


@pytest.mark.parametrize("shape", [(256, 96, 256), (128, 33, 96), (80, 20, 160)])
def test_fp64_manufactured_large(ibs, shape):
    """Manufactured solutions (x_true seeded, b = A x_true formed by the
    oracle's long-double stencil on the CPU) at sizes spanning many tiles of
    the folded transforms (half-lengths 128, 64, 48 and 80, the last an odd
    number of 16-blocks) and of the plain one (nx = 80)."""
    nx, ny, nz = shape
    _say("case fp64 manufactured", shape)
    g = oracle.Grid(nx, ny, nz, beta=2.0)
    S = ibs.Solver(nx, ny, nz, beta=2.0)
    c = 0.125 * min(float(g.dyc.min()), 1.0 / nx) ** 2
    xt = synth.manufactured(nx, ny, nz, seed=4)
    xt = xt - oracle.weighted_mean(g, OP_P, xt)
    r, _, _ = oracle.residual_ld(g, OP_P, 0.0, xt, np.zeros_like(xt))
    err = _rel(_host(S.poisson(_dev(-r))), xt)
    _say("poisson err", err)
    assert err < TOL
    for op, comp in ((OP_U, 0), (OP_V, 1), (OP_W, 2)):
        rows = ny + 1 if op == OP_V else None
        xt = synth.manufactured(nx, ny, nz, seed=5 + comp, rows=rows)
        if op == OP_V:
            xt[:, 0, :] = 0
            xt[:, ny, :] = 0
        r, _, _ = oracle.residual_ld(g, op, c, xt, np.zeros_like(xt))
        (x,) = S.helmholtz([comp], [c], [_dev(-r)])
        err = _rel(_host(x), xt)
        _say("helmholtz", comp, "err", err)
        assert err < TOL


def test_tile_candidates_bitwise_equal(ibs):
    """Every tile candidate of the folded transforms gives the same bits;
    ibs_autotune() returns valid choices and keeps them in the plan."""
    nx, ny, nz = 96, 33, 64
    _say("case tile candidates", (nx, ny, nz))
    b = synth.scalar(nx, ny, nz, seed=9)
    u, v, w = synth.velocity(nx, ny, nz, seed=10)
    S = ibs.Solver(nx, ny, nz, beta=1.5)
    ref = None
    for cand in range(8):
        ibs.ibs_plan_set_tiles(S.plan, [cand, cand])
        out = [_host(S.poisson(_dev(b)))]
        out += [_host(x) for x in S.helmholtz([0, 1, 2], [1e-3] * 3, [_dev(u), _dev(v), _dev(w)])]
        if ref is None:
            ref = out
        else:
            for o, r in zip(out, ref):
                np.testing.assert_array_equal(o, r, err_msg=f"candidate {cand}")
    ch = S.autotune()
    _say("autotune choices", ch)
    assert len(ch) == 2 and all(0 <= c < 8 for c in ch)
    np.testing.assert_array_equal(_host(S.poisson(_dev(b))), ref[0])


@pytest.mark.parametrize("refined", [False, True])
def test_v_walls_ignored_and_zeroed(ibs, refined):
    """The v wall faces of the right-hand side are ignored (NaN there changes
    nothing) and the v wall faces of the solution are written as zeros
    whatever the output buffer held."""
    nx, ny, nz = 64, 20, 32
    _say("case v walls", refined)
    prec = ibs.IBS_REFINED_BF16X3 if refined else ibs.IBS_FP64
    S = ibs.Solver(nx, ny, nz, beta=1.0, precision=prec)
    v = synth.scalar(nx, ny, nz, 3, rows=ny + 1)
    v[:, 0, :] = 0
    v[:, ny, :] = 0
    (ref,) = S.helmholtz([1], [2e-3], [_dev(v)])
    ref = _host(ref)
    vn = v.copy()
    vn[:, 0, :] = np.nan
    vn[:, ny, :] = np.nan
    out = torch.full((nz, ny + 1, nx), float("nan"), dtype=torch.float64, device="cuda")
    S.helmholtz([1], [2e-3], [_dev(vn)], [out])
    got = _host(out)
    assert np.all(got[:, 0, :] == 0) and np.all(got[:, ny, :] == 0)
    np.testing.assert_array_equal(got, ref)
