"""Pins of the oracle's stretched wall-bounded x and z (this library's
extension of Section 2.1's staggered grid: an x or z with walls may carry
non-uniform faces, as y does).  The operators are the flux forms over the
local cell widths Delta and centre distances delta: pinned by dense
Kronecker products built independently of the C row assembly, structure
(the volume-weighted operator is symmetric; definiteness), the flux-form
residual, the projection, the reduction to the uniform grid, and
second-order convergence to analytic solutions of the continuous
problems.  All CPU."""
import numpy as np
import pytest

import oracle
from oracle import OP_P, OP_U, OP_V, OP_W, dense
from paper_2406_19920_amd import synth


def _csr_dense(g, op, c=0.0):
    rp, ci, av, n = oracle.assemble(g, op, c)
    A = np.zeros((n, n))
    for r in range(n):
        for q in range(rp[r], rp[r + 1]):
            A[r, ci[q]] += av[q]
    return A


def _random_faces(n, length, seed):
    """Strictly increasing faces 0 = f_0 < ... < f_n = length with widths
    spread over a factor of about four (not a smooth map)."""
    w = np.random.default_rng(seed).uniform(0.5, 2.0, n)
    f = np.concatenate([[0.0], np.cumsum(w)])
    return f * (length / f[-1])


CASES = [dict(sx=True), dict(sz=True), dict(sx=True, sz=True), dict(sx=True, sz=True, py=True),
         dict(sx=True, pz=True), dict(sz=True, px=True, beta=0.0)]


def _grid(shape, case, lx=1.2, ly=0.9, lz=0.8):
    nx, ny, nz = shape
    px = case.get("px", False) and not case.get("sx", False)
    pz = case.get("pz", False) and not case.get("sz", False)
    kw = dict(lx=lx, ly=ly, lz=lz, beta=case.get("beta", 1.5), periodic_x=px, periodic_z=pz,
              periodic_y=case.get("py", False))
    if case.get("sx"):
        kw["xf_in"] = _random_faces(nx, lx, 3 + nx)
    if case.get("sz"):
        kw["beta_z"] = 1.7
    return oracle.Grid(nx, ny, nz, **kw)


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("shape", [(6, 5, 4), (3, 4, 5), (5, 6, 3)])
@pytest.mark.parametrize("op", [OP_P, OP_U, OP_V, OP_W])
def test_stretched_dense_bruteforce(op, shape, case):
    if case.get("py") and shape[1] < 3:
        return
    g = _grid(shape, case)
    nx, ny, nz = shape
    rows = ny + 1 if (op == OP_V and not g.periodic_y) else None
    b = synth.scalar(nx, ny, nz, seed=19, rows=rows)
    cc = 0.0 if op == OP_P else 4e-3
    xd = dense.solve(g, op, b, cc)
    xo, info = oracle.solve(g, op, b, c=cc)
    err = np.linalg.norm((xo - xd).ravel()) / np.linalg.norm(xd.ravel())
    assert err < 1e-12, (err, info)
    if op == OP_U and not g.periodic_x:
        assert np.all(xo[:, :, 0] == 0)
    if op == OP_W and not g.periodic_z:
        assert np.all(xo[0] == 0)


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("op", [OP_P, OP_U, OP_V, OP_W])
def test_stretched_structure(op, case):
    g = _grid((7, 6, 5), case)
    if op != OP_P:
        c = 0.29
        A = _csr_dense(g, op, c)
        np.testing.assert_allclose(A, np.eye(A.shape[0]) - c * dense.laplacian(g, op),
                                   rtol=1e-13, atol=1e-9)
        L = (np.eye(A.shape[0]) - A) / c
    else:
        A = _csr_dense(g, op)
        np.testing.assert_allclose(A, dense.divergence_matrix(g) @ dense.gradient_matrix(g),
                                   rtol=1e-13, atol=1e-9)
        L = A
    w = oracle.weights(g, op)
    np.testing.assert_allclose(w, dense.weights(g, op), rtol=1e-14)
    # the weights are the control volumes: cells tile the box exactly
    if op == OP_P:
        assert abs(w.sum() - g.lx * g.ly * g.lz) < 1e-14
    WL = w[:, None] * L
    assert np.abs(WL - WL.T).max() < 1e-12 * np.abs(WL).max()
    ev = np.linalg.eigvalsh(0.5 * (WL + WL.T))
    if op == OP_P:
        assert np.sum(np.abs(ev) < 1e-9 * np.abs(ev).max()) == 1
    else:
        assert ev.max() < 0


def test_stretched_residual_flux_form_matches_csr():
    g = _grid((8, 9, 6), dict(sx=True, sz=True))
    for op in (OP_P, OP_U, OP_V, OP_W):
        c = 0.0 if op == OP_P else 1e-2
        x = synth.scalar(8, 9, 6, 3, rows=10 if op == OP_V else None)
        b = synth.scalar(8, 9, 6, 4, rows=10 if op == OP_V else None)
        if op == OP_W:
            x[0] = 0.0
        if op == OP_U:
            x[:, :, 0] = 0.0
        r, _, _ = oracle.residual_ld(g, op, c, x, b)
        A = _csr_dense(g, op, c)
        ref = oracle.unknowns_of(g, op, b) - A @ oracle.unknowns_of(g, op, x)
        np.testing.assert_allclose(oracle.unknowns_of(g, op, r), ref, rtol=1e-10, atol=1e-9)


@pytest.mark.parametrize("case", [dict(sx=True, sz=True), dict(sx=True, pz=True)])
def test_stretched_projection_divergence_free(case):
    nx, ny, nz = 14, 10, 12
    g = _grid((nx, ny, nz), case)
    u, v, w = synth.velocity(nx, ny, nz, seed=6)
    v[:, 0, :] = 0
    v[:, ny, :] = 0
    u[:, :, 0] = 0.0
    if not g.periodic_z:
        w[0] = 0.0
    d0 = oracle.divergence(g, u, v, w)
    phi, info = oracle.solve(g, OP_P, d0)
    # the walls close the box: the divergence integrates to zero
    assert abs(info.removed_mean) < 1e-12 * np.abs(d0).max()
    gu, gv, gw = oracle.gradient(g, phi)
    assert np.all(gu[:, :, 0] == 0)
    d1 = oracle.divergence(g, u - gu, v - gv, w - gw)
    assert np.abs(d1).max() <= 1e-11 * np.abs(d0).max()


@pytest.mark.parametrize("op", [OP_P, OP_U, OP_V, OP_W])
def test_stretched_uniform_faces_reduce_to_uniform(op):
    """Faces given explicitly at i*l/n take the stretched code path; they
    reproduce the uniform walls (pinned by exact eigenmodes) to rounding."""
    nx, ny, nz = 8, 6, 7
    lx, lz = 1.1, 0.7
    gu = oracle.Grid(nx, ny, nz, lx=lx, lz=lz, beta=1.0, periodic_x=False, periodic_z=False)
    gs = oracle.Grid(nx, ny, nz, lx=lx, lz=lz, beta=1.0, periodic_x=False, periodic_z=False,
                     xf_in=lx * np.arange(nx + 1) / nx, zf_in=lz * np.arange(nz + 1) / nz)
    assert gs.stretched_x and gs.stretched_z
    np.testing.assert_allclose(gs.dxc, gu.dxc, rtol=1e-14)
    rows = ny + 1 if op == OP_V else None
    b = synth.scalar(nx, ny, nz, seed=23, rows=rows)
    c = 0.0 if op == OP_P else 5e-3
    xu, _ = oracle.solve(gu, op, b, c=c)
    xs, _ = oracle.solve(gs, op, b, c=c)
    assert np.linalg.norm((xs - xu).ravel()) <= 1e-12 * np.linalg.norm(xu.ravel())
    np.testing.assert_allclose(oracle.weights(gs, op), oracle.weights(gu, op), rtol=1e-13)


def test_stretched_rejects_periodic_axis():
    with pytest.raises(ValueError):
        oracle.Grid(8, 6, 8, beta_x=1.0)
    with pytest.raises(ValueError):
        oracle.Grid(8, 6, 8, zf_in=np.linspace(0, 1, 9))


def _convergence_errors(op, sizes):
    """Max errors of the discrete solution against the continuous one on
    smoothly stretched (tanh) x, y, z with walls everywhere.  Pressure:
    p = cos(pi x/lx) cos(pi y/ly) cos(pi z/lz), Neumann everywhere,
    compared after removing each one's weighted mean.  Velocities: the
    product of sines that vanishes on every wall, f = (1 + cK) q; each
    component sampled at its own points (the normal faces, else centres)."""
    lx, ly, lz = 1.3, 1.0, 0.8
    K = (np.pi / lx) ** 2 + (np.pi / ly) ** 2 + (np.pi / lz) ** 2
    errs = []
    for n in sizes:
        g = oracle.Grid(n, n, n, lx=lx, ly=ly, lz=lz, beta=1.2, beta_x=1.0, beta_z=0.8,
                        periodic_x=False, periodic_z=False)
        xs = g.xf[:n] if op == OP_U else g.xc
        ys = g.yf if op == OP_V else g.yc
        zs = g.zf[:n] if op == OP_W else g.zc
        Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
        if op == OP_P:
            q = np.cos(np.pi * X / lx) * np.cos(np.pi * Y / ly) * np.cos(np.pi * Z / lz)
            x, _ = oracle.solve(g, op, -K * q, tol=1e-13)
            ref = q - oracle.weighted_mean(g, OP_P, q)
        else:
            q = np.sin(np.pi * X / lx) * np.sin(np.pi * Y / ly) * np.sin(np.pi * Z / lz)
            c = 0.01
            x, _ = oracle.solve(g, op, (1.0 + c * K) * q, c=c, tol=1e-13)
            ref = q
        errs.append(np.abs(x - ref).max() / np.abs(ref).max())
    return np.array(errs)


@pytest.mark.parametrize("op", [OP_P, OP_U, OP_V, OP_W])
def test_stretched_second_order_convergence(op):
    sizes = np.array([16, 32, 48])
    errs = _convergence_errors(op, sizes)
    rates = np.log(errs[:-1] / errs[1:]) / np.log(sizes[1:] / sizes[:-1])
    assert np.all(rates > 1.8), (errs, rates)
