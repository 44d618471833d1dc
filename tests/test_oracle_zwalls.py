"""Pins of the oracle's walls in z, alone and together with walls in x (a
duct): the same construction as the walls in x (w Dirichlet on the wall
faces, plane 0 of w being the wall face z = 0; u and v Dirichlet through a
mirror ghost; the pressure homogeneous Neumann), pinned by exact discrete
eigenmodes, brute-force dense solves from Kronecker products built
independently of the C assembly, structure, the flux-form residual and the
projection.  All CPU."""
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


def _lam_half(n, h, a):
    return -(4.0 / h ** 2) * np.sin(np.pi * a / (2 * n)) ** 2


def _wall_mode(n, a, faces):
    """cosine (a >= 0, centres; faces=None), sine on the centres (faces=False)
    or sine on the faces 0..n-1 (faces=True, slot 0 the wall)."""
    i = np.arange(n)
    if faces is None:
        return np.cos(np.pi * a * (i + 0.5) / n)
    if faces:
        return np.sin(np.pi * a * i / n)
    return np.sin(np.pi * a * (i + 0.5) / n)


def _mode_y(ny, b, op):
    if op == OP_P:
        return np.cos(np.pi * b * (np.arange(ny) + 0.5) / ny)
    if op in (OP_U, OP_W):
        return np.sin(np.pi * b * (np.arange(ny) + 0.5) / ny)
    return np.sin(np.pi * b * np.arange(ny + 1) / ny)


def _axis(op, normal_op):
    """(kind, lowest index, highest index) of the wall-bounded mode along an
    axis whose normal velocity component is normal_op."""
    if op == OP_P:
        return None, 0, None
    return (op == normal_op), 1, None


@pytest.mark.parametrize("duct", [False, True])
@pytest.mark.parametrize("op", [OP_P, OP_U, OP_V, OP_W])
@pytest.mark.parametrize("shape", [(8, 6, 8), (12, 10, 16)])
def test_zwalls_p1_eigenmodes(op, shape, duct):
    nx, ny, nz = shape
    g = oracle.Grid(nx, ny, nz, lx=1.1, ly=1.3, lz=0.7, periodic_z=False, periodic_x=not duct)
    rng = np.random.default_rng(11)
    c = 2e-3
    for _ in range(4):
        # z factor
        if op == OP_P:
            az = int(rng.integers(0, nz))
            mz = _wall_mode(nz, az, None)
        elif op == OP_W:
            az = int(rng.integers(1, nz))
            mz = _wall_mode(nz, az, True)
        else:
            az = int(rng.integers(1, nz + 1))
            mz = _wall_mode(nz, az, False)
        lam = _lam_half(nz, g.hz, az)
        # x factor
        if duct:
            if op == OP_P:
                ax = int(rng.integers(0, nx))
                mx = _wall_mode(nx, ax, None)
            elif op == OP_U:
                ax = int(rng.integers(1, nx))
                mx = _wall_mode(nx, ax, True)
            else:
                ax = int(rng.integers(1, nx + 1))
                mx = _wall_mode(nx, ax, False)
            lam += _lam_half(nx, g.hx, ax)
        else:
            ax = int(rng.integers(0, nx // 2 + 1))
            mx = np.cos(2 * np.pi * ax * np.arange(nx) / nx)
            lam += -(4.0 / g.hx ** 2) * np.sin(np.pi * ax / nx) ** 2
        # y factor
        if op == OP_P:
            b = int(rng.integers(0, ny))
            if b == 0 and az == 0 and (ax == 0):
                b = 1
        elif op == OP_V:
            b = int(rng.integers(1, ny))
        else:
            b = int(rng.integers(1, ny + 1))
        lam += _lam_half(ny, g.ly / ny, b)
        m = mz[:, None, None] * _mode_y(ny, b, op)[None, :, None] * mx[None, None, :]
        if np.abs(m).max() < 1e-8:
            continue
        if op == OP_P:
            x, info = oracle.solve(g, op, lam * m)
            ref = m - oracle.weighted_mean(g, OP_P, m)
        else:
            x, info = oracle.solve(g, op, (1.0 - c * lam) * m, c=c)
            ref = m
        err = np.linalg.norm((x - ref).ravel()) / np.linalg.norm(ref.ravel())
        assert err < 1e-13, (op, shape, duct, ax, b, az, err, info)


@pytest.mark.parametrize("case", [dict(beta=0.0), dict(beta=2.0), dict(beta=1.0, px=False),
                                  dict(beta=0.0, py=True), dict(beta=0.0, py=True, px=False)])
@pytest.mark.parametrize("shape", [(8, 6, 4), (4, 8, 8), (3, 5, 3), (6, 4, 5)])
@pytest.mark.parametrize("op", [OP_P, OP_U, OP_V, OP_W])
def test_zwalls_p2_dense_bruteforce(op, shape, case):
    nx, ny, nz = shape
    py, px = case.get("py", False), case.get("px", True)
    if (py and ny < 3) or (not px and nx < 3):
        return
    g = oracle.Grid(nx, ny, nz, beta=case["beta"], periodic_z=False, periodic_x=px, periodic_y=py)
    rows = ny + 1 if (op == OP_V and not py) else None
    b = synth.scalar(nx, ny, nz, seed=17, rows=rows)
    cc = 0.0 if op == OP_P else 3e-3
    xd = dense.solve(g, op, b, cc)
    xo, info = oracle.solve(g, op, b, c=cc)
    err = np.linalg.norm((xo - xd).ravel()) / np.linalg.norm(xd.ravel())
    assert err < 1e-13, (err, info)
    if op == OP_W:
        assert np.all(xo[0] == 0)


@pytest.mark.parametrize("px", [True, False])
@pytest.mark.parametrize("op", [OP_P, OP_U, OP_V, OP_W])
def test_zwalls_p3_structure(op, px):
    g = oracle.Grid(6, 7, 5, lx=1.2, ly=0.9, lz=0.8, beta=1.5, periodic_z=False, periodic_x=px)
    if op != OP_P:
        c = 0.37
        A = _csr_dense(g, op, c)
        np.testing.assert_allclose(A, np.eye(A.shape[0]) - c * dense.laplacian(g, op), rtol=1e-13, atol=1e-9)
        L = (np.eye(A.shape[0]) - A) / c
    else:
        A = _csr_dense(g, op)
        np.testing.assert_allclose(A, dense.divergence_matrix(g) @ dense.gradient_matrix(g), rtol=1e-13, atol=1e-9)
        L = A
    w = oracle.weights(g, op)
    np.testing.assert_allclose(w, dense.weights(g, op), rtol=1e-15)
    WL = w[:, None] * L
    assert np.abs(WL - WL.T).max() < 1e-12 * np.abs(WL).max()
    ev = np.linalg.eigvalsh(0.5 * (WL + WL.T))
    if op == OP_P:
        assert np.sum(np.abs(ev) < 1e-9 * np.abs(ev).max()) == 1
    else:
        assert ev.max() < 0


def test_zwalls_residual_flux_form_matches_csr():
    g = oracle.Grid(8, 9, 6, beta=2.5, periodic_z=False, periodic_x=False)
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
        if op == OP_W:
            assert np.all(r[0] == 0)


@pytest.mark.parametrize("px", [True, False])
def test_zwalls_p4_projection_divergence_free(px):
    nx, ny, nz = 16, 12, 10
    g = oracle.Grid(nx, ny, nz, beta=2.0, periodic_z=False, periodic_x=px)
    u, v, w = synth.velocity(nx, ny, nz, seed=5)
    v[:, 0, :] = 0
    v[:, ny, :] = 0
    w[0] = 0.0
    if not px:
        u[:, :, 0] = 0.0
    d0 = oracle.divergence(g, u, v, w)
    phi, info = oracle.solve(g, OP_P, d0)
    assert abs(info.removed_mean) < 1e-12 * np.abs(d0).max()
    gu, gv, gw = oracle.gradient(g, phi)
    assert np.all(gw[0] == 0)
    d1 = oracle.divergence(g, u - gu, v - gv, w - gw)
    assert np.abs(d1).max() <= 1e-12 * np.abs(d0).max()
    # the wall plane of w is ignored by the divergence
    w2 = w.copy()
    w2[0] = 5.0
    np.testing.assert_array_equal(oracle.divergence(g, u, v, w2), d0)
