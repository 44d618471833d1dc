"""Pins of the oracle's walls in x (the non-periodic direction of the
paper's inflow-outflow example, Section 3.2, taken as walls: u Dirichlet
on the wall faces, v and w Dirichlet through a mirror ghost, the pressure
homogeneous Neumann).  The same families of pins as for the periodic x:
exact discrete eigenmodes (cosine and sine series of the uniform
staggered grid), brute-force dense solves from Kronecker products built
independently of the C assembly, structure (symmetry in the weighted form,
definiteness, the constant null mode of L_p = D G), the flux-form residual
and the projection to a divergence-free field.  All CPU."""
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
    """Eigenvalue of the wall-bounded second difference on n cells for the
    mode of index a: -(4/h^2) sin^2(pi a / (2n))."""
    return -(4.0 / h ** 2) * np.sin(np.pi * a / (2 * n)) ** 2


def _mode_xw(nx, a, op):
    """x factor of an exact eigenmode with x walls: cosine series on the
    cell centres for the pressure (a = 0..nx-1), sine series on the faces
    for u (a = 1..nx-1; slot 0 is the wall face, zero), sine series on the
    cell centres for v and w (a = 1..nx)."""
    i = np.arange(nx)
    if op == OP_P:
        return np.cos(np.pi * a * (i + 0.5) / nx)
    if op == OP_U:
        return np.sin(np.pi * a * i / nx)
    return np.sin(np.pi * a * (i + 0.5) / nx)


def _mode_y(ny, b, op):
    if op == OP_P:
        return np.cos(np.pi * b * (np.arange(ny) + 0.5) / ny)
    if op in (OP_U, OP_W):
        return np.sin(np.pi * b * (np.arange(ny) + 0.5) / ny)
    return np.sin(np.pi * b * np.arange(ny + 1) / ny)


def _mode_z(nz, a, kind):
    k = np.arange(nz)
    return np.cos(2 * np.pi * a * k / nz) if kind == "c" else np.sin(2 * np.pi * a * k / nz)


@pytest.mark.parametrize("op", [OP_P, OP_U, OP_V, OP_W])
@pytest.mark.parametrize("shape", [(8, 6, 4), (16, 12, 10), (12, 16, 8)])
def test_xwalls_p1_eigenmodes(op, shape):
    nx, ny, nz = shape
    g = oracle.Grid(nx, ny, nz, lx=1.1, ly=1.3, lz=0.7, periodic_x=False)
    rng = np.random.default_rng(7)
    c = 2e-3
    lo_a = {OP_P: 0, OP_U: 1, OP_V: 1, OP_W: 1}[op]
    hi_a = {OP_P: nx - 1, OP_U: nx - 1, OP_V: nx, OP_W: nx}[op]
    for _ in range(4):
        a = int(rng.integers(lo_a, hi_a + 1))
        cz = int(rng.integers(0, nz // 2 + 1))
        if op == OP_P:
            b = int(rng.integers(0, ny))
            if a == 0 and cz == 0 and b == 0:
                b = 1
        elif op == OP_V:
            b = int(rng.integers(1, ny))
        else:
            b = int(rng.integers(1, ny + 1))
        m = (_mode_z(nz, cz, "c" if rng.random() < 0.5 or cz == 0 else "s")[:, None, None]
             * _mode_y(ny, b, op)[None, :, None] * _mode_xw(nx, a, op)[None, None, :])
        if np.abs(m).max() < 1e-8:
            continue
        lam = (_lam_half(nx, g.hx, a) - (4.0 / g.hz ** 2) * np.sin(np.pi * cz / nz) ** 2
               + _lam_half(ny, g.ly / ny, b))
        if op == OP_P:
            x, info = oracle.solve(g, op, lam * m)
            ref = m - oracle.weighted_mean(g, OP_P, m)
        else:
            x, info = oracle.solve(g, op, (1.0 - c * lam) * m, c=c)
            ref = m
        err = np.linalg.norm((x - ref).ravel()) / np.linalg.norm(ref.ravel())
        assert err < 1e-13, (op, shape, a, b, cz, err, info)
        # the operator itself on the mode (flux-form residual with b = 0)
        r, _, _ = oracle.residual_ld(g, op, c if op != OP_P else 0.0, m, np.zeros_like(m))
        Am = lam * m if op == OP_P else (1.0 - c * lam) * m
        np.testing.assert_allclose(-r, Am, rtol=0, atol=1e-10 * np.abs(Am).max())


@pytest.mark.parametrize("beta,py", [(0.0, False), (1.5, False), (3.0, False), (0.0, True)])
@pytest.mark.parametrize("shape", [(8, 6, 4), (4, 8, 8), (3, 5, 2), (6, 4, 3)])
@pytest.mark.parametrize("op", [OP_P, OP_U, OP_V, OP_W])
def test_xwalls_p2_dense_bruteforce(op, shape, beta, py):
    nx, ny, nz = shape
    g = oracle.Grid(nx, ny, nz, beta=beta, periodic_x=False, periodic_y=py)
    rows = ny + 1 if (op == OP_V and not py) else None
    b = synth.scalar(nx, ny, nz, seed=13, rows=rows)
    c = 0.0 if op == OP_P else 3e-3
    xd = dense.solve(g, op, b, c)
    xo, info = oracle.solve(g, op, b, c=c)
    err = np.linalg.norm((xo - xd).ravel()) / np.linalg.norm(xd.ravel())
    assert err < 1e-13, (err, info)
    if op == OP_U:
        assert np.all(xo[:, :, 0] == 0)     # the wall face x = 0


@pytest.mark.parametrize("beta", [0.0, 2.0])
@pytest.mark.parametrize("op", [OP_P, OP_U, OP_V, OP_W])
def test_xwalls_p3_structure(op, beta):
    g = oracle.Grid(6, 7, 5, lx=1.2, ly=0.9, lz=0.8, beta=beta, periodic_x=False)
    if op != OP_P:
        c = 0.37
        A = _csr_dense(g, op, c)
        Ld = dense.laplacian(g, op)
        np.testing.assert_allclose(A, np.eye(A.shape[0]) - c * Ld, rtol=1e-13, atol=1e-9)
        L = (np.eye(A.shape[0]) - A) / c
    else:
        A = _csr_dense(g, op)
        Ld = dense.divergence_matrix(g) @ dense.gradient_matrix(g)   # L_p = D G
        np.testing.assert_allclose(A, Ld, rtol=1e-13, atol=1e-9)
        L = A
        assert np.abs(L @ np.ones(L.shape[0])).max() < 1e-9 * np.abs(L).max()
    w = oracle.weights(g, op)
    np.testing.assert_allclose(w, dense.weights(g, op), rtol=1e-15)
    WL = w[:, None] * L
    assert np.abs(WL - WL.T).max() < 1e-12 * np.abs(WL).max()
    ev = np.linalg.eigvalsh(0.5 * (WL + WL.T))
    if op == OP_P:
        assert ev.max() <= 1e-9 * np.abs(ev).max()
        assert np.sum(np.abs(ev) < 1e-9 * np.abs(ev).max()) == 1     # one null mode
    else:
        assert ev.max() < 0


def test_xwalls_residual_flux_form_matches_csr():
    g = oracle.Grid(8, 9, 6, beta=2.5, periodic_x=False)
    for op in (OP_P, OP_U, OP_V, OP_W):
        c = 0.0 if op == OP_P else 1e-2
        x = synth.scalar(8, 9, 6, 3, rows=10 if op == OP_V else None)
        b = synth.scalar(8, 9, 6, 4, rows=10 if op == OP_V else None)
        if op == OP_U:
            x[:, :, 0] = 0.0      # the wall face holds zero
        r, _, _ = oracle.residual_ld(g, op, c, x, b)
        A = _csr_dense(g, op, c)
        ref = oracle.unknowns_of(g, op, b) - A @ oracle.unknowns_of(g, op, x)
        np.testing.assert_allclose(oracle.unknowns_of(g, op, r), ref, rtol=1e-10, atol=1e-9)
        if op == OP_U:
            assert np.all(r[:, :, 0] == 0)


@pytest.mark.parametrize("py", [False, True])
def test_xwalls_p4_projection_divergence_free(py):
    nx, ny, nz = 16, 12, 8
    g = oracle.Grid(nx, ny, nz, beta=0.0 if py else 2.0, periodic_x=False, periodic_y=py)
    u, v, w = synth.velocity(nx, ny, nz, seed=2)
    if py:
        v = np.ascontiguousarray(v[:, :ny, :])
    else:
        v[:, 0, :] = 0
        v[:, ny, :] = 0
    u[:, :, 0] = 0.0
    d0 = oracle.divergence(g, u, v, w)
    phi, info = oracle.solve(g, OP_P, d0)
    assert abs(info.removed_mean) < 1e-12 * np.abs(d0).max()    # walls closed: compatible
    gu, gv, gw = oracle.gradient(g, phi)
    assert np.all(gu[:, :, 0] == 0)
    d1 = oracle.divergence(g, u - gu, v - gv, w - gw)
    assert np.abs(d1).max() <= 1e-12 * np.abs(d0).max()


def test_xwalls_divergence_ignores_wall_slot():
    nx, ny, nz = 8, 6, 4
    g = oracle.Grid(nx, ny, nz, periodic_x=False)
    u, v, w = synth.velocity(nx, ny, nz, seed=3)
    d0 = oracle.divergence(g, u, v, w)
    u2 = u.copy()
    u2[:, :, 0] = 123.0
    np.testing.assert_array_equal(oracle.divergence(g, u2, v, w), d0)
    # the last cell's east face is the wall x = lx (zero)
    ref = (0.0 - u[:, :, nx - 1]) / g.hx + (v[:, 1:, :] - v[:, :-1, :])[:, :, nx - 1] / g.dyc[None, :] \
        + (np.roll(w, -1, axis=0) - w)[:, :, nx - 1] / g.hz
    np.testing.assert_allclose(d0[:, :, nx - 1], ref, rtol=1e-14, atol=1e-12)
