"""Pins of the oracle's Runge-Kutta sub-step (Section 2.1, eqs. a-h) against
what the discretisation and the mathematics fix: the divergence-form
convective term conserves momentum always and kinetic energy for
divergence-free fields on uniform grids; the Roma kernel sums to one and
reproduces linear fields; spreading conserves the total force and is the
adjoint of interpolation; a Stokes mode decays by the exact discrete factor
of the semi-implicit stage; a gradient field is removed by the projection;
a stage leaves a discretely divergence-free velocity.  All CPU."""
import numpy as np
import pytest

import oracle
from oracle import OP_P, OP_U, OP_V, OP_W, fstep


def _divfree(g, seed):
    rng = np.random.default_rng(seed)
    u, v, w = (rng.standard_normal(g.shape(op)) for op in (OP_U, OP_V, OP_W))
    if not g.periodic_y:
        v[:, 0, :] = 0
        v[:, g.ny, :] = 0
    b = oracle.divergence(g, u, v, w)
    phi, _ = oracle.solve(g, OP_P, b)
    gu, gv, gw = oracle.gradient(g, phi)
    return u - gu, v - gv, w - gw


def _weights(g):
    wu = g.hx * g.hz * g.dyc[None, :, None]
    wv = g.hx * g.hz * (g.dyf[None, :g.ny, None] if g.periodic_y else g.dyf[None, :, None])
    return wu, wv, wu


@pytest.mark.parametrize("py", [False, True])
def test_convective_conserves_energy_and_momentum(py):
    g = oracle.Grid(8, 12, 6, periodic_y=py)
    u, v, w = _divfree(g, 3)
    N = fstep.convective(g, u, v, w)
    W = _weights(g)
    e = sum((Wq * f * n).sum() for Wq, f, n in zip(W, (u, v, w), N))
    s = sum((Wq * np.abs(f * n)).sum() for Wq, f, n in zip(W, (u, v, w), N))
    assert abs(e) < 1e-14 * s
    # momentum (divergence form, any field): the total of each component's
    # convective term vanishes in periodic directions and with impermeable walls
    rng = np.random.default_rng(4)
    a, b, c = (rng.standard_normal(g.shape(op)) for op in (OP_U, OP_V, OP_W))
    if not py:
        b[:, 0, :] = 0
        b[:, g.ny, :] = 0
    Na, Nb, Nc = fstep.convective(g, a, b, c)
    for Wq, n in ((W[0], Na), (W[2], Nc)):
        assert abs((Wq * n).sum()) < 1e-13 * (Wq * np.abs(n)).sum()
    if py:
        assert abs((W[1] * Nb).sum()) < 1e-13 * (W[1] * np.abs(Nb)).sum()


def test_convective_uniform_and_parallel_flows_vanish():
    g = oracle.Grid(8, 10, 6, periodic_y=True)
    u = np.full(g.shape(OP_U), 0.7)
    v = np.full(g.shape(OP_V), -0.3)
    w = np.full(g.shape(OP_W), 1.1)
    for n in fstep.convective(g, u, v, w):
        assert np.abs(n).max() < 1e-13
    gw = oracle.Grid(8, 10, 6, beta=2.0)
    z = (np.arange(6) + 0.5) / 6
    u = np.broadcast_to(np.sin(2 * np.pi * z)[:, None, None], gw.shape(OP_U)).copy()
    for n in fstep.convective(gw, u, np.zeros(gw.shape(OP_V)), np.zeros(gw.shape(OP_W))):
        assert np.abs(n).max() < 1e-13


def test_roma_kernel_and_interpolation():
    # partition of unity and zero first moment on a unit lattice
    for s in np.linspace(-0.5, 0.5, 11):
        k = np.arange(-2, 3)
        wts = fstep.roma3(k - s)
        assert abs(wts.sum() - 1) < 1e-14
        assert abs((wts * (k - s)).sum()) < 1e-14
    g = oracle.Grid(16, 16, 16)
    rng = np.random.default_rng(1)
    markers = rng.uniform(0.3, 0.7, size=(20, 3))
    const = [np.full(g.shape(op), c) for op, c in ((OP_U, 0.5), (OP_V, -2.0), (OP_W, 3.0))]
    U = fstep.interpolate(g, const, markers)
    np.testing.assert_allclose(U, np.tile([0.5, -2.0, 3.0], (20, 1)), rtol=0, atol=1e-14)
    # linear profiles (away from the periodic seam) are reproduced exactly
    h = 1.0 / 16
    lin = [np.broadcast_to((np.arange(16) * h)[None, None, :], g.shape(OP_U)).copy(),
           np.broadcast_to((np.arange(17) * h)[None, :, None], g.shape(OP_V)).copy(),
           np.broadcast_to((np.arange(16) * h)[:, None, None], g.shape(OP_W)).copy()]
    U = fstep.interpolate(g, lin, markers)
    np.testing.assert_allclose(U, markers, rtol=0, atol=1e-14)


@pytest.mark.parametrize("py", [False, True])
def test_spreading_conserves_force_and_is_adjoint(py):
    g = oracle.Grid(16, 16, 16, periodic_y=py)
    rng = np.random.default_rng(2)
    markers = rng.uniform(0.1, 0.9, size=(30, 3))
    F = rng.standard_normal((30, 3))
    dv = rng.uniform(0.5, 1.5, size=30) * g.hx ** 3
    f = fstep.spread(g, F, markers, dv)
    vol = g.hx * (1.0 / 16) * g.hz
    for comp in range(3):
        assert abs(f[comp].sum() * vol - (F[:, comp] * dv).sum()) < 1e-13 * np.abs(F[:, comp] * dv).sum()
    u = [rng.standard_normal(g.shape(op)) for op in (OP_U, OP_V, OP_W)]
    U = fstep.interpolate(g, u, markers)
    lhs = (U * F * dv[:, None]).sum()
    rhs = sum((uq * fq).sum() * vol for uq, fq in zip(u, f))
    assert abs(lhs - rhs) < 1e-13 * abs(lhs)


def test_stage_stokes_mode_exact_factor():
    """u = sin(2 pi m z) e_x in a triply periodic box: no convection, no
    pressure; the stage multiplies it by (1 + alpha dt lam/Re) / (1 - beta
    dt lam/Re), lam the mode's discrete eigenvalue."""
    nx, ny, nz = 8, 6, 16
    g = oracle.Grid(nx, ny, nz, lz=2.0, periodic_y=True)
    m = 3
    z = (np.arange(nz) + 0.5) * g.hz
    u = np.broadcast_to(np.sin(2 * np.pi * m * z / 2.0)[:, None, None], g.shape(OP_U)).copy()
    v, w, p = np.zeros(g.shape(OP_V)), np.zeros(g.shape(OP_W)), np.zeros(g.shape(OP_P))
    coef = dict(alpha=4 / 15, beta=4 / 15, gamma=8 / 15, zeta=0.0, dt=0.01, re=0.5)
    out = fstep.stage(g, u, v, w, p, coef)
    lam = -(4 / g.hz ** 2) * np.sin(np.pi * m / nz) ** 2
    fac = (1 + coef["alpha"] * coef["dt"] * lam / coef["re"]) / (1 - coef["beta"] * coef["dt"] * lam / coef["re"])
    np.testing.assert_allclose(out["u"], fac * u, rtol=0, atol=1e-13)
    assert np.abs(out["v"]).max() < 1e-13 and np.abs(out["w"]).max() < 1e-13
    assert np.abs(out["p"]).max() < 1e-12


def test_stage_removes_gradient_fields():
    """Without convection, a velocity that is a discrete gradient stays one
    through (a) and (e) and is removed by the projection (g)."""
    g = oracle.Grid(8, 12, 8, periodic_y=True)
    rng = np.random.default_rng(5)
    q = rng.standard_normal(g.shape(OP_P))
    u, v, w = oracle.gradient(g, q)
    p = rng.standard_normal(g.shape(OP_P))
    coef = dict(alpha=1 / 15, beta=1 / 15, gamma=0.0, zeta=0.0, dt=0.02, re=100.0)
    out = fstep.stage(g, u, v, w, p, coef)
    scale = max(np.abs(u).max(), np.abs(v).max(), np.abs(w).max())
    for f in (out["u"], out["v"], out["w"]):
        assert np.abs(f).max() < 1e-12 * scale


@pytest.mark.parametrize("py", [False, True])
def test_stage_divergence_free_with_markers(py):
    g = oracle.Grid(16, 16, 16, periodic_y=py)
    u, v, w = _divfree(g, 7)
    rng = np.random.default_rng(8)
    p = rng.standard_normal(g.shape(OP_P))
    markers = rng.uniform(0.3, 0.7, size=(25, 3))
    ud = rng.standard_normal((25, 3)) * 0.1
    dv = np.full(25, g.hx ** 3)
    coef = dict(alpha=4 / 15, beta=4 / 15, gamma=8 / 15, zeta=0.0, dt=0.005, re=200.0)
    out = fstep.stage(g, u, v, w, p, coef, markers=markers, ud=ud, dvol=dv)
    d = oracle.divergence(g, out["u"], out["v"], out["w"])
    ds = oracle.divergence(g, *[out["ue"][q] for q in range(3)])
    assert np.abs(d).max() < 1e-11 * max(np.abs(ds).max(), 1.0)
    assert out["force"].shape == (25, 3)
    # second stage with the stored convective term (zeta != 0)
    coef2 = dict(alpha=1 / 15, beta=1 / 15, gamma=5 / 12, zeta=-17 / 60, dt=0.005, re=200.0)
    out2 = fstep.stage(g, out["u"], out["v"], out["w"], out["p"], coef2, n_prev=out["n"],
                       markers=markers, ud=ud, dvol=dv)
    d2 = oracle.divergence(g, out2["u"], out2["v"], out2["w"])
    assert np.abs(d2).max() < 1e-11 * max(np.abs(ds).max(), 1.0)
