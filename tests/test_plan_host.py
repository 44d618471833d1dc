"""CPU checks of the C-ABI library that need no GPU: symbols, plan tables,
byte counts, argument errors, and a host emulation of the separable
algorithm built from the plan's exported tables, compared with the oracle.
"""
import ctypes

import numpy as np
import pytest
import scipy.linalg as sla

import oracle
from oracle import OP_P, OP_U, OP_V, OP_W
from paper_2406_19920_amd import synth

ibs = pytest.importorskip("paper_2406_19920_amd.ibsolve")


def test_exports_every_header_symbol():
    import re
    import os
    hdr = open(os.path.join(os.path.dirname(__file__), "..", "include", "ibsolve.h")).read()
    declared = set(re.findall(r"^\s*(?:ibs_status|const char \*)\s*(\w+)\s*\(", hdr, re.M))
    assert declared == set(ibs.EXPORTS), declared ^ set(ibs.EXPORTS)
    for name in declared:
        assert hasattr(ibs.lib, name)
    assert "gfx950" in ibs.ibs_version()


def _plan(nx=32, ny=24, nz=16, **kw):
    return ibs.solver_plan(ibs.make_desc(nx, ny, nz, **kw))


def test_plan_tables_match_paper_closed_forms():
    nx, ny, nz = 32, 20, 48
    p = _plan(nx, ny, nz, beta=1.7, lx=2.0, lz=0.5)
    try:
        Qx = ibs.ibs_plan_export(p, 1).reshape(nx, nx)
        Qz = ibs.ibs_plan_export(p, 2).reshape(nz, nz)
        lx = ibs.ibs_plan_export(p, 3)
        lz = ibs.ibs_plan_export(p, 4)
        np.testing.assert_allclose(Qx.T @ Qx, np.eye(nx), atol=1e-14)
        np.testing.assert_allclose(Qz.T @ Qz, np.eye(nz), atol=1e-14)
        # Q diagonalises the periodic second difference with eigenvalues equal
        # to minus the modified wavenumber squared (Appendix A)
        for Q, lam, n, h in ((Qx, lx, nx, 2.0 / nx), (Qz, lz, nz, 0.5 / nz)):
            L = (np.roll(np.eye(n), 1, 0) + np.roll(np.eye(n), -1, 0) - 2 * np.eye(n)) / h ** 2
            np.testing.assert_allclose(Q.T @ L @ Q, np.diag(lam), atol=1e-9 / h ** 2)
            kk = np.array([a if a <= n // 2 else a - n // 2 for a in range(n)])
            kappa2 = (2 / h ** 2) * (1 - np.cos(2 * np.pi * kk / n))
            np.testing.assert_allclose(-lam, kappa2, rtol=1e-13, atol=1e-9)
        g = oracle.Grid(nx, ny, nz, lx=2.0, lz=0.5, beta=1.7)
        np.testing.assert_array_equal(ibs.ibs_plan_export(p, 0), g.yf)
    finally:
        ibs.solver_plan_destroy(p)


def test_plan_bytes_and_errors():
    p = _plan(64, 64, 64)
    try:
        cb, wb = ibs.solver_plan_bytes(p, ibs.IBS_OP_POISSON)
        assert wb == 64 ** 3 * 8 and cb >= 4 * 64 * 64 * 8
        _, wh = ibs.solver_plan_bytes(p, ibs.IBS_OP_HELMHOLTZ_U, 3)
        assert wh == 3 * 64 * 65 * 64 * 8
        # the refined path holds three FP32 fields per component
        pr = _plan(64, 64, 64, precision=ibs.IBS_REFINED_BF16X3)
        try:
            assert ibs.solver_plan_bytes(pr, ibs.IBS_OP_POISSON)[1] == 64 ** 3 * 12
            assert ibs.solver_plan_bytes(pr, ibs.IBS_OP_HELMHOLTZ_U, 2)[1] == 2 * 64 * 65 * 64 * 12
        finally:
            ibs.solver_plan_destroy(pr)
        with pytest.raises(ibs.IbsError) as e:
            ibs.solver_plan_bytes(p, 9)
        assert e.value.status == ibs.IBS_ERR_INVALID_ARG
        # solving before upload is refused on the host
        with pytest.raises(ibs.IbsError) as e:
            ibs.solve_poisson(p, 256, 256, 256, wb, None, None)
        assert e.value.status == ibs.IBS_ERR_NOT_UPLOADED
    finally:
        ibs.solver_plan_destroy(p)
    for bad in (dict(nx=24), dict(nz=8), dict(ny=1), dict(ny=900)):
        kw = dict(nx=32, ny=16, nz=32)
        kw.update(bad)
        with pytest.raises(ibs.IbsError) as e:
            _plan(**kw)
        assert e.value.status == ibs.IBS_ERR_UNSUPPORTED
    for bad in (dict(nx=48), dict(nz=544)):
        kw = dict(nx=64, ny=16, nz=64, precision=ibs.IBS_REFINED_BF16X3)
        kw.update(bad)
        with pytest.raises(ibs.IbsError) as e:
            _plan(**kw)
        assert e.value.status == ibs.IBS_ERR_UNSUPPORTED
    p = _plan(64, 16, 64)
    try:
        assert ibs.ibs_autotune_bytes(p) == 2 * 64 * 17 * 64 * 8
        with pytest.raises(ibs.IbsError) as e:   # refused on the host before any device call
            ibs.ibs_autotune(p, 256, 1 << 30)
        assert e.value.status == ibs.IBS_ERR_NOT_UPLOADED
        ibs.ibs_plan_set_tiles(p, [3, -1])
        with pytest.raises(ibs.IbsError) as e:
            ibs.ibs_plan_set_tiles(p, [8, 0])
        assert e.value.status == ibs.IBS_ERR_INVALID_ARG
    finally:
        ibs.solver_plan_destroy(p)
    with pytest.raises(ibs.IbsError) as e:
        _plan(32, 16, 32, bc_x=ibs.IBS_DIRICHLET)
    assert e.value.status == ibs.IBS_ERR_UNSUPPORTED
    with pytest.raises(ibs.IbsError) as e:
        _plan(32, 16, 32, beta=-1.0)
    assert e.value.status == ibs.IBS_ERR_INVALID_ARG
    with pytest.raises(ibs.IbsError) as e:
        _plan(32, 4, 32, y_faces=[0.0, 0.5, 0.4, 0.8, 1.0])
    assert e.value.status == ibs.IBS_ERR_INVALID_ARG


def test_axis_tables_shared_between_plans():
    """Plans that share an axis length take that axis's tables from a
    process-wide cache: a plan built after others with the same nx or nz
    (different ny, stretching, precision or axis role) exports exactly the
    tables a plan of its own would, for both the folded and plain sizes."""
    R, F = ibs.IBS_REFINED_BF16X3, ibs.IBS_FP64
    cases = [(64, 10, 96, 0.0, F), (96, 30, 64, 2.0, R), (64, 7, 64, 1.0, R), (96, 12, 96, 3.0, F),
             (64, 10, 96, 0.0, F)]
    ref = {}
    for nx, ny, nz, beta, prec in cases:
        p = _plan(nx, ny, nz, beta=beta, precision=prec)
        try:
            Qx = ibs.ibs_plan_export(p, 1).reshape(nx, nx)
            Qz = ibs.ibs_plan_export(p, 2).reshape(nz, nz)
            lx, lz = ibs.ibs_plan_export(p, 3), ibs.ibs_plan_export(p, 4)
        finally:
            ibs.solver_plan_destroy(p)
        for n, Q, lam in ((nx, Qx, lx), (nz, Qz, lz)):
            np.testing.assert_allclose(Q.T @ Q, np.eye(n), atol=1e-14)
            if n in ref:
                np.testing.assert_array_equal(Q, ref[n][0])
                np.testing.assert_array_equal(lam, ref[n][1])
            ref[n] = (Q.copy(), lam.copy())


# ------------------------------------------------------------------------
# host emulation of the separable algorithm from the plan tables
# ------------------------------------------------------------------------
def _tables(p, kind):
    lo = ibs.ibs_plan_export(p, 5 + 3 * kind)
    di = ibs.ibs_plan_export(p, 6 + 3 * kind)
    up = ibs.ibs_plan_export(p, 7 + 3 * kind)
    return lo, di, up


def emulate(p, nx, ny, nz, op, rhs, c=0.0, yf=None):
    Qx = ibs.ibs_plan_export(p, 1).reshape(nx, nx)
    Qz = ibs.ibs_plan_export(p, 2).reshape(nz, nz)
    lx = ibs.ibs_plan_export(p, 3)
    lz = ibs.ibs_plan_export(p, 4)
    kind = {OP_P: 0, OP_U: 1, OP_W: 1, OP_V: 2}[op]
    lo, di, up = _tables(p, kind)
    n = ny + 1 if op == OP_V else ny
    lo, di, up = lo[:n], di[:n], up[:n]
    f = rhs.copy()
    if op == OP_V:
        f[:, 0, :] = 0
        f[:, ny, :] = 0
    h = np.einsum("kc,kja->cja", Qz, f @ Qx)
    yfv = ibs.ibs_plan_export(p, 0)
    dyc = np.diff(yfv)
    out = np.zeros_like(h)
    for cz in range(nz):
        for a in range(nx):
            s = lx[a] + lz[cz]
            if op == OP_P:
                A = np.diag(di + s) + np.diag(lo[1:], -1) + np.diag(up[:-1], 1)
            else:
                A = np.eye(n) * (1 - c * s) - c * (np.diag(di) + np.diag(lo[1:], -1) + np.diag(up[:-1], 1))
            rr = h[cz, :, a].copy()
            if op == OP_P and a == 0 and cz == 0:
                rr -= (dyc @ rr) / dyc.sum()
                A[0, :] = 0
                A[0, 0] = 1
                rr[0] = 0
                x = np.linalg.solve(A, rr)
                x -= (dyc @ x) / dyc.sum()
            else:
                x = np.linalg.solve(A, rr)
            out[cz, :, a] = x
    return np.einsum("kc,cja->kja", Qz, out) @ Qx.T


@pytest.mark.parametrize("beta", [0.0, 2.0])
@pytest.mark.parametrize("op", [OP_P, OP_U, OP_V, OP_W])
def test_host_emulation_matches_oracle(op, beta):
    nx, ny, nz = 16, 12, 32
    p = _plan(nx, ny, nz, beta=beta)
    try:
        g = oracle.Grid(nx, ny, nz, beta=beta)
        rhs = synth.scalar(nx, ny, nz, 21, rows=ny + 1 if op == OP_V else None)
        c = 0.0 if op == OP_P else 2e-3
        xo, _ = oracle.solve(g, op, rhs, c=c)
        xe = emulate(p, nx, ny, nz, op, rhs, c=c)
        err = np.linalg.norm(xe - xo) / np.linalg.norm(xo)
        assert err < 1e-13, err
    finally:
        ibs.solver_plan_destroy(p)
