"""Reference (oracle) solver for the staggered Poisson and Helmholtz problems.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by
the benchmark's CPU-baseline leg.  The GPU library neither imports nor links
anything here, and this package imports nothing from the GPU library.

Two independent parts:

* ``orc.c`` (loaded through ctypes): grid, staggered divergence/gradient,
  CSR assembly of the 7-point operators and a Jacobi-preconditioned
  conjugate-gradient solver to a true relative residual of 1e-14, polished
  by refinement against a long-double residual (paper eqs. e and f of the
  Runge-Kutta sub-step, Section 2.1; Appendix B for the wall rows).
* ``dense.py``: brute-force dense solves for grids up to 8^3, with the
  operators built as products of 1-D difference matrices (L_p = D G).

Layout: C order [z][y][x]; v is [nz][ny+1][nx] with wall faces j=0, j=ny.
Operator codes: 0 pressure Poisson (A = L_p), 1 u, 2 v, 3 w Helmholtz
(A = I - c L).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liborc.so")
_SRC = os.path.join(_HERE, "orc.c")

OP_P, OP_U, OP_V, OP_W = 0, 1, 2, 3


def build(force: bool = True) -> str:
    """Compile orc.c into liborc.so with gcc + OpenMP."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared", _SRC,
             "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        L.orc_grid.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double,
                               dp, dp, dp, dp, dp]
        L.orc_grid.restype = ctypes.c_int
        for name in ("orc_divergence",):
            getattr(L, name).argtypes = [ctypes.c_void_p, dp, dp, dp,
                                         ctypes.c_double, dp]
        L.orc_gradient.argtypes = [ctypes.c_void_p, dp, dp, dp, dp]
        L.orc_num_unknowns.argtypes = [ctypes.c_void_p, ctypes.c_int]
        L.orc_num_unknowns.restype = ctypes.c_int64
        L.orc_assemble.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_double,
                                   ctypes.POINTER(ctypes.c_int64),
                                   ctypes.POINTER(ctypes.c_int64), dp]
        L.orc_assemble.restype = ctypes.c_int64
        L.orc_weights.argtypes = [ctypes.c_void_p, ctypes.c_int, dp]
        L.orc_residual_ld.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_double,
                                      dp, dp, dp, dp]
        L.orc_residual_bc_ld.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_double,
                                         dp, dp, dp, dp, dp, dp]
        L.orc_solve.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_double,
                                dp, dp, ctypes.c_double, ctypes.c_int,
                                ctypes.c_void_p]
        L.orc_solve.restype = ctypes.c_int
        L.orc_weighted_mean.argtypes = [ctypes.c_void_p, ctypes.c_int, dp]
        L.orc_weighted_mean.restype = ctypes.c_double
        L.orc_num_threads.restype = ctypes.c_int
        L.orc_set_num_threads.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class _CGeom(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("hx", ctypes.c_double), ("hz", ctypes.c_double),
                ("dyc", ctypes.POINTER(ctypes.c_double)),
                ("dyf", ctypes.POINTER(ctypes.c_double)),
                ("py", ctypes.c_int), ("wx", ctypes.c_int), ("wz", ctypes.c_int),
                ("dxc", ctypes.POINTER(ctypes.c_double)),
                ("dxf", ctypes.POINTER(ctypes.c_double)),
                ("dzc", ctypes.POINTER(ctypes.c_double)),
                ("dzf", ctypes.POINTER(ctypes.c_double))]


class _CInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("polish_steps", ctypes.c_int),
                ("polish_iters", ctypes.c_int), ("stagnated", ctypes.c_int),
                ("rel_residual", ctypes.c_double), ("removed_mean", ctypes.c_double)]


@dataclass
class Grid:
    """Staggered grid: uniform periodic x and z, walls in y (optionally
    tanh-stretched faces).  Section 2.1 describes the uniform staggered grid;
    the tanh stretching in y is this library's extension.  periodic_y: the
    triply periodic branch (Section 2.3.3, items S1 and S2): y wraps, no
    walls, v has ny faces, and delta_0 = delta_ny is the distance between
    the centres of cells ny-1 and 0 across the wrap.  periodic_x=False: walls
    at x = 0 and x = lx (the paper's non-periodic direction, Section 3.2):
    u Dirichlet (zero on the wall faces; slot 0 of u is the wall face x = 0,
    the face x = lx is not stored), v and w Dirichlet through a mirror ghost,
    the pressure homogeneous Neumann.  periodic_z=False: the same walls at
    z = 0 and z = lz (w's plane 0 is the wall face z = 0).  A wall-bounded x
    or z may be stretched like y (beta_x / xf_in, beta_z / zf_in; this
    library's extension): its operators are the flux forms over the local
    widths, dxc (cell widths) and dxf (centre distances)."""
    nx: int
    ny: int
    nz: int
    lx: float = 1.0
    ly: float = 1.0
    lz: float = 1.0
    beta: float = 0.0
    yf_in: np.ndarray | None = None
    periodic_y: bool = False
    periodic_x: bool = True
    periodic_z: bool = True
    beta_x: float = 0.0
    xf_in: np.ndarray | None = None
    beta_z: float = 0.0
    zf_in: np.ndarray | None = None
    yf: np.ndarray = field(init=False)
    yc: np.ndarray = field(init=False)
    dyc: np.ndarray = field(init=False)
    dyf: np.ndarray = field(init=False)

    def __post_init__(self):
        ny = self.ny
        self.yf = np.zeros(ny + 1)
        self.yc = np.zeros(ny)
        self.dyc = np.zeros(ny)
        self.dyf = np.zeros(ny + 1)
        yin = None
        if self.yf_in is not None:
            yin = np.ascontiguousarray(self.yf_in, dtype=np.float64)
            assert yin.shape == (ny + 1,)
        rc = lib().orc_grid(ny, self.ly, self.beta,
                            _dp(yin) if yin is not None else None,
                            _dp(self.yf), _dp(self.yc), _dp(self.dyc), _dp(self.dyf))
        if rc != 0:
            raise ValueError(f"orc_grid failed ({rc})")
        if self.periodic_y:
            if ny < 3:
                raise ValueError("periodic y needs ny >= 3")
            self.dyf[0] = self.dyf[ny] = 0.5 * (self.dyc[0] + self.dyc[ny - 1])
        if not self.periodic_x and self.nx < 3:
            raise ValueError("walls in x need nx >= 3")
        if not self.periodic_z and self.nz < 3:
            raise ValueError("walls in z need nz >= 3")
        self.stretched_x = self.beta_x != 0.0 or self.xf_in is not None
        self.stretched_z = self.beta_z != 0.0 or self.zf_in is not None
        if self.stretched_x and self.periodic_x:
            raise ValueError("a stretched x needs walls in x")
        if self.stretched_z and self.periodic_z:
            raise ValueError("a stretched z needs walls in z")
        self.xf, self.xc, self.dxc, self.dxf = self._axis(self.nx, self.lx, self.beta_x, self.xf_in)
        self.zf, self.zc, self.dzc, self.dzf = self._axis(self.nz, self.lz, self.beta_z, self.zf_in)
        self._c = _CGeom(self.nx, self.ny, self.nz, self.hx, self.hz,
                         _dp(self.dyc), _dp(self.dyf), 1 if self.periodic_y else 0,
                         0 if self.periodic_x else 1, 0 if self.periodic_z else 1,
                         _dp(self.dxc) if self.stretched_x else None,
                         _dp(self.dxf) if self.stretched_x else None,
                         _dp(self.dzc) if self.stretched_z else None,
                         _dp(self.dzf) if self.stretched_z else None)

    @staticmethod
    def _axis(n, length, beta, faces):
        """Faces, centres, cell widths and centre distances of a wall-bounded
        axis (the y construction); uniform: the widths are exactly h."""
        f, c, dc, df = np.zeros(n + 1), np.zeros(n), np.zeros(n), np.zeros(n + 1)
        fin = None if faces is None else np.ascontiguousarray(faces, dtype=np.float64)
        if fin is not None:
            assert fin.shape == (n + 1,)
        rc = lib().orc_grid(n, length, beta, _dp(fin) if fin is not None else None,
                            _dp(f), _dp(c), _dp(dc), _dp(df))
        if rc != 0:
            raise ValueError(f"orc_grid failed ({rc})")
        if beta == 0.0 and fin is None:
            dc[:] = length / n
            df[:] = length / n
        return f, c, dc, df

    @property
    def hx(self) -> float:
        return self.lx / self.nx

    @property
    def hz(self) -> float:
        return self.lz / self.nz

    def shape(self, op: int) -> tuple:
        if op == OP_V and not self.periodic_y:
            return (self.nz, self.ny + 1, self.nx)
        return (self.nz, self.ny, self.nx)

    @property
    def cptr(self):
        return ctypes.byref(self._c)


def divergence(g: Grid, u, v, w, scale: float = 1.0) -> np.ndarray:
    u, v, w = (np.ascontiguousarray(a, dtype=np.float64) for a in (u, v, w))
    assert u.shape == g.shape(OP_U) and v.shape == g.shape(OP_V) and w.shape == g.shape(OP_W)
    b = np.empty(g.shape(OP_P))
    lib().orc_divergence(g.cptr, _dp(u), _dp(v), _dp(w), scale, _dp(b))
    return b


def gradient(g: Grid, phi):
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    gu, gv, gw = np.empty(g.shape(OP_U)), np.empty(g.shape(OP_V)), np.empty(g.shape(OP_W))
    lib().orc_gradient(g.cptr, _dp(phi), _dp(gu), _dp(gv), _dp(gw))
    return gu, gv, gw


def num_unknowns(g: Grid, op: int) -> int:
    return int(lib().orc_num_unknowns(g.cptr, op))


def assemble(g: Grid, op: int, c: float = 0.0):
    """Unweighted operator A (L_p for op 0, I - cL otherwise) in CSR over the
    unknowns (v: interior faces only).  Returns (indptr, indices, data, n)."""
    n = num_unknowns(g, op)
    rp = np.zeros(n + 1, dtype=np.int64)
    ci = np.zeros(7 * n, dtype=np.int64)
    av = np.zeros(7 * n)
    lib().orc_assemble(g.cptr, op, c, rp.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                       ci.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _dp(av))
    nnz = int(rp[-1])
    return rp, ci[:nnz].copy(), av[:nnz].copy(), n


def weights(g: Grid, op: int) -> np.ndarray:
    w = np.zeros(num_unknowns(g, op))
    lib().orc_weights(g.cptr, op, _dp(w))
    return w


def unknowns_of(g: Grid, op: int, x: np.ndarray) -> np.ndarray:
    """Flatten a full-layout field to the unknown ordering (drops the wall
    faces of v, and of u with x walls)."""
    if op == OP_V and not g.periodic_y:
        return np.ascontiguousarray(x[:, 1:g.ny, :]).reshape(-1)
    if op == OP_U and not g.periodic_x:
        return np.ascontiguousarray(x[:, :, 1:]).reshape(-1)
    if op == OP_W and not g.periodic_z:
        return np.ascontiguousarray(x[1:, :, :]).reshape(-1)
    return np.ascontiguousarray(x).reshape(-1)


def residual_ld(g: Grid, op: int, c: float, x, b):
    """r = b - A x evaluated from the flux form in long double; returns
    (r, ||r||_2, ||b||_2)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    r = np.zeros(g.shape(op))
    norms = np.zeros(2)
    lib().orc_residual_ld(g.cptr, op, c, _dp(x), _dp(b), _dp(r), _dp(norms))
    return r, float(norms[0]), float(norms[1])


def wall_shape(g: Grid) -> tuple:
    """Shape of one wall-data plane: [nz][nx] (one value per wall column)."""
    return (g.nz, g.nx)


def residual_bc_ld(g: Grid, op: int, c: float, x, b, lo=None, hi=None):
    """r = b - A(x; lo, hi): the operator with inhomogeneous wall data at
    y = 0 (lo) and y = ly (hi), each [nz][nx] or None (zero), evaluated from
    the flux form in long double.  Poisson: lo, hi are the prescribed wall
    fluxes d(phi)/dy; u, w: wall values through the mirror ghost 2g - f_0
    (Appendix B, alpha = 2); v: wall-face values (alpha = 1).  Returns
    (r, ||r||_2, ||b||_2)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    dat = []
    for d in (lo, hi):
        if d is None:
            dat.append(None)
        else:
            d = np.ascontiguousarray(d, dtype=np.float64)
            assert d.shape == wall_shape(g)
            dat.append(d)
    r = np.zeros(g.shape(op))
    norms = np.zeros(2)
    lib().orc_residual_bc_ld(g.cptr, op, c, _dp(x), _dp(b),
                             _dp(dat[0]) if dat[0] is not None else None,
                             _dp(dat[1]) if dat[1] is not None else None, _dp(r), _dp(norms))
    return r, float(norms[0]), float(norms[1])


def solve_bc(g: Grid, op: int, b, lo=None, hi=None, c: float = 0.0, tol: float = 1e-14):
    """Solve A(x; lo, hi) = b with inhomogeneous wall data (Appendix B's
    boundary terms, Section 2.3.3): the operator is affine in the data, so
    x solves the homogeneous system with right-hand side b - A(0; lo, hi),
    the data's contribution evaluated by the flux form at x = 0.  Poisson:
    the weighted mean of that right-hand side is removed as in solve() and
    x has zero weighted mean.  v: the returned wall faces hold the data.
    Returns (x, info)."""
    b = np.ascontiguousarray(b, dtype=np.float64)
    if g.periodic_y:
        raise ValueError("wall data need walls (periodic y has none)")
    zero = np.zeros(g.shape(op))
    r0, _, _ = residual_bc_ld(g, op, c, zero, b, lo, hi)   # b - A(0; lo, hi)
    x, info = solve(g, op, r0, c=c, tol=tol)
    if op == OP_V:
        x[:, 0, :] = 0.0 if lo is None else lo
        x[:, g.ny, :] = 0.0 if hi is None else hi
    return x, info


@dataclass
class SolveInfo:
    iters: int
    polish_steps: int
    polish_iters: int
    stagnated: bool
    rel_residual: float
    removed_mean: float


def solve(g: Grid, op: int, b, c: float = 0.0, tol: float = 1e-14,
          maxit: int = 200000):
    """Solve A x = b (A = L_p for op 0 with the weighted mean of b removed and
    x of zero weighted mean; A = I - cL for ops 1..3).  Returns (x, info)."""
    b = np.ascontiguousarray(b, dtype=np.float64)
    assert b.shape == g.shape(op)
    x = np.zeros(g.shape(op))
    info = _CInfo()
    rc = lib().orc_solve(g.cptr, op, c, _dp(b), _dp(x), tol, maxit, ctypes.byref(info))
    if rc != 0:
        raise ValueError(f"orc_solve failed ({rc})")
    return x, SolveInfo(info.iters, info.polish_steps, info.polish_iters,
                        bool(info.stagnated), info.rel_residual, info.removed_mean)


def weighted_mean(g: Grid, op: int, x) -> float:
    x = np.ascontiguousarray(x, dtype=np.float64)
    return float(lib().orc_weighted_mean(g.cptr, op, _dp(x)))


def remove_weighted_mean(g: Grid, x) -> np.ndarray:
    """O7: x - (1^T W x / 1^T W 1) for a cell field."""
    return x - weighted_mean(g, OP_P, x)


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_num_threads(n: int) -> None:
    lib().orc_set_num_threads(int(n))
