"""Brute-force dense reference for tiny grids (up to about 8^3 cells).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The operators are built here from scratch, independently of ``orc.c``: as
products of 1-D staggered difference matrices combined by Kronecker
products, following the definitions of Section 2.1 (second-order central
differences on a staggered grid) and Appendix B (wall rows):

* the pressure Laplacian is literally L_p = D G, with D the divergence
  (cells <- faces of all three components) and G the gradient
  (faces <- cells, zero on the wall faces: homogeneous Neumann);
* the operator for u and w (stored at cell-centre height) uses, at a wall,
  the flux of a mirror ghost value (Dirichlet u = 0 half a cell away);
* the operator for v (interior y faces) is G_y D_y with wall values v = 0;
* periodic y (the triply periodic branch): the y differences wrap, the
  pressure Laplacian is still literally D G, u and w take D_y G_y and v
  G_y D_y over all ny faces;
* walls in x (``periodic_x=False``): the x differences stop at the walls.
  The u slots are faces 0..nx-1 with slot 0 the wall face (a zero column
  of D_x, a zero row of G_x) and the face nx absent (zero), so L_p = D G
  is again literal; u takes G_x D_x on the interior faces 1..nx-1, and v,
  w the mirror-ghost rows in x, as u and w have at the y walls;
* walls in z (``periodic_z=False``): the same along z, w's plane 0 being
  the wall face.

The dense solve uses ``numpy.linalg.solve``.  For the singular Neumann
pressure problem it solves the bordered system
    [[L_p, 1], [w^T, 0]] [x; mu] = [b; 0],
whose solution satisfies L_p x = b - mu 1 (the compatible projection of b,
mu = w^T b / w^T 1) and w^T x = 0 (zero volume-weighted mean).
"""
from __future__ import annotations

import numpy as np

from . import Grid, OP_P, OP_U, OP_V, OP_W


def _circ_diff_fwd(n: int, h: float) -> np.ndarray:
    """(f_{i+1} - f_i)/h, periodic (cells <- faces in x or z)."""
    m = np.zeros((n, n))
    for i in range(n):
        m[i, (i + 1) % n] += 1.0 / h
        m[i, i] -= 1.0 / h
    return m


def _circ_diff_bwd(n: int, h: float) -> np.ndarray:
    """(f_i - f_{i-1})/h, periodic (faces <- cells in x or z)."""
    m = np.zeros((n, n))
    for i in range(n):
        m[i, i] += 1.0 / h
        m[i, (i - 1) % n] -= 1.0 / h
    return m


def dy_faces_to_cells(g: Grid) -> np.ndarray:
    """(ny x ny+1): (F_{j+1} - F_j)/Delta_j."""
    ny = g.ny
    m = np.zeros((ny, ny + 1))
    for j in range(ny):
        m[j, j + 1] = 1.0 / g.dyc[j]
        m[j, j] = -1.0 / g.dyc[j]
    return m


def gy_cells_to_faces_neumann(g: Grid) -> np.ndarray:
    """(ny+1 x ny): (f_j - f_{j-1})/delta_j on interior faces, 0 on walls."""
    ny = g.ny
    m = np.zeros((ny + 1, ny))
    for j in range(1, ny):
        m[j, j] = 1.0 / g.dyf[j]
        m[j, j - 1] = -1.0 / g.dyf[j]
    return m


def gy_cells_to_faces_dirichlet_mirror(g: Grid) -> np.ndarray:
    """(ny+1 x ny): interior as Neumann; at the walls the gradient between the
    first (last) value and its mirror ghost, which has the opposite sign and
    sits one cell height away: 2 f_0/Delta_0 and -2 f_{ny-1}/Delta_{ny-1}."""
    m = gy_cells_to_faces_neumann(g)
    m[0, 0] = 2.0 / g.dyc[0]
    m[g.ny, g.ny - 1] = -2.0 / g.dyc[g.ny - 1]
    return m


def dy_faces_to_cells_periodic(g: Grid) -> np.ndarray:
    """(ny x ny), periodic y: (F_{j+1} - F_j)/Delta_j, face ny = face 0."""
    ny = g.ny
    m = np.zeros((ny, ny))
    for j in range(ny):
        m[j, (j + 1) % ny] += 1.0 / g.dyc[j]
        m[j, j] -= 1.0 / g.dyc[j]
    return m


def gy_cells_to_faces_periodic(g: Grid) -> np.ndarray:
    """(ny x ny), periodic y: (f_j - f_{j-1})/delta_j on every face, face 0
    between cells ny-1 and 0 (delta_0 across the wrap)."""
    ny = g.ny
    m = np.zeros((ny, ny))
    for j in range(ny):
        m[j, j] += 1.0 / g.dyf[j]
        m[j, (j - 1) % ny] -= 1.0 / g.dyf[j]
    return m


def dx_faces_to_cells_walls(dc: np.ndarray) -> np.ndarray:
    """(n x n), walls: (F_{i+1} - F_i)/Delta_i with the face slots 0..n-1,
    slot 0 the wall face (its column is zero: u = 0 there) and face n
    absent; dc[i] = Delta_i the cell widths (uniform: h)."""
    n = len(dc)
    m = np.zeros((n, n))
    for i in range(n):
        if i + 1 < n:
            m[i, i + 1] = 1.0 / dc[i]
        if i >= 1:
            m[i, i] = -1.0 / dc[i]
    return m


def gx_cells_to_faces_walls(df: np.ndarray) -> np.ndarray:
    """(n x n), walls: (f_i - f_{i-1})/delta_i on the face slots 1..n-1,
    zero on the wall slot 0 (homogeneous Neumann); df[i] = delta_i the
    centre distances (n+1 entries, 1..n-1 used)."""
    n = len(df) - 1
    m = np.zeros((n, n))
    for i in range(1, n):
        m[i, i] = 1.0 / df[i]
        m[i, i - 1] = -1.0 / df[i]
    return m


def lx_mirror_walls(dc: np.ndarray, df: np.ndarray) -> np.ndarray:
    """(n x n) part of the Laplacian of a velocity cell-centred along a
    wall-bounded axis: D over the n+1 faces of the gradient whose wall faces
    take the mirror ghost (opposite sign, one cell away, at distance
    Delta/2): 2 f_0/Delta_0 and -2 f_{n-1}/Delta_{n-1}."""
    n = len(dc)
    G = np.zeros((n + 1, n))
    for i in range(1, n):
        G[i, i] = 1.0 / df[i]
        G[i, i - 1] = -1.0 / df[i]
    G[0, 0] = 2.0 / dc[0]
    G[n, n - 1] = -2.0 / dc[n - 1]
    D = np.zeros((n, n + 1))
    for i in range(n):
        D[i, i + 1] = 1.0 / dc[i]
        D[i, i] = -1.0 / dc[i]
    return D @ G


def _k3(az, ay, ax):
    return np.kron(az, np.kron(ay, ax))


def divergence_matrix(g: Grid) -> np.ndarray:
    """D: cells <- (u faces, v faces incl. walls, w faces)."""
    Ix, Iy, Iz = np.eye(g.nx), np.eye(g.ny), np.eye(g.nz)
    Dx = _circ_diff_fwd(g.nx, g.hx) if g.periodic_x else dx_faces_to_cells_walls(g.dxc)
    Du = _k3(Iz, Iy, Dx)
    Dv = _k3(Iz, dy_faces_to_cells_periodic(g) if g.periodic_y else dy_faces_to_cells(g), Ix)
    Dz = _circ_diff_fwd(g.nz, g.hz) if g.periodic_z else dx_faces_to_cells_walls(g.dzc)
    Dw = _k3(Dz, Iy, Ix)
    return np.hstack([Du, Dv, Dw])


def gradient_matrix(g: Grid) -> np.ndarray:
    """G: (u faces, v faces incl. walls, w faces) <- cells."""
    Ix, Iy, Iz = np.eye(g.nx), np.eye(g.ny), np.eye(g.nz)
    Gx = _circ_diff_bwd(g.nx, g.hx) if g.periodic_x else gx_cells_to_faces_walls(g.dxf)
    Gu = _k3(Iz, Iy, Gx)
    Gv = _k3(Iz, gy_cells_to_faces_periodic(g) if g.periodic_y else gy_cells_to_faces_neumann(g), Ix)
    Gz = _circ_diff_bwd(g.nz, g.hz) if g.periodic_z else gx_cells_to_faces_walls(g.dzf)
    Gw = _k3(Gz, Iy, Ix)
    return np.vstack([Gu, Gv, Gw])


def laplacian(g: Grid, op: int) -> np.ndarray:
    """Unweighted Laplacian over the unknowns of ``op`` (v: interior faces)."""
    Ix, Iz = np.eye(g.nx), np.eye(g.nz)
    if op == OP_P:
        return divergence_matrix(g) @ gradient_matrix(g)
    if g.periodic_x:
        Lx = _circ_diff_bwd(g.nx, g.hx) @ _circ_diff_fwd(g.nx, g.hx)
    elif op == OP_U:
        full = gx_cells_to_faces_walls(g.dxf) @ dx_faces_to_cells_walls(g.dxc)
        Lx = full[1:, 1:]
        Ix = np.eye(g.nx - 1)
    else:
        Lx = lx_mirror_walls(g.dxc, g.dxf)
    if g.periodic_z:
        Lz = _circ_diff_bwd(g.nz, g.hz) @ _circ_diff_fwd(g.nz, g.hz)
    elif op == OP_W:
        full = gx_cells_to_faces_walls(g.dzf) @ dx_faces_to_cells_walls(g.dzc)
        Lz = full[1:, 1:]
        Iz = np.eye(g.nz - 1)
    else:
        Lz = lx_mirror_walls(g.dzc, g.dzf)
    if g.periodic_y:
        Iy = np.eye(g.ny)
        if op in (OP_U, OP_W):
            Ly = dy_faces_to_cells_periodic(g) @ gy_cells_to_faces_periodic(g)
        elif op == OP_V:
            Ly = gy_cells_to_faces_periodic(g) @ dy_faces_to_cells_periodic(g)
        else:
            raise ValueError(op)
    elif op in (OP_U, OP_W):
        Ly = dy_faces_to_cells(g) @ gy_cells_to_faces_dirichlet_mirror(g)
        Iy = np.eye(g.ny)
    elif op == OP_V:
        full = gy_cells_to_faces_neumann(g) @ dy_faces_to_cells(g)
        Ly = full[1:g.ny, 1:g.ny]
        Iy = np.eye(g.ny - 1)
    else:
        raise ValueError(op)
    return _k3(Iz, Iy, Lx) + _k3(Iz, Ly, Ix) + _k3(Lz, Iy, Ix)


def weights(g: Grid, op: int) -> np.ndarray:
    nxu = g.nx - 1 if (op == OP_U and not g.periodic_x) else g.nx
    nzu = g.nz - 1 if (op == OP_W and not g.periodic_z) else g.nz
    if op == OP_V and g.periodic_y:
        wy = g.dyf[:g.ny]
        nyu = g.ny
    elif op == OP_V:
        wy = g.dyf[1:g.ny]
        nyu = g.ny - 1
    else:
        wy = g.dyc
        nyu = g.ny
    # control-cell widths in x and z: cells Delta, faces delta (slots 1..n-1)
    wx = g.dxf[1:g.nx] if (op == OP_U and not g.periodic_x) else g.dxc
    wz = g.dzf[1:g.nz] if (op == OP_W and not g.periodic_z) else g.dzc
    return (wz[:, None, None] * wy[None, :, None] * wx[None, None, :]).reshape(-1).copy()


def operator(g: Grid, op: int, c: float = 0.0) -> np.ndarray:
    L = laplacian(g, op)
    if op == OP_P:
        return L
    return np.eye(L.shape[0]) - c * L


def solve(g: Grid, op: int, b: np.ndarray, c: float = 0.0) -> np.ndarray:
    """Dense solve; b and the result in the full array layout."""
    walls = op == OP_V and not g.periodic_y
    xwalls = op == OP_U and not g.periodic_x
    zwalls = op == OP_W and not g.periodic_z
    if walls:
        rhs = np.ascontiguousarray(b[:, 1:g.ny, :]).reshape(-1)
    elif xwalls:
        rhs = np.ascontiguousarray(b[:, :, 1:]).reshape(-1)
    elif zwalls:
        rhs = np.ascontiguousarray(b[1:, :, :]).reshape(-1)
    else:
        rhs = np.ascontiguousarray(b).reshape(-1)
    A = operator(g, op, c)
    if op == OP_P:
        n = A.shape[0]
        w = weights(g, op)
        B = np.zeros((n + 1, n + 1))
        B[:n, :n] = A
        B[:n, n] = 1.0
        B[n, :n] = w
        sol = np.linalg.solve(B, np.concatenate([rhs, [0.0]]))[:n]
    else:
        sol = np.linalg.solve(A, rhs)
    out = np.zeros(g.shape(op))
    if walls:
        out[:, 1:g.ny, :] = sol.reshape(g.nz, g.ny - 1, g.nx)
    elif xwalls:
        out[:, :, 1:] = sol.reshape(g.nz, g.ny, g.nx - 1)
    elif zwalls:
        out[1:, :, :] = sol.reshape(g.nz - 1, g.ny, g.nx)
    else:
        out[...] = sol.reshape(g.shape(op))
    return out
