"""Reference (oracle) Runge-Kutta sub-step of the fractional-step method.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``): plain numpy written
from the sub-step's equations (Section 2.1, eqs. a-h), slow and direct.

One stage n with coefficients alpha, beta, gamma, zeta, time step dt and
Reynolds number Re:

  (a) u^e = u + dt [ (alpha+beta)/Re L u - (alpha+beta) G p
                     - gamma N(u) - zeta N(u^{n-2}) ]
  (b) U^e(X) = sum_xi u^e(x_xi) delta_h(x_xi - X) V_xi   (interpolation)
  (c) F(X) = (U^d(X) - U^e(X)) / dt
  (d) f(x_xi) = sum_eta F(X_eta) delta_h(x_xi - X_eta) dV_eta   (spreading)
  (e) (I - c L) u* = u^e - c L u + dt f,   c = beta dt / Re
  (f) L_p phi = D u* / ((alpha+beta) dt)
  (g) u^n = u* - (alpha+beta) dt G phi
  (h) p^n = p + phi - c L_p phi   (L_p phi taken as the right-hand side of f)

Discretisation (second-order central differences on the staggered grid,
Section 2.1): L, G, D, L_p as in orc.c (walls in y: Dirichlet velocity,
Neumann pressure; or periodic y); the convective term N(u) = div(u u) in
divergence form, each product formed on the face or edge where its
derivative needs it, from arithmetic means of the neighbouring values.
delta_h is the three-point kernel of Roma, Peskin and Berger in each
direction, scaled by the local spacing; the immersed-boundary part needs a
uniform spacing in y (beta = 0), as the paper's grid.
"""
from __future__ import annotations

import numpy as np

from . import Grid, OP_P, OP_U, OP_V, OP_W, divergence, gradient, solve


# ------------------------------------------------------------------------
# one-dimensional helpers along y (walls or periodic)
# ------------------------------------------------------------------------
def _yshift(a, s, g, axis=1):
    """a shifted so that out[j] = a[j + s] along y; with walls the values
    beyond the ends are zero (periodic: wrap)."""
    if g.periodic_y:
        return np.roll(a, -s, axis=axis)
    out = np.zeros_like(a)
    n = a.shape[axis]
    src = [slice(None)] * a.ndim
    dst = [slice(None)] * a.ndim
    if s > 0:
        src[axis] = slice(s, n)
        dst[axis] = slice(0, n - s)
    else:
        src[axis] = slice(0, n + s)
        dst[axis] = slice(-s, n)
    out[tuple(dst)] = a[tuple(src)]
    return out


def laplacian(g: Grid, op: int, f: np.ndarray) -> np.ndarray:
    """L f with the boundary conditions of op (as in orc.c's flux form):
    x, z periodic; y: Neumann (p), mirror ghost Dirichlet (u, w), wall
    faces zero (v), or periodic."""
    f = np.asarray(f, dtype=np.float64)
    out = ((np.roll(f, -1, 2) - f) - (f - np.roll(f, 1, 2))) / g.hx ** 2
    out += ((np.roll(f, -1, 0) - f) - (f - np.roll(f, 1, 0))) / g.hz ** 2
    ny = g.ny
    if g.periodic_y:
        fn, fs = np.roll(f, -1, 1), np.roll(f, 1, 1)
        if op == OP_V:
            dcs = np.roll(g.dyc, 1)     # Delta_{j-1}
            out += ((fn - f) / g.dyc[None, :, None] - (f - fs) / dcs[None, :, None]) \
                / g.dyf[None, :ny, None]
        else:
            out += ((fn - f) / g.dyf[None, 1:, None] - (f - fs) / g.dyf[None, :ny, None]) \
                / g.dyc[None, :, None]
        return out
    if op == OP_V:
        res = np.zeros_like(f)
        for j in range(1, ny):
            vu = f[:, j + 1, :] if j + 1 <= ny - 1 else 0.0
            vl = f[:, j - 1, :] if j - 1 >= 1 else 0.0
            res[:, j, :] = ((vu - f[:, j, :]) / g.dyc[j] - (f[:, j, :] - vl) / g.dyc[j - 1]) / g.dyf[j]
        out[:, 1:ny, :] += res[:, 1:ny, :]
        out[:, 0, :] = 0.0
        out[:, ny, :] = 0.0
        return out
    for j in range(ny):
        D = g.dyc[j]
        if j + 1 < ny:
            fu = (f[:, j + 1, :] - f[:, j, :]) / g.dyf[j + 1]
        else:
            fu = 0.0 if op == OP_P else -f[:, j, :] / (D / 2)
        if j > 0:
            fl = (f[:, j, :] - f[:, j - 1, :]) / g.dyf[j]
        else:
            fl = 0.0 if op == OP_P else f[:, j, :] / (D / 2)
        out[:, j, :] += (fu - fl) / D
    return out


# ------------------------------------------------------------------------
# convective term div(u u) on the staggered grid
# ------------------------------------------------------------------------
def convective(g: Grid, u, v, w):
    """(N_u, N_v, N_w) = div(u u) at the u, v and w faces.  Index
    conventions: u[k, j, i] at x-face i, v[k, j, i] at y-face j, w[k, j, i]
    at z-face k.  Walls (y = 0, ly): v = 0 there, so no product crosses
    them; N_v is zero on the wall faces."""
    u, v, w = (np.asarray(a, dtype=np.float64) for a in (u, v, w))
    hx, hz = g.hx, g.hz
    ny = g.ny
    Dy = g.dyc[None, :, None]
    # v at the y-faces below (j) and above (j+1) each cell row
    if g.periodic_y:
        v_lo, v_hi = v, np.roll(v, -1, 1)
    else:
        v_lo, v_hi = v[:, :ny, :], v[:, 1:, :]

    # ---- N_u at x-face (i, j, k)
    uc = 0.5 * (u + np.roll(u, -1, 2))                      # cell centre i (faces i, i+1)
    dxx = (uc ** 2 - np.roll(uc, 1, 2) ** 2) / hx            # centres i and i-1
    # y-flux v u on the edges (x-face i, y-face j), j = 0..ny (walls: 0)
    ve = 0.5 * (v + np.roll(v, 1, 2))                        # v at x-face i (cells i-1, i)
    if g.periodic_y:
        ue = 0.5 * (u + np.roll(u, 1, 1))                    # u at y-face j (cells j-1, j)
        fy = ve * ue
        dyy = (np.roll(fy, -1, 1) - fy) / Dy
    else:
        fy = np.zeros((g.nz, ny + 1, g.nx))
        fy[:, 1:ny, :] = ve[:, 1:ny, :] * 0.5 * (u[:, :ny - 1, :] + u[:, 1:, :])
        dyy = (fy[:, 1:, :] - fy[:, :ny, :]) / Dy
    we = 0.5 * (w + np.roll(w, 1, 2))                        # w at x-face i (z-face k)
    ue_z = 0.5 * (u + np.roll(u, 1, 0))                      # u at z-face k
    fz = we * ue_z
    dzz = (np.roll(fz, -1, 0) - fz) / hz
    Nu = dxx + dyy + dzz

    # ---- N_w at z-face (i, j, k): mirror of N_u with x <-> z
    wc = 0.5 * (w + np.roll(w, -1, 0))
    dzz_w = (wc ** 2 - np.roll(wc, 1, 0) ** 2) / hz
    vz = 0.5 * (v + np.roll(v, 1, 0))                        # v at z-face k
    if g.periodic_y:
        wy = 0.5 * (w + np.roll(w, 1, 1))
        fyw = vz * wy
        dyy_w = (np.roll(fyw, -1, 1) - fyw) / Dy
    else:
        fyw = np.zeros((g.nz, ny + 1, g.nx))
        fyw[:, 1:ny, :] = vz[:, 1:ny, :] * 0.5 * (w[:, :ny - 1, :] + w[:, 1:, :])
        dyy_w = (fyw[:, 1:, :] - fyw[:, :ny, :]) / Dy
    ux = 0.5 * (u + np.roll(u, 1, 0))                        # u at z-face k (x-face i)
    wx = 0.5 * (w + np.roll(w, 1, 2))                        # w at x-face i
    fxw = ux * wx
    dxx_w = (np.roll(fxw, -1, 2) - fxw) / hx
    Nw = dxx_w + dyy_w + dzz_w

    # ---- N_v at y-face (i, j, k)
    vc = 0.5 * (v_lo + v_hi)                                 # cell centres j
    Nv = np.zeros_like(v)
    if g.periodic_y:
        dyy_v = (vc ** 2 - np.roll(vc, 1, 1) ** 2) / g.dyf[None, :ny, None]
        uy = 0.5 * (u + np.roll(u, 1, 1))                    # u at y-face j (x-face i)
        wy2 = 0.5 * (w + np.roll(w, 1, 1))                   # w at y-face j (z-face k)
        vx = 0.5 * (v + np.roll(v, 1, 2))                    # v at x-face i
        vz2 = 0.5 * (v + np.roll(v, 1, 0))                   # v at z-face k
        fxv = uy * vx
        fzv = wy2 * vz2
        Nv = dyy_v + (np.roll(fxv, -1, 2) - fxv) / hx + (np.roll(fzv, -1, 0) - fzv) / hz
        return Nu, Nv, Nw
    for j in range(1, ny):
        d = g.dyf[j]
        dyy_v = (vc[:, j, :] ** 2 - vc[:, j - 1, :] ** 2) / d
        uy = 0.5 * (u[:, j - 1, :] + u[:, j, :])             # u at y-face j, x-face i
        vx = 0.5 * (v[:, j, :] + np.roll(v[:, j, :], 1, 1))  # v at x-face i
        fxv = uy * vx
        wy2 = 0.5 * (w[:, j - 1, :] + w[:, j, :])            # w at y-face j, z-face k
        vz2 = 0.5 * (v[:, j, :] + np.roll(v[:, j, :], 1, 0))
        fzv = wy2 * vz2
        Nv[:, j, :] = dyy_v + (np.roll(fxv, -1, 1) - fxv) / hx + (np.roll(fzv, -1, 0) - fzv) / hz
    return Nu, Nv, Nw


# ------------------------------------------------------------------------
# immersed boundary: Roma three-point kernel on the staggered grids
# ------------------------------------------------------------------------
def roma3(r):
    """Three-point regularised delta of Roma, Peskin and Berger (1999), in
    grid units (sums to one over any unit-spaced lattice)."""
    a = np.abs(np.asarray(r, dtype=np.float64))
    out = np.zeros_like(a)
    m1 = a <= 0.5
    out[m1] = (1.0 + np.sqrt(1.0 - 3.0 * a[m1] ** 2)) / 3.0
    m2 = (a > 0.5) & (a <= 1.5)
    out[m2] = (5.0 - 3.0 * a[m2] - np.sqrt(np.maximum(0.0, 1.0 - 3.0 * (1.0 - a[m2]) ** 2))) / 6.0
    return out


def _support(g: Grid, comp: int, X):
    """Indices and 1-D weights of the 3 x 3 x 3 lattice points of component
    comp (0 u, 1 v, 2 w) around marker X (physical coordinates), for a grid
    with uniform spacing in y.  Returns (kk, jj, ii, wz, wy, wx, valid_y)."""
    hy = g.ly / g.ny
    off = [(0.0, 0.5, 0.5), (0.5, 0.0, 0.5), (0.5, 0.5, 0.0)][comp]    # (x, y, z) offsets
    p = (X[0] / g.hx - off[0], X[1] / hy - off[1], X[2] / g.hz - off[2])
    idx = [int(np.floor(q + 0.5)) + np.arange(-1, 2) for q in p]
    wts = [roma3(ii - q) for ii, q in zip(idx, p)]
    ii, jj, kk = idx
    rows = g.shape(OP_V if comp == 1 else OP_U)[1]
    if g.periodic_y:
        valid = np.ones(3, dtype=bool)
        jj = jj % g.ny
    else:
        valid = (jj >= 0) & (jj < rows)
    return kk % g.nz, jj, ii % g.nx, wts[2], wts[1], wts[0], valid


def interpolate(g: Grid, fields, markers):
    """(b): U(X_eta) = sum_xi u(x_xi) delta_h(x_xi - X_eta) V_xi for each
    component; returns [nm][3]."""
    out = np.zeros((len(markers), 3))
    for m, X in enumerate(markers):
        for comp in range(3):
            kk, jj, ii, wz, wy, wx, ok = _support(g, comp, X)
            f = fields[comp]
            s = 0.0
            for a in range(3):
                for b in range(3):
                    if not ok[b]:
                        continue
                    for c_ in range(3):
                        s += f[kk[a], jj[b], ii[c_]] * wz[a] * wy[b] * wx[c_]
            out[m, comp] = s
    return out


def spread(g: Grid, F, markers, dvol):
    """(d): f(x_xi) = sum_eta F(X_eta) delta_h(x_xi - X_eta) dV_eta on the
    three face grids (delta_h = product of the 1-D kernels over the
    spacings)."""
    hy = g.ly / g.ny
    vol = g.hx * hy * g.hz
    out = [np.zeros(g.shape(op)) for op in (OP_U, OP_V, OP_W)]
    for m, X in enumerate(markers):
        for comp in range(3):
            kk, jj, ii, wz, wy, wx, ok = _support(g, comp, X)
            for a in range(3):
                for b in range(3):
                    if not ok[b]:
                        continue
                    for c_ in range(3):
                        out[comp][kk[a], jj[b], ii[c_]] += F[m, comp] * wz[a] * wy[b] * wx[c_] * dvol[m] / vol
    return out


# ------------------------------------------------------------------------
# one Runge-Kutta stage
# ------------------------------------------------------------------------
def stage(g: Grid, u, v, w, p, coef, n_prev=None, markers=None, ud=None, dvol=None):
    """One sub-step (eqs. a-h).  coef: dict alpha, beta, gamma, zeta, dt, re.
    n_prev: (N_u, N_v, N_w) of the stage before (needed when zeta != 0).
    Returns dict with u, v, w, p (the new fields), n (N of the input
    velocity, for the next stage), force ([nm][3] or None), phi, ue."""
    if not g.periodic_x:
        raise ValueError("the sub-step is written for a periodic x")
    al, be, ga, ze = (coef[k] for k in ("alpha", "beta", "gamma", "zeta"))
    dt, re = coef["dt"], coef["re"]
    vel = [np.asarray(a, dtype=np.float64) for a in (u, v, w)]
    ops = (OP_U, OP_V, OP_W)
    N = convective(g, *vel)
    gp = gradient(g, p)
    Lu = [laplacian(g, op, f) for op, f in zip(ops, vel)]
    ue = []
    for q in range(3):
        e = vel[q] + dt * ((al + be) / re * Lu[q] - (al + be) * gp[q] - ga * N[q])
        if ze != 0.0:
            e = e - dt * ze * n_prev[q]
        ue.append(e)
    if not g.periodic_y:
        ue[1][:, 0, :] = 0.0
        ue[1][:, g.ny, :] = 0.0
    force = None
    f = [np.zeros_like(a) for a in vel]
    if markers is not None and len(markers):
        Ue = interpolate(g, ue, markers)
        force = (np.asarray(ud) - Ue) / dt
        f = spread(g, force, markers, dvol)
    c = be * dt / re
    star = []
    for q, op in enumerate(ops):
        rhs = ue[q] - c * Lu[q] + dt * f[q]
        x, _ = solve(g, op, rhs, c=c)
        star.append(x)
    b = divergence(g, *star, scale=1.0 / ((al + be) * dt))
    phi, _ = solve(g, OP_P, b)
    gphi = gradient(g, phi)
    new = [star[q] - (al + be) * dt * gphi[q] for q in range(3)]
    if not g.periodic_y:
        new[1][:, 0, :] = 0.0
        new[1][:, g.ny, :] = 0.0
    pn = np.asarray(p, dtype=np.float64) + phi - c * b
    return dict(u=new[0], v=new[1], w=new[2], p=pn, n=N, force=force, phi=phi, ue=ue, b=b)
