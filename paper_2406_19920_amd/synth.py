"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module holds no arithmetic of the solver: it only draws random fields
(numpy PCG64 ``default_rng``), low-pass filters them in index space and
synthesises an immersed-boundary-like forcing shell.  Discrete operators
(divergence, Laplacians) are applied by each side on its own.

Layout: C order [z][y][x]; u, w are [nz][ny][nx]; v is [nz][ny+1][nx] with
the wall faces j = 0 and j = ny included.
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft


def velocity(nx: int, ny: int, nz: int, seed: int):
    """i.i.d. N(0,1) face velocities, drawn in the order u, v, w, each in
    C order; v includes its wall faces."""
    rng = np.random.default_rng(seed)
    u = rng.standard_normal((nz, ny, nx))
    v = rng.standard_normal((nz, ny + 1, nx))
    w = rng.standard_normal((nz, ny, nx))
    return u, v, w


def scalar(nx: int, ny: int, nz: int, seed: int, rows: int | None = None):
    """One i.i.d. N(0,1) field of shape [nz][rows or ny][nx]."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((nz, ny if rows is None else rows, nx))


def lowpass(f: np.ndarray, kmax: float = 16.0) -> np.ndarray:
    """Keep modes with sqrt(kx^2 + ky^2 + kz^2) <= kmax in index space:
    kx, kz are the (signed) periodic DFT indices, ky the DCT-II index along
    y.  Used to make smooth, channel-like synthetic fields."""
    nz, ny, nx = f.shape
    F = sfft.rfft(f, axis=2)
    F = sfft.fft(F, axis=0)
    F = sfft.dct(F.real, type=2, axis=1, norm="ortho") + 1j * sfft.dct(F.imag, type=2, axis=1, norm="ortho")
    kx = np.arange(F.shape[2])
    kz = np.fft.fftfreq(nz, d=1.0 / nz)
    ky = np.arange(ny)
    K2 = kz[:, None, None] ** 2 + ky[None, :, None] ** 2 + kx[None, None, :] ** 2
    F = np.where(K2 <= kmax * kmax, F, 0.0)
    F = sfft.idct(F.real, type=2, axis=1, norm="ortho") + 1j * sfft.idct(F.imag, type=2, axis=1, norm="ortho")
    F = sfft.ifft(F, axis=0)
    return np.ascontiguousarray(sfft.irfft(F, n=nx, axis=2))


def filtered_velocity(nx: int, ny: int, nz: int, seed: int, kmax: float = 16.0,
                      zero_wall_v: bool = True):
    """N(0,1) face velocities low-pass filtered to index radius kmax; the
    wall faces of v are set to zero after filtering when requested."""
    u, v, w = velocity(nx, ny, nz, seed)
    u, v, w = lowpass(u, kmax), lowpass(v, kmax), lowpass(w, kmax)
    if zero_wall_v:
        v[:, 0, :] = 0.0
        v[:, ny, :] = 0.0
    return u, v, w


def _roma3(r: np.ndarray) -> np.ndarray:
    """Three-point regularised delta kernel of Roma, Peskin and Berger
    (1999), in index units; it sums to one over any unit-spaced lattice."""
    a = np.abs(r)
    out = np.zeros_like(a)
    m1 = a <= 0.5
    out[m1] = (1.0 + np.sqrt(1.0 - 3.0 * a[m1] ** 2)) / 3.0
    m2 = (a > 0.5) & (a <= 1.5)
    out[m2] = (5.0 - 3.0 * a[m2] - np.sqrt(np.maximum(0.0, 1.0 - 3.0 * (1.0 - a[m2]) ** 2))) / 6.0
    return out


def forcing_shell(nx: int, ny: int, nz: int, seed: int, radius_frac: float = 0.1):
    """Immersed-boundary-like source: markers on a sphere (Fibonacci
    lattice) of radius radius_frac * nx index units, centre uniform in
    [0.3, 0.7] of each index extent, marker forces N(0,1)^3, spread to the
    three staggered face grids with the Roma kernel in index space.  The
    geometry lives in index space (stretching is ignored): it is a synthetic
    source, not a physical body.  Returns (fu, fv, fw)."""
    rng = np.random.default_rng(seed)
    centre = rng.uniform(0.3, 0.7, size=3) * np.array([nx, ny, nz], dtype=np.float64)
    R = radius_frac * nx
    nmark = max(8, int(round(4.0 * np.pi * R * R)))
    q = np.arange(nmark) + 0.5
    zc = 1.0 - 2.0 * q / nmark
    th = np.pi * (1.0 + 5.0 ** 0.5) * q
    rr = np.sqrt(np.maximum(0.0, 1.0 - zc * zc))
    X = centre[0] + R * rr * np.cos(th)
    Y = centre[1] + R * rr * np.sin(th)
    Z = centre[2] + R * zc
    F = rng.standard_normal((nmark, 3))
    fu = np.zeros((nz, ny, nx))
    fv = np.zeros((nz, ny + 1, nx))
    fw = np.zeros((nz, ny, nx))
    # staggered positions in index units: u (i, j+.5, k+.5), v (i+.5, j, k+.5),
    # w (i+.5, j+.5, k)
    for comp, (arr, off) in enumerate(((fu, (0.0, 0.5, 0.5)), (fv, (0.5, 0.0, 0.5)),
                                       (fw, (0.5, 0.5, 0.0)))):
        nyr = arr.shape[1]
        for m in range(nmark):
            px, py, pz = X[m] - off[0], Y[m] - off[1], Z[m] - off[2]
            ix0, iy0, iz0 = int(np.floor(px)) - 1, int(np.floor(py)) - 1, int(np.floor(pz)) - 1
            ii = np.arange(ix0, ix0 + 4)
            jj = np.arange(iy0, iy0 + 4)
            kk = np.arange(iz0, iz0 + 4)
            wx, wy, wz = _roma3(ii - px), _roma3(jj - py), _roma3(kk - pz)
            ok = (jj >= 0) & (jj < nyr)
            wgt = wz[:, None, None] * wy[None, :, None] * wx[None, None, :] * F[m, comp]
            wgt = wgt[:, ok, :]
            arr[np.ix_(kk % nz, jj[ok], ii % nx)] += wgt
    return fu, fv, fw


def sphere_markers(count: int, radius: float, centre=(0.5, 0.5, 0.5)) -> np.ndarray:
    """count points spread evenly over a sphere (golden-angle spiral), as
    [count][3] physical coordinates (x, y, z): the Lagrangian markers of a
    synthetic immersed body."""
    q = np.arange(count) + 0.5
    zc = 1.0 - 2.0 * q / count
    th = np.pi * (1.0 + 5.0 ** 0.5) * q
    r = np.sqrt(np.maximum(0.0, 1.0 - zc * zc))
    return np.stack([centre[0] + radius * r * np.cos(th), centre[1] + radius * r * np.sin(th),
                     centre[2] + radius * zc], axis=1)


def manufactured(nx: int, ny: int, nz: int, seed: int, rows: int | None = None,
                 kmax: float | None = 8.0, noise: float = 1e-3):
    """A smooth seeded field plus a small white-noise part: used as a known
    exact solution x_true (the right-hand side A x_true is then formed by
    whichever side is being checked)."""
    f = scalar(nx, ny, nz, seed, rows)
    g = lowpass(f, kmax) if kmax is not None else np.zeros_like(f)
    return g + noise * scalar(nx, ny, nz, seed + 7919, rows)


# Grid sizes (nx, ny, nz) of the mixed-size batch workload.
BATCH_SIZES = ((64, 64, 64), (96, 128, 96), (128, 128, 128), (192, 256, 192))


def batch_specs(njobs: int = 64, seed: int = 4, sizes=BATCH_SIZES, beta_max: float = 3.0):
    """Job list of the mixed-size batch: sizes uniform over ``sizes``,
    tanh stretching beta ~ U[0, beta_max], per-job seeds 1000 + i."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(njobs):
        nx, ny, nz = sizes[int(rng.integers(0, len(sizes)))]
        out.append(dict(nx=nx, ny=ny, nz=nz, beta=float(rng.uniform(0.0, beta_max)),
                        seed=1000 + i))
    return out


def device_normal(shape, seed: int, device):
    """Seeded N(0,1) FP64 field generated on the device (torch's Philox
    generator); used where host generation of large batches would dominate."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    return torch.randn(shape, generator=g, dtype=torch.float64, device=device)


def serving_requests(rate: float, count: int, seed: int, nmin: int = 32, nmax: int = 384,
                     multiple: int = 16, multiple_refined: int = 32, beta_max: float = 3.0,
                     geometries: int = 0):
    """Request stream of the serving workload: Poisson-process arrivals at
    `rate` per second; kind 50/50 pressure Poisson or Helmholtz x3; precision
    50/50 FP64 or refined; cubic grid n log-uniform on [nmin, nmax], rounded
    to a multiple of `multiple` (FP64 requests) or `multiple_refined`
    (refined requests: the split matrix-core path takes multiples of 32);
    tanh beta ~ U[0, beta_max]; per-request seeds.  With `geometries` > 0
    the (n, beta) pairs are drawn once into a pool of that many and each
    request takes one of them uniformly (clients re-solving on a few grids,
    so plans can be reused; n is rounded per request as above); with 0
    every request draws its own grid.  Returns a list of dicts sorted by
    arrival time (seconds)."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=count)
    t = np.cumsum(gaps) - gaps[0]

    def rounded(n, m):
        return int(max(m, min(nmax - nmax % m, m * round(n / m))))

    def grid(g):
        return float(np.exp(g.uniform(np.log(nmin), np.log(nmax)))), float(g.uniform(0.0, beta_max))

    pool = None
    if geometries > 0:
        g = np.random.default_rng([seed, geometries])
        pool = [grid(g) for _ in range(geometries)]
    out = []
    for i in range(count):
        if pool is None:
            nraw = float(np.exp(rng.uniform(np.log(nmin), np.log(nmax))))
        else:
            nraw, beta = pool[int(rng.integers(geometries))]
        kind = "poisson" if rng.random() < 0.5 else "helmholtz"
        refined = bool(rng.random() < 0.5)
        if pool is None:
            beta = float(rng.uniform(0.0, beta_max))
        n = rounded(nraw, multiple_refined if refined else multiple)
        out.append(dict(rid=i, arrival=float(t[i]), kind=kind, refined=refined, n=n,
                        beta=beta, seed=int(seed * 100003 + i)))
    return out
