// Kernels of the Runge-Kutta sub-step around the linear solves (Section 2.1,
// eqs. a-e; kernels E1 and L1 of Section 2.3.2).
//
// explicit_kernel (E1): for every face of the three staggered grids,
//   u^e = u + dt [ (alpha+beta)/Re L u - (alpha+beta) G p
//                  - gamma N(u) - zeta N_prev ]                    (eq. a)
// together with the Helmholtz right-hand side without the forcing,
//   r = u^e - c L u,  c = beta dt / Re                             (eq. e)
// and N(u) itself (kept for the next stage's zeta term).  N is the
// convective term in divergence form, each product formed on the face or
// edge where its derivative needs it from arithmetic means of the
// neighbouring values; with walls, v = 0 on the wall faces and no product
// crosses them.  One thread per (i, j, k): the u and w faces of cell (i, j,
// k) and the v face j below it (rows 0..ny with walls: the wall faces get
// zeros); x fastest across the lanes, neighbours through L2.
//
// ibm_kernel (L1): one thread per marker: for each component, the 3 x 3 x 3
// support of the Roma three-point kernel on that component's grid,
// U^e(X) = sum u^e(x) w (eq. b), F = (U^d - U^e)/dt (eq. c), and
// r += dt F w dV / (hx hy hz) at each support point (eq. d, the spreading
// added straight into the Helmholtz right-hand side) by atomic adds, as
// the paper's L1 does.  Needs a uniform spacing in y (as the paper's grid).
#include "ibs_internal.h"

#include <cmath>

namespace ibs {

struct FsGeo {
    int nx, ny, nz, py;
    double hx, hz, hy;           // hy: uniform y spacing (immersed boundary only)
    const double *dyc, *dyf;     // Delta_j [ny], delta_j [ny+1]
};

struct FsCoef {
    double ab;     // alpha + beta
    double gam, zet, dt, re, c;
};

// y rows of v: ny + 1 with walls, ny when periodic
static __device__ __forceinline__ int vrows(const FsGeo &g) { return g.py ? g.ny : g.ny + 1; }

__global__ __launch_bounds__(256) void explicit_kernel(FsGeo g, FsCoef cf, const double *__restrict__ u,
                                                       const double *__restrict__ v,
                                                       const double *__restrict__ w,
                                                       const double *__restrict__ p,
                                                       const double *nu_prev, const double *nv_prev,
                                                       const double *nw_prev, double *ue, double *ve,
                                                       double *we, double *ru, double *rv, double *rw,
                                                       double *nu_out, double *nv_out, double *nw_out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y, k = blockIdx.z;
    if (i >= g.nx) return;
    const int nx = g.nx, ny = g.ny, nz = g.nz, vr = vrows(g);
    const int ip = i + 1 == nx ? 0 : i + 1, im = i == 0 ? nx - 1 : i - 1;
    const int kp = k + 1 == nz ? 0 : k + 1, km = k == 0 ? nz - 1 : k - 1;
    // cell fields (u, w, p: [nz][ny][nx]) and v ([nz][vr][nx])
    auto C = [&](const double *a, int kk, int jj, int ii) { return a[((size_t)kk * ny + jj) * nx + ii]; };
    auto V = [&](int kk, int jj, int ii) {
        // wall faces read as zero (their stored values are ignored)
        if (!g.py && (jj <= 0 || jj >= ny)) return 0.0;
        if (g.py) jj = jj < 0 ? jj + ny : (jj >= ny ? jj - ny : jj);
        return v[((size_t)kk * vr + jj) * nx + ii];
    };
    const double ihx = 1.0 / g.hx, ihz = 1.0 / g.hz;
    const double vis = cf.ab / cf.re;
    const bool zprev = cf.zet != 0.0;

    if (j < ny) {
        const size_t o = ((size_t)k * ny + j) * nx + i;
        const int jn = j + 1 < ny ? j + 1 : (g.py ? 0 : -1);   // -1: wall above
        const int js = j > 0 ? j - 1 : (g.py ? ny - 1 : -1);   // -1: wall below
        const double D = g.dyc[j];
        // y part of the Laplacian of a cell-height field f at row j (mirror
        // ghost at a wall; fluxes over delta, delta_0 = delta_ny across the
        // periodic wrap)
        auto lapy = [&](const double *f) {
            const double fc = C(f, k, j, i);
            const double fu = jn >= 0 ? (C(f, k, jn, i) - fc) / g.dyf[j + 1] : -fc / (0.5 * D);
            const double fl = js >= 0 ? (fc - C(f, k, js, i)) / g.dyf[j] : fc / (0.5 * D);
            return (fu - fl) / D;
        };
        // ---- u at x-face (i, j, k)
        {
            const double uc = C(u, k, j, i);
            const double lap = (C(u, k, j, ip) - 2.0 * uc + C(u, k, j, im)) * ihx * ihx +
                               (C(u, kp, j, i) - 2.0 * uc + C(u, km, j, i)) * ihz * ihz + lapy(u);
            const double gp = (C(p, k, j, i) - C(p, k, j, im)) * ihx;
            const double c1 = 0.5 * (uc + C(u, k, j, ip)), c0 = 0.5 * (C(u, k, j, im) + uc);
            const double dxx = (c1 * c1 - c0 * c0) * ihx;
            // y fluxes v u on the faces j (below) and j+1 (above) at x-face i
            const double fb = js >= 0 ? 0.5 * (V(k, j, i) + V(k, j, im)) * 0.5 * (C(u, k, js, i) + uc) : 0.0;
            const double ft = jn >= 0 ? 0.5 * (V(k, j + 1, i) + V(k, j + 1, im)) * 0.5 * (uc + C(u, k, jn, i)) : 0.0;
            const double dyy = (ft - fb) / D;
            const double zb = 0.5 * (C(w, k, j, i) + C(w, k, j, im)) * 0.5 * (C(u, km, j, i) + uc);
            const double zt = 0.5 * (C(w, kp, j, i) + C(w, kp, j, im)) * 0.5 * (uc + C(u, kp, j, i));
            const double N = dxx + dyy + (zt - zb) * ihz;
            double e = uc + cf.dt * (vis * lap - cf.ab * gp - cf.gam * N);
            if (zprev) e -= cf.dt * cf.zet * nu_prev[o];
            ue[o] = e;
            ru[o] = e - cf.c * lap;
            nu_out[o] = N;
        }
        // ---- w at z-face (i, j, k): the x <-> z mirror of u
        {
            const double wc = C(w, k, j, i);
            const double lap = (C(w, k, j, ip) - 2.0 * wc + C(w, k, j, im)) * ihx * ihx +
                               (C(w, kp, j, i) - 2.0 * wc + C(w, km, j, i)) * ihz * ihz + lapy(w);
            const double gp = (C(p, k, j, i) - C(p, km, j, i)) * ihz;
            const double c1 = 0.5 * (wc + C(w, kp, j, i)), c0 = 0.5 * (C(w, km, j, i) + wc);
            const double dzz = (c1 * c1 - c0 * c0) * ihz;
            const double fb = js >= 0 ? 0.5 * (V(k, j, i) + V(km, j, i)) * 0.5 * (C(w, k, js, i) + wc) : 0.0;
            const double ft = jn >= 0 ? 0.5 * (V(k, j + 1, i) + V(km, j + 1, i)) * 0.5 * (wc + C(w, k, jn, i)) : 0.0;
            const double dyy = (ft - fb) / D;
            const double xb = 0.5 * (C(u, k, j, i) + C(u, km, j, i)) * 0.5 * (C(w, k, j, im) + wc);
            const double xt = 0.5 * (C(u, k, j, ip) + C(u, km, j, ip)) * 0.5 * (wc + C(w, k, j, ip));
            const double N = (xt - xb) * ihx + dyy + dzz;
            double e = wc + cf.dt * (vis * lap - cf.ab * gp - cf.gam * N);
            if (zprev) e -= cf.dt * cf.zet * nw_prev[o];
            we[o] = e;
            rw[o] = e - cf.c * lap;
            nw_out[o] = N;
        }
    }
    // ---- v at y-face (i, j, k)
    if (j < vr) {
        const size_t o = ((size_t)k * vr + j) * nx + i;
        if (!g.py && (j == 0 || j == ny)) {   // wall faces
            ve[o] = 0.0;
            rv[o] = 0.0;
            nv_out[o] = 0.0;
            return;
        }
        const int jm = j > 0 ? j - 1 : ny - 1;       // cell below the face (wraps when periodic)
        const int jc = j;                            // cell above the face (j < ny here)
        const double vc = V(k, j, i);
        const double d = g.dyf[j];
        const double lapy = ((V(k, j + 1, i) - vc) / g.dyc[jc] - (vc - V(k, j - 1, i)) / g.dyc[jm]) / d;
        const double lap = (V(k, j, ip) - 2.0 * vc + V(k, j, im)) * ihx * ihx +
                           (V(kp, j, i) - 2.0 * vc + V(km, j, i)) * ihz * ihz + lapy;
        const double gp = (C(p, k, jc, i) - C(p, k, jm, i)) / d;
        const double c1 = 0.5 * (vc + V(k, j + 1, i)), c0 = 0.5 * (V(k, j - 1, i) + vc);
        const double dyy = (c1 * c1 - c0 * c0) / d;
        // x fluxes u v on the x-faces i and i+1 at y-face j
        const double xb = 0.5 * (C(u, k, jm, i) + C(u, k, jc, i)) * 0.5 * (vc + V(k, j, im));
        const double xt = 0.5 * (C(u, k, jm, ip) + C(u, k, jc, ip)) * 0.5 * (V(k, j, ip) + vc);
        const double zb = 0.5 * (C(w, k, jm, i) + C(w, k, jc, i)) * 0.5 * (vc + V(km, j, i));
        const double zt = 0.5 * (C(w, kp, jm, i) + C(w, kp, jc, i)) * 0.5 * (V(kp, j, i) + vc);
        const double N = (xt - xb) * ihx + dyy + (zt - zb) * ihz;
        double e = vc + cf.dt * (vis * lap - cf.ab * gp - cf.gam * N);
        if (zprev) e -= cf.dt * cf.zet * nv_prev[o];
        ve[o] = e;
        rv[o] = e - cf.c * lap;
        nv_out[o] = N;
    }
}

// Roma, Peskin and Berger's three-point regularised delta, grid units.
static __device__ __forceinline__ double roma3(double r)
{
    const double a = fabs(r);
    if (a <= 0.5) return (1.0 + sqrt(1.0 - 3.0 * a * a)) / 3.0;
    if (a <= 1.5) {
        const double t = 1.0 - a;
        return (5.0 - 3.0 * a - sqrt(fmax(0.0, 1.0 - 3.0 * t * t))) / 6.0;
    }
    return 0.0;
}

__global__ __launch_bounds__(64) void ibm_kernel(FsGeo g, double dt, int nm, const double *__restrict__ X,
                                                 const double *__restrict__ ud,
                                                 const double *__restrict__ dvol,
                                                 const double *__restrict__ ue,
                                                 const double *__restrict__ ve,
                                                 const double *__restrict__ we, double *ru, double *rv,
                                                 double *rw, double *force)
{
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= nm) return;
    const double vol = g.hx * g.hy * g.hz;
    const double scale = dt * dvol[m] / vol;
    for (int comp = 0; comp < 3; ++comp) {
        // staggered offsets (x, y, z) of the component, in grid units
        const double ox = comp == 0 ? 0.0 : 0.5, oy = comp == 1 ? 0.0 : 0.5, oz = comp == 2 ? 0.0 : 0.5;
        const double px = X[3 * m] / g.hx - ox, py = X[3 * m + 1] / g.hy - oy, pz = X[3 * m + 2] / g.hz - oz;
        const int bx = (int)floor(px + 0.5) - 1, by = (int)floor(py + 0.5) - 1, bz = (int)floor(pz + 0.5) - 1;
        const int rows = comp == 1 ? vrows(g) : g.ny;
        const double *f = comp == 0 ? ue : (comp == 1 ? ve : we);
        double *r = comp == 0 ? ru : (comp == 1 ? rv : rw);
        double wx[3], wy[3], wz[3];
        int ix[3], iy[3], iz[3];
        bool oky[3];
        for (int t = 0; t < 3; ++t) {
            wx[t] = roma3(bx + t - px);
            wy[t] = roma3(by + t - py);
            wz[t] = roma3(bz + t - pz);
            ix[t] = ((bx + t) % g.nx + g.nx) % g.nx;
            iz[t] = ((bz + t) % g.nz + g.nz) % g.nz;
            int jy = by + t;
            if (g.py) {
                jy = (jy % g.ny + g.ny) % g.ny;
                oky[t] = true;
            } else {
                oky[t] = jy >= 0 && jy < rows;
            }
            iy[t] = jy;
        }
        double U = 0.0;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                if (!oky[b]) continue;
                for (int c = 0; c < 3; ++c)
                    U += f[((size_t)iz[a] * rows + iy[b]) * g.nx + ix[c]] * wz[a] * wy[b] * wx[c];
            }
        const double F = (ud[3 * m + comp] - U) / dt;
        if (force) force[3 * m + comp] = F;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                if (!oky[b]) continue;
                for (int c = 0; c < 3; ++c)
                    atomicAdd(&r[((size_t)iz[a] * rows + iy[b]) * g.nx + ix[c]],
                              F * wz[a] * wy[b] * wx[c] * scale);
            }
    }
}

static FsGeo fs_geo(const Plan &p)
{
    FsGeo g;
    g.nx = p.nx; g.ny = p.ny; g.nz = p.nz; g.py = p.py ? 1 : 0;
    g.hx = p.hx; g.hz = p.hz; g.hy = p.desc.ly / p.ny;
    g.dyc = blob_ptr(p, p.lay.dyc);
    g.dyf = blob_ptr(p, p.lay.dyf);
    return g;
}

hipError_t launch_explicit(const Plan &p, const FsStage &s, hipStream_t st)
{
    FsGeo g = fs_geo(p);
    FsCoef cf;
    cf.ab = s.alpha + s.beta;
    cf.gam = s.gamma;
    cf.zet = s.zeta;
    cf.dt = s.dt;
    cf.re = s.re;
    cf.c = s.beta * s.dt / s.re;
    const int blk = p.nx >= 256 ? 256 : ((p.nx + 63) / 64) * 64;
    dim3 grid((p.nx + blk - 1) / blk, p.py ? p.ny : p.ny + 1, p.nz);
    hipLaunchKernelGGL(explicit_kernel, grid, dim3(blk), 0, st, g, cf, s.u, s.v, s.w, s.p, s.nu, s.nv, s.nw,
                       s.ue, s.ve, s.we, s.ru, s.rv, s.rw, s.nu, s.nv, s.nw);
    return hipGetLastError();
}

hipError_t launch_ibm(const Plan &p, const FsStage &s, hipStream_t st)
{
    if (s.nmarkers <= 0) return hipSuccess;
    FsGeo g = fs_geo(p);
    hipLaunchKernelGGL(ibm_kernel, dim3((s.nmarkers + 63) / 64), dim3(64), 0, st, g, s.dt, s.nmarkers,
                       s.markers, s.ud, s.dvol, s.ue, s.ve, s.we, s.ru, s.rv, s.rw, s.force);
    return hipGetLastError();
}

}  // namespace ibs
