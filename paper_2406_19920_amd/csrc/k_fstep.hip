// Kernels of the Runge-Kutta sub-step around the linear solves (Section 2.1,
// eqs. a-e; kernels E1 and L1 of Section 2.3.2).
//
// explicit_kernel (E1): for every face of the three staggered grids,
//   u^e = u + dt [ (alpha+beta)/Re L u - (alpha+beta) G p
//                  - gamma N(u) - zeta N_prev ]                    (eq. a)
// together with the Helmholtz right-hand side without the forcing,
//   r = u^e - c L u,  c = beta dt / Re                             (eq. e)
// and N(u) itself (kept for the next stage's zeta term); u^e is written only
// when markers will interpolate it.  N is the
// convective term in divergence form, each product formed on the face or
// edge where its derivative needs it from arithmetic means of the
// neighbouring values; with walls, v = 0 on the wall faces and no product
// crosses them.  One thread per (i, j) of a block's tile, marching in z:
// the u and w faces of cell (i, j, k) and the v face j below it (rows
// 0..ny with walls: the wall faces get zeros); neighbours from an LDS ring
// of three planes.
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

// Tiling of the explicit kernel: a block owns ETX x ETY (x, y) points, one
// thread each, and marches through EKZ consecutive z planes.  The planes
// k-1, k, k+1 of u, v, w, p sit in LDS as a ring of three tiles with a
// one-point halo in x and y, so each plane of each field is read from HBM
// once per block (plus the halo, which the neighbouring tiles on the same
// XCD share in L2) instead of once per neighbour; the loads of plane k+2
// are in flight while plane k is computed.  (A four-slot ring with one
// barrier per plane needs 32 x 8 tiles to fit beside a second block and
// measured slower: three waves per SIMD instead of four.)
constexpr int ETX = 32, ETY = 16, ENT = ETX * ETY;
constexpr int EHX = ETX + 2, EHY = ETY + 2, EPL = EHX * EHY;
constexpr int EKZ = 16;                               // nz is a multiple of 16
constexpr int EPER = (4 * EPL + ENT - 1) / ENT;       // staged values per thread and plane

__global__ __launch_bounds__(ENT) void explicit_kernel(FsGeo g, FsCoef cf, const double *__restrict__ u,
                                                       const double *__restrict__ v,
                                                       const double *__restrict__ w,
                                                       const double *__restrict__ p,
                                                       const double *nu_prev, const double *nv_prev,
                                                       const double *nw_prev, double *ue, double *ve,
                                                       double *we, double *ru, double *rv, double *rw,
                                                       double *nu_out, double *nv_out, double *nw_out,
                                                       int keep_ue)
{
    __shared__ double sm[3][4 * EPL];   // ring slot, then field (u, v, w, p) x tile
    const int nx = g.nx, ny = g.ny, nz = g.nz, vr = vrows(g);
    // XCD-aware order: the hardware deals consecutive blocks to the 8 XCDs
    // in turn; block b takes tile (b % 8) * per + b / 8, so each XCD walks a
    // contiguous run of tiles (x fastest, then y, then z) and the halo lines
    // that neighbouring tiles share are fetched into its own L2 once
    const int gx = (nx + ETX - 1) / ETX, gy = (vr + ETY - 1) / ETY, ntile = gx * gy * (nz / EKZ);
    const int per = (ntile + 7) / 8;
    const int tile = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
    if (tile >= ntile) return;   // whole block: before any barrier
    const int bx = tile % gx, by = (tile / gx) % gy, bz = tile / (gx * gy);
    const int tx = threadIdx.x % ETX, ty = threadIdx.x / ETX;
    const int i0 = bx * ETX, j0 = by * ETY, k0 = bz * EKZ;
    const int k1 = k0 + EKZ;
    const int i = i0 + tx, j = j0 + ty;

    // staging of one plane: this thread's EPER (field, tile point) values
    double stg[EPER];
#define ETILE_FETCH(kk_)                                                                       \
    do {                                                                                       \
        const int kq = (kk_);                                                                  \
        const int kw = kq < 0 ? kq + nz : (kq >= nz ? kq - nz : kq);                           \
        _Pragma("unroll") for (int e = 0; e < EPER; ++e) {                                     \
            const int idx = threadIdx.x + e * ENT;                                             \
            double val = 0.0;                                                                  \
            if (idx < 4 * EPL) {                                                               \
                const int f = idx / EPL, r = idx - f * EPL;                                    \
                const int hy = r / EHX, hx = r - hy * EHX;                                     \
                int gi = i0 - 1 + hx;                                                          \
                gi = gi < 0 ? gi + nx : (gi >= nx ? gi - nx : gi);                             \
                int gj = j0 - 1 + hy;                                                          \
                const int rows = f == 1 ? vr : ny;                                             \
                if (g.py) gj = gj < 0 ? gj + ny : (gj >= ny ? gj - ny : gj);                   \
                if (gj >= 0 && gj < rows && gi < nx) {                                         \
                    const double *src = f == 0 ? u : (f == 1 ? v : (f == 2 ? w : p));          \
                    val = src[((size_t)kw * rows + gj) * nx + gi];                             \
                }                                                                              \
            }                                                                                  \
            stg[e] = val;                                                                      \
        }                                                                                      \
    } while (0)
#define ETILE_PUT(kk_)                                                                         \
    do {                                                                                       \
        double *dst = sm[((kk_) - k0 + 1) % 3];                                                \
        _Pragma("unroll") for (int e = 0; e < EPER; ++e) {                                     \
            const int idx = threadIdx.x + e * ENT;                                             \
            if (idx < 4 * EPL) dst[idx] = stg[e];                                              \
        }                                                                                      \
    } while (0)

    const double ihx = 1.0 / g.hx, ihz = 1.0 / g.hz;
    const double vis = cf.ab / cf.re;
    const bool zprev = cf.zet != 0.0;

    // a thread keeps its (i, j) through the march: the y metric of its row
    // as reciprocals, once (cell rows: 1/Delta_j, 1/delta_j, 1/delta_{j+1},
    // and 2/Delta_j for the mirror-ghost flux; face rows: 1/delta_j and
    // 1/Delta of the cells above and below)
    const bool crow = i < nx && j < ny;
    const double iD = crow ? 1.0 / g.dyc[j] : 0.0;
    const double i2D = 2.0 * iD;
    const double idn = crow && (g.py || j + 1 < ny) ? 1.0 / g.dyf[j + 1] : 0.0;
    const double ids = crow && (g.py || j > 0) ? 1.0 / g.dyf[j] : 0.0;
    const bool frow = i < nx && j < vr && (g.py || (j > 0 && j < ny));
    const int jm = j > 0 ? j - 1 : ny - 1;   // the cell below a face (wraps when periodic)
    const double ifd = frow ? 1.0 / g.dyf[j] : 0.0;
    const double ifa = frow ? 1.0 / g.dyc[j] : 0.0;
    const double ifb = frow ? 1.0 / g.dyc[jm] : 0.0;

    // rows outside a field (beyond a wall) are staged as zero; the formulas
    // below never use them
    ETILE_FETCH(k0 - 1);
    ETILE_PUT(k0 - 1);
    ETILE_FETCH(k0);
    ETILE_PUT(k0);
    ETILE_FETCH(k0 + 1);
    for (int k = k0; k < k1; ++k) {
        ETILE_PUT(k + 1);   // into the slot of plane k-2
        __syncthreads();
        if (k + 2 <= k1) ETILE_FETCH(k + 2);
        // field f at plane k + dk, row j + dj, column i + di (tile offsets)
        auto L = [&](int f, int dk, int dj, int di) {
            return sm[(k - k0 + 1 + dk) % 3][f * EPL + (ty + 1 + dj) * EHX + (tx + 1 + di)];
        };
        // v with its wall faces read as zero (their stored values are ignored)
        auto V = [&](int dk, int dj, int di) {
            const int jj = j + dj;
            if (!g.py && (jj <= 0 || jj >= ny)) return 0.0;
            return L(1, dk, dj, di);
        };
        if (crow) {
            const size_t o = ((size_t)k * ny + j) * nx + i;
            const bool hn = g.py || j + 1 < ny;   // a cell row above (else the wall)
            const bool hs = g.py || j > 0;        // a cell row below
            // y part of the Laplacian of a cell-height field at row j
            // (mirror ghost at a wall; fluxes over delta, delta_0 = delta_ny
            // across the periodic wrap)
            auto lapy = [&](int f) {
                const double fc = L(f, 0, 0, 0);
                const double fu = hn ? (L(f, 0, 1, 0) - fc) * idn : -fc * i2D;
                const double fl = hs ? (fc - L(f, 0, -1, 0)) * ids : fc * i2D;
                return (fu - fl) * iD;
            };
            // ---- u at x-face (i, j, k)
            {
                const double uc = L(0, 0, 0, 0);
                const double lap = (L(0, 0, 0, 1) - 2.0 * uc + L(0, 0, 0, -1)) * ihx * ihx +
                                   (L(0, 1, 0, 0) - 2.0 * uc + L(0, -1, 0, 0)) * ihz * ihz + lapy(0);
                const double gp = (L(3, 0, 0, 0) - L(3, 0, 0, -1)) * ihx;
                const double c1 = 0.5 * (uc + L(0, 0, 0, 1)), c0 = 0.5 * (L(0, 0, 0, -1) + uc);
                const double dxx = (c1 * c1 - c0 * c0) * ihx;
                // y fluxes v u on the faces j (below) and j+1 (above) at x-face i
                const double fb = hs ? 0.5 * (V(0, 0, 0) + V(0, 0, -1)) * 0.5 * (L(0, 0, -1, 0) + uc) : 0.0;
                const double ft = hn ? 0.5 * (V(0, 1, 0) + V(0, 1, -1)) * 0.5 * (uc + L(0, 0, 1, 0)) : 0.0;
                const double dyy = (ft - fb) * iD;
                const double zb = 0.5 * (L(2, 0, 0, 0) + L(2, 0, 0, -1)) * 0.5 * (L(0, -1, 0, 0) + uc);
                const double zt = 0.5 * (L(2, 1, 0, 0) + L(2, 1, 0, -1)) * 0.5 * (uc + L(0, 1, 0, 0));
                const double N = dxx + dyy + (zt - zb) * ihz;
                double e = uc + cf.dt * (vis * lap - cf.ab * gp - cf.gam * N);
                if (zprev) e -= cf.dt * cf.zet * nu_prev[o];
                if (keep_ue) ue[o] = e;
                ru[o] = e - cf.c * lap;
                nu_out[o] = N;
            }
            // ---- w at z-face (i, j, k): the x <-> z mirror of u
            {
                const double wc = L(2, 0, 0, 0);
                const double lap = (L(2, 0, 0, 1) - 2.0 * wc + L(2, 0, 0, -1)) * ihx * ihx +
                                   (L(2, 1, 0, 0) - 2.0 * wc + L(2, -1, 0, 0)) * ihz * ihz + lapy(2);
                const double gp = (L(3, 0, 0, 0) - L(3, -1, 0, 0)) * ihz;
                const double c1 = 0.5 * (wc + L(2, 1, 0, 0)), c0 = 0.5 * (L(2, -1, 0, 0) + wc);
                const double dzz = (c1 * c1 - c0 * c0) * ihz;
                const double fb = hs ? 0.5 * (V(0, 0, 0) + V(-1, 0, 0)) * 0.5 * (L(2, 0, -1, 0) + wc) : 0.0;
                const double ft = hn ? 0.5 * (V(0, 1, 0) + V(-1, 1, 0)) * 0.5 * (wc + L(2, 0, 1, 0)) : 0.0;
                const double dyy = (ft - fb) * iD;
                const double xb = 0.5 * (L(0, 0, 0, 0) + L(0, -1, 0, 0)) * 0.5 * (L(2, 0, 0, -1) + wc);
                const double xt = 0.5 * (L(0, 0, 0, 1) + L(0, -1, 0, 1)) * 0.5 * (wc + L(2, 0, 0, 1));
                const double N = (xt - xb) * ihx + dyy + dzz;
                double e = wc + cf.dt * (vis * lap - cf.ab * gp - cf.gam * N);
                if (zprev) e -= cf.dt * cf.zet * nw_prev[o];
                if (keep_ue) we[o] = e;
                rw[o] = e - cf.c * lap;
                nw_out[o] = N;
            }
        }
        // ---- v at y-face (i, j, k)
        if (i < nx && j < vr) {
            const size_t o = ((size_t)k * vr + j) * nx + i;
            if (!g.py && (j == 0 || j == ny)) {   // wall faces
                if (keep_ue) ve[o] = 0.0;
                rv[o] = 0.0;
                nv_out[o] = 0.0;
            } else {
                const double vc = V(0, 0, 0);
                const double lapy = ((V(0, 1, 0) - vc) * ifa - (vc - V(0, -1, 0)) * ifb) * ifd;
                const double lap = (V(0, 0, 1) - 2.0 * vc + V(0, 0, -1)) * ihx * ihx +
                                   (V(1, 0, 0) - 2.0 * vc + V(-1, 0, 0)) * ihz * ihz + lapy;
                const double gp = (L(3, 0, 0, 0) - L(3, 0, -1, 0)) * ifd;
                const double c1 = 0.5 * (vc + V(0, 1, 0)), c0 = 0.5 * (V(0, -1, 0) + vc);
                const double dyy = (c1 * c1 - c0 * c0) * ifd;
                // x fluxes u v on the x-faces i and i+1 at y-face j
                const double xb = 0.5 * (L(0, 0, -1, 0) + L(0, 0, 0, 0)) * 0.5 * (vc + V(0, 0, -1));
                const double xt = 0.5 * (L(0, 0, -1, 1) + L(0, 0, 0, 1)) * 0.5 * (V(0, 0, 1) + vc);
                const double zb = 0.5 * (L(2, 0, -1, 0) + L(2, 0, 0, 0)) * 0.5 * (vc + V(-1, 0, 0));
                const double zt = 0.5 * (L(2, 1, -1, 0) + L(2, 1, 0, 0)) * 0.5 * (V(1, 0, 0) + vc);
                const double N = (xt - xb) * ihx + dyy + (zt - zb) * ihz;
                double e = vc + cf.dt * (vis * lap - cf.ab * gp - cf.gam * N);
                if (zprev) e -= cf.dt * cf.zet * nv_prev[o];
                if (keep_ue) ve[o] = e;
                rv[o] = e - cf.c * lap;
                nv_out[o] = N;
            }
        }
        __syncthreads();   // the slot of plane k-1 is refilled next
    }
#undef ETILE_FETCH
#undef ETILE_PUT
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
    const int vr = p.py ? p.ny : p.ny + 1;
    const int ntile = ((p.nx + ETX - 1) / ETX) * ((vr + ETY - 1) / ETY) * (p.nz / EKZ);
    dim3 grid(8 * ((ntile + 7) / 8));   // a whole number of blocks per XCD
    hipLaunchKernelGGL(explicit_kernel, grid, dim3(ENT), 0, st, g, cf, s.u, s.v, s.w, s.p, s.nu, s.nv, s.nw,
                       s.ue, s.ve, s.we, s.ru, s.rv, s.rw, s.nu, s.nv, s.nw, s.nmarkers > 0 ? 1 : 0);
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
