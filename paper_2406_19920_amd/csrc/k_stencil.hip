// Stencil kernels on the staggered grid (Section 2.1; kernels E2 and E3 of
// Section 2.3.2) and the FP64 residual of the 7-point operators.
//
// One thread per grid point, x fastest across the lanes (coalesced rows);
// neighbours in y and z come through L2.  No ghost cells are stored: the
// periodic wrap in x and z and the wall conditions in y are applied inline.
#include "ibs_internal.h"

namespace ibs {

struct Geo {
    int nx, ny, nz;
    double ihx, ihz;          // 1/hx, 1/hz
    const double *dyc;        // Delta_j [ny]
    const double *dyf;        // delta_j [ny+1] (periodic y: delta_0 = delta_ny across the wrap)
    int py;                   // periodic y: no walls, v has ny faces
    int wx;                   // walls in x: u slot 0 is the wall face x = 0
                              // (zero), face nx is not stored (zero)
    int wz;                   // walls in z: the same for w's plane 0
    const double *sgx, *sgz;  // stretched wall-bounded x / z: per-index geometry
                              // (StretchSlot arrays of nx / nz), else null
};

// x / z kind of the 3-point rows of operator op (the pressure's, the
// mirror-ghost velocity components', the face-normal component's)
static __device__ __forceinline__ int x_kind(int op)
{
    return op == IBS_OP_POISSON ? XK_P : (op == IBS_OP_HELMHOLTZ_U ? XK_F : XK_C);
}
static __device__ __forceinline__ int z_kind(int op)
{
    return op == IBS_OP_POISSON ? XK_P : (op == IBS_OP_HELMHOLTZ_W ? XK_F : XK_C);
}

static Geo geo_of(const Plan &p)
{
    Geo g;
    g.nx = p.nx; g.ny = p.ny; g.nz = p.nz;
    g.py = p.py ? 1 : 0;
    g.wx = p.wx ? 1 : 0;
    g.wz = p.wz ? 1 : 0;
    g.ihx = 1.0 / p.hx; g.ihz = 1.0 / p.hz;
    g.dyc = blob_ptr(p, p.lay.dyc);
    g.dyf = blob_ptr(p, p.lay.dyf);
    g.sgx = p.sx ? blob_ptr(p, p.lay.sgx) : nullptr;
    g.sgz = p.sz ? blob_ptr(p, p.lay.sgz) : nullptr;
    return g;
}

// XCD-aware order of the row blocks: the hardware deals consecutive blocks
// to the 8 XCDs in turn, so block b takes tile (b % 8) * per + b / 8 (per =
// ceil(ntiles / 8)), and each XCD walks a contiguous run of rows, x blocks
// fastest, then y, then z: the neighbouring rows and planes a stencil reads
// were mostly fetched into that XCD's own L2 by the blocks just before.
// Returns false for the padding blocks of the last XCD's run.  Used by the
// correction (2 % faster in same-box runs, HBM traffic 1.14x -> 1.00x of
// algorithmic); the divergence keeps the hardware's round-robin order, in
// which it measured 4 % faster although it fetches 1.25x.
static __device__ __forceinline__ bool xcd_tile(int gx, int rows, int nz, int &bx, int &j, int &k)
{
    const int ntiles = gx * rows * nz, per = (ntiles + 7) / 8;
    const int t = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
    if (t >= ntiles) return false;
    bx = t % gx;
    const int r = t / gx;
    j = r % rows;
    k = r / rows;
    return true;
}

// b = scale * ((u_{i+1}-u_i)/hx + (v_{j+1}-v_j)/Delta_j + (w_{k+1}-w_k)/hz)
// (a stretched x or z: over the cell's own width Delta_i, Delta_k)
__global__ __launch_bounds__(256) void divergence_kernel(Geo g, const double *__restrict__ u,
                                                         const double *__restrict__ v,
                                                         const double *__restrict__ w,
                                                         double *__restrict__ b, double scale)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y, k = blockIdx.z;
    if (i >= g.nx) return;
    const size_t plane = (size_t)g.ny * g.nx;
    const size_t c = (size_t)k * plane + (size_t)j * g.nx + i;
    const int ip = (i + 1 == g.nx) ? 0 : i + 1;
    const size_t kp = (k + 1 == g.nz) ? 0 : (size_t)(k + 1);
    const size_t vc = ((size_t)k * (g.ny + 1 - g.py) + j) * g.nx + i;
    // the face above cell j: j + 1, or face 0 at the top when y is periodic
    const size_t vn = (g.py && j + 1 == g.ny) ? vc - (size_t)j * g.nx : vc + g.nx;
    // with walls in x the wall faces x = 0 and x = lx carry u = 0
    const double ue = (g.wx && ip == 0) ? 0.0 : u[c - i + ip];
    const double uw = (g.wx && i == 0) ? 0.0 : u[c];
    const double du = (ue - uw) * (g.sgx ? g.sgx[SG_RC * g.nx + i] : g.ihx);
    const double dv = (v[vn] - v[vc]) / g.dyc[j];
    const double wt = (g.wz && kp == 0) ? 0.0 : w[kp * plane + (size_t)j * g.nx + i];
    const double wb = (g.wz && k == 0) ? 0.0 : w[c];
    const double dw = (wt - wb) * (g.sgz ? g.sgz[(size_t)SG_RC * g.nz + k] : g.ihz);
    b[c] = scale * (du + dv + dw);
}

// u -= g dphi/dx, v -= g dphi/dy (walls: 0), w -= g dphi/dz (differences
// over the centre distances: hx, hz, or delta_i, delta_k when stretched);
// p += phi - cp * lap (optional).  Grid rows j = 0..ny (v has ny+1 rows).
__global__ __launch_bounds__(256) void correct_kernel(Geo g, const double *__restrict__ phi,
                                                      double *__restrict__ u, double *__restrict__ v,
                                                      double *__restrict__ w, double gs,
                                                      double *__restrict__ pr,
                                                      const double *__restrict__ lap, double cp)
{
    int bx, j, k;
    if (!xcd_tile((g.nx + blockDim.x - 1) / blockDim.x, g.ny + 1 - g.py, g.nz, bx, j, k)) return;
    const int i = bx * blockDim.x + threadIdx.x;
    if (i >= g.nx) return;
    const size_t plane = (size_t)g.ny * g.nx;
    const size_t vc = ((size_t)k * (g.ny + 1 - g.py) + j) * g.nx + i;
    if (j < g.ny) {
        const size_t c = (size_t)k * plane + (size_t)j * g.nx + i;
        const int im = (i == 0) ? g.nx - 1 : i - 1;
        const size_t km = (k == 0) ? (size_t)(g.nz - 1) : (size_t)(k - 1);
        const double ph = phi[c];
        if (g.wx && i == 0) u[c] = 0.0;   // the wall face x = 0
        else u[c] -= gs * (ph - phi[c - i + im]) * (g.sgx ? g.sgx[SG_RF * g.nx + i] : g.ihx);
        if (g.wz && k == 0) w[c] = 0.0;   // the wall face z = 0
        else w[c] -= gs * (ph - phi[km * plane + (size_t)j * g.nx + i]) *
                     (g.sgz ? g.sgz[(size_t)SG_RF * g.nz + k] : g.ihz);
        if (pr) pr[c] += ph - (cp != 0.0 ? cp * lap[c] : 0.0);
        if (j > 0) v[vc] -= gs * (ph - phi[c - g.nx]) / g.dyf[j];
        else if (g.py) v[vc] -= gs * (ph - phi[c + (size_t)(g.ny - 1) * g.nx]) / g.dyf[0];   // across the wrap
        else v[vc] = 0.0;
    } else {
        v[vc] = 0.0;
    }
}

// Deterministic block sum: wave butterflies, then the waves in order.
static __device__ __forceinline__ double block_sum(double v, double *sm)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0) sm[w] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int q = 0; q < (int)(blockDim.x >> 6); ++q) t += sm[q];
    return t;
}

// Residual r = b - A x for op 0 (A = L_p) or ops 1..3 (A = I - c L).  Each
// block walks a fixed set of grid rows; its partial sums of r^2 and b^2 go
// to red[2*block], summed later by one block in a fixed order.
__global__ __launch_bounds__(256) void residual_kernel(Geo g, int op, double cc,
                                                       const double *__restrict__ x,
                                                       const double *__restrict__ b,
                                                       double *__restrict__ r,
                                                       double *__restrict__ red)
{
    __shared__ double sm[8];
    const int rows = (op == IBS_OP_HELMHOLTZ_V && !g.py) ? g.ny + 1 : g.ny;
    const size_t plane = (size_t)rows * g.nx;
    const int nrow = rows * g.nz;
    double rr = 0.0, bb = 0.0;
    // rows (j, k) in a fixed block-cyclic order: the partial sums depend on
    // the problem size only, never on timing
    for (int rw = blockIdx.x; rw < nrow; rw += gridDim.x) {
        const int j = rw % rows, k = rw / rows;
        for (int i = threadIdx.x; i < g.nx; i += blockDim.x) {
            const size_t c = (size_t)k * plane + (size_t)j * g.nx + i;
            const int ip = (i + 1 == g.nx) ? 0 : i + 1, im = (i == 0) ? g.nx - 1 : i - 1;
            const size_t kp = (k + 1 == g.nz) ? 0 : (size_t)(k + 1);
            const size_t km = (k == 0) ? (size_t)(g.nz - 1) : (size_t)(k - 1);
            const double xc = x[c];
            double xe = x[c - i + ip], xw = x[c - i + im];
            bool unknown = true;
            if (g.wx) {
                // walls in x: a missing neighbour is the wall's ghost, xc
                // (pressure, Neumann), -xc (v, w, mirror) or 0 (u: the wall
                // faces; slot 0 is the wall x = 0 itself)
                const double gx = op == IBS_OP_POISSON ? xc : (op == IBS_OP_HELMHOLTZ_U ? 0.0 : -xc);
                if (op == IBS_OP_HELMHOLTZ_U && i == 1) xw = 0.0;
                if (i == 0) xw = gx;
                if (i + 1 == g.nx) xe = gx;
                if (op == IBS_OP_HELMHOLTZ_U && i == 0) unknown = false;
            }
            double xt = x[kp * plane + (size_t)j * g.nx + i];
            double xb = x[km * plane + (size_t)j * g.nx + i];
            if (g.wz) {
                // walls in z: as in x, with w the face-normal component
                const double gz = op == IBS_OP_POISSON ? xc : (op == IBS_OP_HELMHOLTZ_W ? 0.0 : -xc);
                if (op == IBS_OP_HELMHOLTZ_W && k == 1) xb = 0.0;
                if (k == 0) xb = gz;
                if (k + 1 == g.nz) xt = gz;
                if (op == IBS_OP_HELMHOLTZ_W && k == 0) unknown = false;
            }
            double lap;
            if (!g.sgx && !g.sgz) {
                lap = ((xe - xc) - (xc - xw)) * (g.ihx * g.ihx) + ((xt - xc) - (xc - xb)) * (g.ihz * g.ihz);
            } else {
                // a stretched x or z: the flux form over the local widths
                const double lx = g.sgx ? (xe - xc) * g.sgx[(size_t)sg_ae(x_kind(op)) * g.nx + i] -
                                              (xc - xw) * g.sgx[(size_t)sg_aw(x_kind(op)) * g.nx + i]
                                        : ((xe - xc) - (xc - xw)) * (g.ihx * g.ihx);
                const double lz = g.sgz ? (xt - xc) * g.sgz[(size_t)sg_ae(z_kind(op)) * g.nz + k] -
                                              (xc - xb) * g.sgz[(size_t)sg_aw(z_kind(op)) * g.nz + k]
                                        : ((xt - xc) - (xc - xb)) * (g.ihz * g.ihz);
                lap = lx + lz;
            }
            if (g.py) {
                // periodic y: interior formulas everywhere, neighbours wrapping
                const int jn = (j + 1 == g.ny) ? 0 : j + 1, js = (j == 0) ? g.ny - 1 : j - 1;
                const double xn = x[c + (ptrdiff_t)(jn - j) * g.nx], xs = x[c + (ptrdiff_t)(js - j) * g.nx];
                if (op == IBS_OP_HELMHOLTZ_V)
                    lap += ((xn - xc) / g.dyc[j] - (xc - xs) / g.dyc[js]) / g.dyf[j];
                else
                    lap += ((xn - xc) / g.dyf[j + 1] - (xc - xs) / g.dyf[j]) / g.dyc[j];
            } else if (op != IBS_OP_HELMHOLTZ_V) {
                const double D = g.dyc[j];
                double fu, fl;
                if (j + 1 < g.ny) fu = (x[c + g.nx] - xc) / g.dyf[j + 1];
                else fu = (op == IBS_OP_POISSON) ? 0.0 : -2.0 * xc / D;
                if (j > 0) fl = (xc - x[c - g.nx]) / g.dyf[j];
                else fl = (op == IBS_OP_POISSON) ? 0.0 : 2.0 * xc / D;
                lap += (fu - fl) / D;
            } else if (j >= 1 && j <= g.ny - 1) {
                const double vu = (j + 1 <= g.ny - 1) ? x[c + g.nx] : 0.0;
                const double vl = (j - 1 >= 1) ? x[c - g.nx] : 0.0;
                lap += ((vu - xc) / g.dyc[j] - (xc - vl) / g.dyc[j - 1]) / g.dyf[j];
            } else {
                unknown = false;
            }
            if (unknown) {
                const double ax = (op == IBS_OP_POISSON) ? lap : xc - cc * lap;
                const double bc = b[c];
                const double res = bc - ax;
                r[c] = res;
                rr += res * res;
                bb += bc * bc;
            } else {
                r[c] = 0.0;
            }
        }
    }
    if (red) {
        const double s1 = block_sum(rr, sm);
        __syncthreads();
        const double s2 = block_sum(bb, sm);
        if (threadIdx.x == 0) {
            red[2 * blockIdx.x] = s1;
            red[2 * blockIdx.x + 1] = s2;
        }
    }
}

// Second stage: one block sums the per-block partials in a fixed order.
__global__ __launch_bounds__(256) void reduce_pairs_kernel(const double *__restrict__ red, int nslots,
                                                           double *__restrict__ out)
{
    __shared__ double sm[8];
    double a = 0.0, b = 0.0;
    for (int s = threadIdx.x; s < nslots; s += blockDim.x) {
        a += red[2 * s];
        b += red[2 * s + 1];
    }
    const double ta = block_sum(a, sm);
    __syncthreads();
    const double tb = block_sum(b, sm);
    if (threadIdx.x == 0) {
        out[0] = ta;
        out[1] = tb;
    }
}

static dim3 row_block(int nx) { return dim3(nx >= 256 ? 256 : ((nx + 63) / 64) * 64); }
// one-dimensional grid of xcd_tile's order: a whole number of blocks per XCD
static dim3 xcd_grid(int nx, dim3 blk, int rows, int nz)
{
    const int ntiles = (int)((nx + blk.x - 1) / blk.x) * rows * nz;
    return dim3(8 * ((ntiles + 7) / 8));
}

hipError_t launch_divergence(const Plan &p, const double *u, const double *v, const double *w,
                             double *b, double scale, hipStream_t s)
{
    Geo g = geo_of(p);
    dim3 blk = row_block(p.nx);
    dim3 grid((p.nx + blk.x - 1) / blk.x, p.ny, p.nz);
    hipLaunchKernelGGL(divergence_kernel, grid, blk, 0, s, g, u, v, w, b, scale);
    return hipGetLastError();
}

hipError_t launch_correct(const Plan &p, const double *phi, double *u, double *v, double *w,
                          double gs, double *pr, const double *lap, double cp, hipStream_t s)
{
    Geo g = geo_of(p);
    dim3 blk = row_block(p.nx);
    dim3 grid = xcd_grid(p.nx, blk, p.py ? p.ny : p.ny + 1, p.nz);   // the v face rows
    hipLaunchKernelGGL(correct_kernel, grid, blk, 0, s, g, phi, u, v, w, gs, pr, lap, cp);
    return hipGetLastError();
}

// Inhomogeneous wall data (Appendix B's boundary terms, the pencil
// right-hand sides BC2.2 forms): the operator with data is the homogeneous
// one plus a term in the rows next to the walls, so the data move to the
// right-hand side there before the transforms (transforming the data planes
// and correcting the pencils, as the paper does, gives the same result by
// linearity).  One thread per wall column (i, k); lo/hi null = zero data.
//   Poisson (data: wall flux dphi/dy): b_0 += lo/Delta_0,
//                                       b_{ny-1} -= hi/Delta_{ny-1}
//   u, w (data: wall value, mirror ghost 2g - f_0):
//       r_0 += 2c lo/Delta_0^2,  r_{ny-1} += 2c hi/Delta_{ny-1}^2
//   v (data: wall-face value): r_1 += c lo/(Delta_0 delta_1),
//       r_{ny-1} += c hi/(Delta_{ny-1} delta_{ny-1})
__global__ __launch_bounds__(256) void wall_data_kernel(Geo g, int op, double c,
                                                        const double *__restrict__ lo,
                                                        const double *__restrict__ hi,
                                                        double *__restrict__ rhs)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int k = blockIdx.y;
    if (i >= g.nx) return;
    const size_t col = (size_t)k * g.nx + i;
    const double gl = lo ? lo[col] : 0.0, gh = hi ? hi[col] : 0.0;
    const int rows = op == IBS_OP_HELMHOLTZ_V ? g.ny + 1 : g.ny;
    double *pl = rhs + ((size_t)k * rows) * g.nx + i;   // row 0 of this column
    const size_t nx = g.nx;
    const double D0 = g.dyc[0], D1 = g.dyc[g.ny - 1];
    if (op == IBS_OP_POISSON) {
        pl[0] += gl / D0;
        pl[(g.ny - 1) * nx] -= gh / D1;
    } else if (op == IBS_OP_HELMHOLTZ_V) {
        pl[nx] += c * gl / (D0 * g.dyf[1]);
        pl[(g.ny - 1) * nx] += c * gh / (D1 * g.dyf[g.ny - 1]);
    } else {
        pl[0] += 2.0 * c * gl / (D0 * D0);
        pl[(g.ny - 1) * nx] += 2.0 * c * gh / (D1 * D1);
    }
}

hipError_t launch_wall_data(const Plan &p, int op, double c, const double *lo, const double *hi,
                            double *rhs, hipStream_t s)
{
    Geo g = geo_of(p);
    dim3 blk = row_block(p.nx);
    dim3 grid((p.nx + blk.x - 1) / blk.x, p.nz);
    hipLaunchKernelGGL(wall_data_kernel, grid, blk, 0, s, g, op, c, lo, hi, rhs);
    return hipGetLastError();
}

hipError_t launch_residual(const Plan &p, int op, double c, const double *x, const double *b,
                           double *r, double *norms2, double *red, hipStream_t s)
{
    Geo g = geo_of(p);
    const int rows = comp_rows(p, op - 1);
    const int nrow = rows * p.nz;
    const int nblk = nrow < RESID_SLOTS ? nrow : RESID_SLOTS;
    if (!norms2) red = nullptr;
    hipLaunchKernelGGL(residual_kernel, dim3(nblk), dim3(256), 0, s, g, op, c, x, b, r, red);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !norms2) return e;
    hipLaunchKernelGGL(reduce_pairs_kernel, dim3(1), dim3(256), 0, s, red, nblk, norms2);
    return hipGetLastError();
}

// Strict compatibility, first stage: block q of job j walks the cell rows
// (j, k) = q, q + G, ... (fixed order) and writes its partial sums of
// W b and W b^2 to part[2 (j * G + q) ..], W = Delta_j (times Delta_i /
// hbar_x and Delta_k / hbar_z on a stretched x or z, whose shares sum to
// nx and nz as the uniform ones do).
__global__ __launch_bounds__(256) void compat_partials_kernel(Geo g, const double *__restrict__ b0,
                                                              const double *__restrict__ b1,
                                                              const double *__restrict__ b2,
                                                              const double *__restrict__ b3,
                                                              double *__restrict__ part)
{
    __shared__ double sm[8];
    const int job = blockIdx.y;
    const double *__restrict__ b = job == 0 ? b0 : job == 1 ? b1 : job == 2 ? b2 : b3;
    const int nrow = g.ny * g.nz;
    double s1 = 0.0, s2 = 0.0;
    for (int rw = blockIdx.x; rw < nrow; rw += gridDim.x) {
        const int j = rw % g.ny, k = rw / g.ny;
        double w = g.dyc[j];
        if (g.sgz) w *= g.sgz[(size_t)SG_WN * g.nz + k];
        const double *row = b + (size_t)rw * g.nx;
        for (int i = threadIdx.x; i < g.nx; i += blockDim.x) {
            const double v = row[i];
            const double wi = g.sgx ? w * g.sgx[SG_WN * g.nx + i] : w;
            s1 += wi * v;
            s2 += wi * v * v;
        }
    }
    const double t1 = block_sum(s1, sm);
    __syncthreads();
    const double t2 = block_sum(s2, sm);
    if (threadIdx.x == 0) {
        const size_t slot = (size_t)job * gridDim.x + blockIdx.x;
        part[2 * slot] = t1;
        part[2 * slot + 1] = t2;
    }
}

// Second stage, one block per job: mean = sum(W b) / sum(W), rms =
// sqrt(sum(W b^2) / sum(W)); the rhs is incompatible when |mean| > 1e-10
// rms (a compatible rhs, such as the divergence of a field with no wall
// flux, has a mean at rounding level, ~1e-16 rms).  The verdict is kept in
// incompat[job] and overrides the status of the job's report.
__global__ __launch_bounds__(256) void compat_final_kernel(Geo g, const double *__restrict__ part,
                                                           int nblk, void *info0, void *info1,
                                                           void *info2, void *info3,
                                                           int *__restrict__ incompat)
{
    __shared__ double sm[8];
    const int job = blockIdx.x;
    double a = 0.0, c = 0.0;
    for (int q = threadIdx.x; q < nblk; q += blockDim.x) {
        a += part[2 * ((size_t)job * nblk + q)];
        c += part[2 * ((size_t)job * nblk + q) + 1];
    }
    const double s1 = block_sum(a, sm);
    __syncthreads();
    const double s2 = block_sum(c, sm);
    if (threadIdx.x == 0) {
        double wsum = 0.0;
        for (int j = 0; j < g.ny; ++j) wsum += g.dyc[j];
        wsum *= (double)g.nx * (double)g.nz;
        const double mean = s1 / wsum;
        const double rms = sqrt(fmax(s2 / wsum, 0.0));
        const bool bad = fabs(mean) > 1e-10 * rms;
        incompat[job] = bad ? 1 : 0;
        void *info = job == 0 ? info0 : job == 1 ? info1 : job == 2 ? info2 : info3;
        if (bad && info) static_cast<ibs_solve_info *>(info)->status = IBS_ERR_INCOMPATIBLE_RHS;
    }
}

int compat_blocks(const Plan &p)
{
    const int nrow = p.ny * p.nz;
    return nrow < COMPAT_SLOTS ? nrow : COMPAT_SLOTS;
}

hipError_t launch_compat_partials(const Plan &p, const double *const *b, int njobs, const State &st,
                                  hipStream_t s)
{
    if (njobs < 1 || njobs > STATE_JOBS || (size_t)njobs * compat_blocks(p) > COMPAT_SLOTS)
        return hipErrorInvalidValue;
    Geo g = geo_of(p);
    const double *bb[4] = {b[0], njobs > 1 ? b[1] : b[0], njobs > 2 ? b[2] : b[0], njobs > 3 ? b[3] : b[0]};
    hipLaunchKernelGGL(compat_partials_kernel, dim3(compat_blocks(p), njobs), dim3(256), 0, s, g, bb[0],
                       bb[1], bb[2], bb[3], st.compat);
    return hipGetLastError();
}

hipError_t launch_compat_final(const Plan &p, void *const *info, int njobs, const State &st, hipStream_t s)
{
    if (njobs < 1 || njobs > STATE_JOBS) return hipErrorInvalidValue;
    Geo g = geo_of(p);
    void *in[4] = {info[0], njobs > 1 ? info[1] : nullptr, njobs > 2 ? info[2] : nullptr,
                   njobs > 3 ? info[3] : nullptr};
    hipLaunchKernelGGL(compat_final_kernel, dim3(njobs), dim3(256), 0, s, g, st.compat, compat_blocks(p),
                       in[0], in[1], in[2], in[3], st.incompat);
    return hipGetLastError();
}

}  // namespace ibs
