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
    const double *dyf;        // delta_j [ny+1]
};

static Geo geo_of(const Plan &p)
{
    Geo g;
    g.nx = p.nx; g.ny = p.ny; g.nz = p.nz;
    g.ihx = 1.0 / p.hx; g.ihz = 1.0 / p.hz;
    g.dyc = blob_ptr(p, p.lay.dyc);
    g.dyf = blob_ptr(p, p.lay.dyf);
    return g;
}

// b = scale * ((u_{i+1}-u_i)/hx + (v_{j+1}-v_j)/Delta_j + (w_{k+1}-w_k)/hz)
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
    const size_t vc = ((size_t)k * (g.ny + 1) + j) * g.nx + i;
    const double du = (u[c - i + ip] - u[c]) * g.ihx;
    const double dv = (v[vc + g.nx] - v[vc]) / g.dyc[j];
    const double dw = (w[kp * plane + (size_t)j * g.nx + i] - w[c]) * g.ihz;
    b[c] = scale * (du + dv + dw);
}

// u -= g dphi/dx, v -= g dphi/dy (walls: 0), w -= g dphi/dz;
// p += phi - cp * lap (optional).  Grid rows j = 0..ny (v has ny+1 rows).
__global__ __launch_bounds__(256) void correct_kernel(Geo g, const double *__restrict__ phi,
                                                      double *__restrict__ u, double *__restrict__ v,
                                                      double *__restrict__ w, double gs,
                                                      double *__restrict__ pr,
                                                      const double *__restrict__ lap, double cp)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y, k = blockIdx.z;
    if (i >= g.nx) return;
    const size_t plane = (size_t)g.ny * g.nx;
    const size_t vc = ((size_t)k * (g.ny + 1) + j) * g.nx + i;
    if (j < g.ny) {
        const size_t c = (size_t)k * plane + (size_t)j * g.nx + i;
        const int im = (i == 0) ? g.nx - 1 : i - 1;
        const size_t km = (k == 0) ? (size_t)(g.nz - 1) : (size_t)(k - 1);
        const double ph = phi[c];
        u[c] -= gs * (ph - phi[c - i + im]) * g.ihx;
        w[c] -= gs * (ph - phi[km * plane + (size_t)j * g.nx + i]) * g.ihz;
        if (pr) pr[c] += ph - (cp != 0.0 ? cp * lap[c] : 0.0);
        if (j > 0) v[vc] -= gs * (ph - phi[c - g.nx]) / g.dyf[j];
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
    const int rows = (op == IBS_OP_HELMHOLTZ_V) ? g.ny + 1 : g.ny;
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
            const double xe = x[c - i + ip], xw = x[c - i + im];
            const double xt = x[kp * plane + (size_t)j * g.nx + i];
            const double xb = x[km * plane + (size_t)j * g.nx + i];
            double lap = ((xe - xc) - (xc - xw)) * (g.ihx * g.ihx) +
                         ((xt - xc) - (xc - xb)) * (g.ihz * g.ihz);
            bool unknown = true;
            if (op != IBS_OP_HELMHOLTZ_V) {
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
    dim3 grid((p.nx + blk.x - 1) / blk.x, p.ny + 1, p.nz);
    hipLaunchKernelGGL(correct_kernel, grid, blk, 0, s, g, phi, u, v, w, gs, pr, lap, cp);
    return hipGetLastError();
}

hipError_t launch_residual(const Plan &p, int op, double c, const double *x, const double *b,
                           double *r, double *norms2, hipStream_t s)
{
    Geo g = geo_of(p);
    const int rows = (op == IBS_OP_HELMHOLTZ_V) ? p.ny + 1 : p.ny;
    const int nrow = rows * p.nz;
    const int cap = (int)(p.lay.red_count / 2);
    const int nblk = nrow < cap ? nrow : cap;
    double *red = norms2 ? blob_mut(p, p.lay.red) : nullptr;
    hipLaunchKernelGGL(residual_kernel, dim3(nblk), dim3(256), 0, s, g, op, c, x, b, r, red);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !norms2) return e;
    hipLaunchKernelGGL(reduce_pairs_kernel, dim3(1), dim3(256), 0, s, red, nblk, norms2);
    return hipGetLastError();
}

}  // namespace ibs
