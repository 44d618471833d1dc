// Refined (mixed-precision) path: eigen-transforms as split-bfloat16
// matrix-core products with FP32 accumulation, FP32 work arrays, FP64
// residual and FP64 iterate.
//
// Every transform operand v (data and eigenvector entries) is split into
// three bfloat16 terms, v = v0 + v1 + v2 (24 significant bits, the FP32
// significand); a product a*q is formed from the six partial products whose
// order is at most 2^-16 relative (a0q0, a0q1, a1q0, a1q1, a0q2, a2q0), all
// accumulated in FP32 by V_MFMA_F32_16X16X32_BF16.  The transforms are
// therefore accurate to a few FP32 ulps; the accuracy of the solve is won
// back by iterative refinement against the FP64 residual.
//
// Instruction layout (checked on gfx950): lane l holds A[l%16][8(l/16)+e]
// and B[8(l/16)+e][l%16], e = 0..7; result element q is row 4(l/16)+q,
// column l%16.  The eigenvector matrices are pre-split and pre-swizzled on
// the host in exactly that order.
#include "ibs_internal.h"

namespace ibs {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 b8 __attribute__((ext_vector_type(8)));
typedef float fv8 __attribute__((ext_vector_type(8)));
typedef double dv4 __attribute__((ext_vector_type(4)));

static __device__ __forceinline__ f4 mma(b8 a, b8 b, f4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// a*b from three-term splits; small partial products first
static __device__ __forceinline__ f4 mma3(const b8 *a, const b8 *b, f4 c)
{
    c = mma(a[2], b[0], c);
    c = mma(a[0], b[2], c);
    c = mma(a[1], b[1], c);
    c = mma(a[1], b[0], c);
    c = mma(a[0], b[1], c);
    c = mma(a[0], b[0], c);
    return c;
}

static __device__ __forceinline__ void split8(const float *v, b8 *t)
{
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const __bf16 h0 = (__bf16)v[e];
        float r = v[e] - (float)h0;
        const __bf16 h1 = (__bf16)r;
        r -= (float)h1;
        t[0][e] = h0;
        t[1][e] = h1;
        t[2][e] = (__bf16)r;
    }
}

template <typename Tin>
static __device__ __forceinline__ void load8(const Tin *p, float *v);
template <>
__device__ __forceinline__ void load8<float>(const float *p, float *v)
{
    const fv8 x = *reinterpret_cast<const fv8 *>(p);
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = x[e];
}
template <>
__device__ __forceinline__ void load8<double>(const double *p, float *v)
{
    const dv4 x0 = *reinterpret_cast<const dv4 *>(p);
    const dv4 x1 = *reinterpret_cast<const dv4 *>(p + 4);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        v[e] = (float)x0[e];
        v[4 + e] = (float)x1[e];
    }
}

static __device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

// x transform, C = A B with A = rows of the field (M = nz*rows, K = nx),
// B the split swizzled transform (K x N).  MODE 0: FP32 out; MODE 1: FP64
// x = C; MODE 2: FP64 x += C and per-block sums of C^2 and x^2 into red.
// Workgroup: 8 waves laid out wgm x wgn, each owning (16 WM) x (16 WN).
template <int WM, int WN, typename Tin, int MODE>
__global__ __launch_bounds__(512) void split_xgemm_kernel(SplitSet ss, int nz, int K, int N,
                                                          const b8 *__restrict__ qs, int wgn,
                                                          double *__restrict__ red,
                                                          const int *__restrict__ skip)
{
    if (skip && skip[blockIdx.z]) return;   // this job has already converged
    const SplitJob &jb = ss.j[blockIdx.z];
    const int M = nz * jb.rows;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wgm = 8 / wgn;
    const int wm = wave / wgn, wn = wave % wgn;
    const int row0 = (blockIdx.x * wgm + wm) * (16 * WM);
    const int col0 = (blockIdx.y * wgn + wn) * (16 * WN);
    const bool active = row0 < M && col0 < N;
    const int nrb = active ? min(WM, (M - row0) >> 4) : 0;
    const int ncb = active ? min(WN, (N - col0) >> 4) : 0;
    const int li = lane & 15, lg = lane >> 4;
    const int NB = N >> 4;
    f4 acc[WM][WN];
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j) acc[i][j] = (f4){0.f, 0.f, 0.f, 0.f};
    if (active) {
        const Tin *__restrict__ A = static_cast<const Tin *>(jb.in);
        for (int kc = 0; kc < (K >> 5); ++kc) {
            b8 a[WM][3], b[WN][3];
#pragma unroll
            for (int i = 0; i < WM; ++i) {
                float v[8];
                if (i < nrb) {
                    load8<Tin>(A + (size_t)(row0 + 16 * i + li) * K + 32 * kc + 8 * lg, v);
                } else {
#pragma unroll
                    for (int e = 0; e < 8; ++e) v[e] = 0.f;
                }
                split8(v, a[i]);
            }
#pragma unroll
            for (int j = 0; j < WN; ++j) {
                const b8 *q = qs + ((size_t)(kc * NB + (col0 >> 4) + (j < ncb ? j : 0)) * 3) * 64 + lane;
#pragma unroll
                for (int t = 0; t < 3; ++t) b[j][t] = q[t * 64];
            }
#pragma unroll
            for (int i = 0; i < WM; ++i)
#pragma unroll
                for (int j = 0; j < WN; ++j) acc[i][j] = mma3(a[i], b[j], acc[i][j]);
        }
    }
    double sd = 0.0, sx = 0.0;
#pragma unroll
    for (int i = 0; i < WM; ++i) {
#pragma unroll
        for (int j = 0; j < WN; ++j) {
            if (i < nrb && j < ncb) {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const size_t o = (size_t)(row0 + 16 * i + 4 * lg + q) * N + col0 + 16 * j + li;
                    if (MODE == 0) {
                        jb.out[o] = acc[i][j][q];
                    } else if (MODE == 1) {
                        jb.x[o] = (double)acc[i][j][q];
                    } else {
                        const double d = (double)acc[i][j][q];
                        const double xn = jb.x[o] + d;
                        jb.x[o] = xn;
                        sd += d * d;
                        sx += xn * xn;
                    }
                }
            }
        }
    }
    if (MODE == 2) {
        __shared__ double sm[2][8];
        sd = wave_sum(sd);
        sx = wave_sum(sx);
        if (lane == 0) { sm[0][wave] = sd; sm[1][wave] = sx; }
        __syncthreads();
        if (threadIdx.x == 0) {
            double a = 0.0, b = 0.0;
            for (int w = 0; w < 8; ++w) { a += sm[0][w]; b += sm[1][w]; }
            const size_t slot = ((size_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
            red[2 * slot] = a;
            red[2 * slot + 1] = b;
        }
    }
}

// z transform, C = A B with A the split swizzled transform (M x K, M = K =
// nz) and B the field viewed as K x (rows*nx), FP32 in and out.
template <int WM, int WN>
__global__ __launch_bounds__(512) void split_zgemm_kernel(SplitSet ss, int M, int K, int nx,
                                                          const b8 *__restrict__ qs, int wgn,
                                                          const int *__restrict__ skip)
{
    if (skip && skip[blockIdx.z]) return;
    const SplitJob &jb = ss.j[blockIdx.z];
    const int Ncol = jb.rows * nx;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wgm = 8 / wgn;
    const int wm = wave / wgn, wn = wave % wgn;
    const int row0 = (blockIdx.y * wgm + wm) * (16 * WM);
    const int col0 = (blockIdx.x * wgn + wn) * (16 * WN);
    if (row0 >= M || col0 >= Ncol) return;
    const int nrb = min(WM, (M - row0) >> 4);
    const int ncb = min(WN, (Ncol - col0) >> 4);
    const int li = lane & 15, lg = lane >> 4;
    const int MB = M >> 4;
    const float *__restrict__ B = static_cast<const float *>(jb.in);
    f4 acc[WM][WN];
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j) acc[i][j] = (f4){0.f, 0.f, 0.f, 0.f};
    for (int kc = 0; kc < (K >> 5); ++kc) {
        b8 a[WM][3], b[WN][3];
#pragma unroll
        for (int i = 0; i < WM; ++i) {
            const b8 *q = qs + ((size_t)(kc * MB + (row0 >> 4) + (i < nrb ? i : 0)) * 3) * 64 + lane;
#pragma unroll
            for (int t = 0; t < 3; ++t) a[i][t] = q[t * 64];
        }
        const float *brow = B + (size_t)(32 * kc + 8 * lg) * Ncol + col0 + li;
#pragma unroll
        for (int j = 0; j < WN; ++j) {
            float v[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) v[e] = (j < ncb) ? brow[(size_t)e * Ncol + 16 * j] : 0.f;
            split8(v, b[j]);
        }
#pragma unroll
        for (int i = 0; i < WM; ++i)
#pragma unroll
            for (int j = 0; j < WN; ++j) acc[i][j] = mma3(a[i], b[j], acc[i][j]);
    }
#pragma unroll
    for (int i = 0; i < WM; ++i) {
        if (i >= nrb) break;
#pragma unroll
        for (int j = 0; j < WN; ++j) {
            if (j >= ncb) break;
#pragma unroll
            for (int q = 0; q < 4; ++q)
                jb.out[(size_t)(row0 + 16 * i + 4 * lg + q) * Ncol + col0 + 16 * j + li] = acc[i][j][q];
        }
    }
}

// FP32 residual r = b - A x of the FP64 iterate (7-point stencils of
// Section 2.1).  For the pressure problem the weighted mean of b (recorded
// by the first pass) is subtracted first: that constant lies in the null
// space of every correction, and left in r its FP32 rounding would swamp the
// shrinking residual.  The same pass sums Delta_j x per block (fixed block
// count and order), so the next correction can also remove the weighted
// mean that x has picked up from the FP32 transforms.
// grid: (XSUM_SLOTS blocks, jobs); each block walks grid rows (j, k).
__global__ __launch_bounds__(256) void residual_f32_kernel(SplitSet ss, int nx, int ny, int nz,
                                                           double ihx2, double ihz2,
                                                           const double *__restrict__ dyc,
                                                           const double *__restrict__ dyf,
                                                           const double *__restrict__ bmean,
                                                           double *__restrict__ xsum,
                                                           const int *__restrict__ skip)
{
    const int job = blockIdx.y;
    if (skip && skip[job]) return;
    const SplitJob &jb = ss.j[job];
    const int op = jb.op, rows = jb.rows;
    const size_t plane = (size_t)rows * nx;
    const double *__restrict__ x = jb.x;
    const double bm = (op == IBS_OP_POISSON) ? bmean[job] : 0.0;
    double wx = 0.0;
    for (int rw = blockIdx.x; rw < rows * nz; rw += gridDim.x) {
        const int j = rw % rows, k = rw / rows;
        const size_t kp = (k + 1 == nz) ? 0 : (size_t)(k + 1);
        const size_t km = (k == 0) ? (size_t)(nz - 1) : (size_t)(k - 1);
        for (int i = threadIdx.x; i < nx; i += blockDim.x) {
            const size_t c = (size_t)k * plane + (size_t)j * nx + i;
            if (op == IBS_OP_HELMHOLTZ_V && (j == 0 || j == ny)) {
                jb.r[c] = 0.f;
                continue;
            }
            const int ip = (i + 1 == nx) ? 0 : i + 1, im = (i == 0) ? nx - 1 : i - 1;
            const double xc = x[c];
            double lap = ((x[c - i + ip] - xc) - (xc - x[c - i + im])) * ihx2 +
                         ((x[kp * plane + (size_t)j * nx + i] - xc) - (xc - x[km * plane + (size_t)j * nx + i])) * ihz2;
            if (op != IBS_OP_HELMHOLTZ_V) {
                const double D = dyc[j];
                double fu, fl;
                if (j + 1 < ny) fu = (x[c + nx] - xc) / dyf[j + 1];
                else fu = (op == IBS_OP_POISSON) ? 0.0 : -2.0 * xc / D;
                if (j > 0) fl = (xc - x[c - nx]) / dyf[j];
                else fl = (op == IBS_OP_POISSON) ? 0.0 : 2.0 * xc / D;
                lap += (fu - fl) / D;
                wx += D * xc;
            } else {
                const double vu = (j + 1 <= ny - 1) ? x[c + nx] : 0.0;
                const double vl = (j - 1 >= 1) ? x[c - nx] : 0.0;
                lap += ((vu - xc) / dyc[j] - (xc - vl) / dyc[j - 1]) / dyf[j];
            }
            const double ax = (op == IBS_OP_POISSON) ? lap : xc - jb.c * lap;
            jb.r[c] = (float)((jb.b[c] - bm) - ax);
        }
    }
    __shared__ double sm[4];
    wx = wave_sum(wx);
    if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = wx;
    __syncthreads();
    if (threadIdx.x == 0)
        xsum[(size_t)job * XSUM_SLOTS + blockIdx.x] = sm[0] + sm[1] + sm[2] + sm[3];
}

// After refinement pass p >= 1, one block per job sums the update partials of
// pass p (and of pass p-1 when p >= 2) in a fixed order.  rel_correction =
// ||d_p|| / ||x||; the error of the iterate is predicted as rel_correction
// times the last observed contraction ||d_p|| / ||d_{p-1}|| (d_0 = the
// first-pass solution, so the ratio is 1 at p = 1).  The report is written
// and the job's stop flag set when the prediction meets tol; the kernels of
// later passes then return at once, so the sequence of launches is fixed
// (graph-capturable) while the work adapts.  Without convergence by the last
// pass the status stays NOT_CONVERGED.
static __device__ double2 sum_pairs(const double *r, int n)
{
    __shared__ double sm[2][4];
    double a = 0.0, b = 0.0;
    for (int s = threadIdx.x; s < n; s += blockDim.x) {
        a += r[2 * s];
        b += r[2 * s + 1];
    }
    a = wave_sum(a);
    b = wave_sum(b);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0) { sm[0][w] = a; sm[1][w] = b; }
    __syncthreads();
    double2 t = make_double2(0.0, 0.0);
    for (int q = 0; q < 4; ++q) { t.x += sm[0][q]; t.y += sm[1][q]; }
    return t;
}

__global__ __launch_bounds__(256) void refine_check_kernel(SplitSet ss, const double *__restrict__ red_last,
                                                           const double *__restrict__ red_prev,
                                                           int slots_per_job, int pass, double tol,
                                                           int *__restrict__ done)
{
    const int job = blockIdx.x;
    if (pass >= 2 && done[job]) return;     // stopped earlier: report stands
    const SplitJob &jb = ss.j[job];
    const size_t off = (size_t)job * slots_per_job * 2;
    const double2 last = sum_pairs(red_last + off, slots_per_job);
    double rprev = 1.0;
    if (red_prev) {
        const double2 prev = sum_pairs(red_prev + off, slots_per_job);
        rprev = prev.y > 0.0 ? sqrt(prev.x / prev.y) : 0.0;
    }
    if (threadIdx.x == 0) {
        const double rc = last.y > 0.0 ? sqrt(last.x / last.y) : 0.0;
        const double ratio = rprev > 0.0 ? fmin(1.0, rc / rprev) : 1.0;
        const double predicted = rc * ratio;
        const bool ok = predicted <= tol;
        done[job] = ok ? 1 : 0;
        if (jb.info) {
            ibs_solve_info *inf = static_cast<ibs_solve_info *>(jb.info);
            const int base = inf->status == IBS_ERR_NOT_CONVERGED ? IBS_OK : inf->status;
            inf->iters = pass + 1;
            inf->rel_correction = rc;
            inf->rel_residual = predicted;
            inf->status = (base == IBS_OK && !ok) ? IBS_ERR_NOT_CONVERGED : base;
        }
    }
}

static int max_rows(const SplitSet &ss)
{
    int r = 0;
    for (int q = 0; q < ss.n; ++q) r = ss.j[q].rows > r ? ss.j[q].rows : r;
    return r;
}

static void xgemm_grid(const SplitSet &ss, const Plan &p, int &wgn, dim3 &grid)
{
    constexpr int WM = 4, WN = 4;
    const int N = p.nx, M = p.nz * max_rows(ss);
    const int ncolw = N / (16 * WN);
    wgn = ncolw >= 4 ? 4 : (ncolw >= 2 ? 2 : 1);
    const int wgm = 8 / wgn;
    grid = dim3((M + 16 * WM * wgm - 1) / (16 * WM * wgm), (N + 16 * WN * wgn - 1) / (16 * WN * wgn), ss.n);
}

static size_t update_slots(const SplitSet &ss, const Plan &p);

hipError_t launch_split_xgemm(const SplitSet &ss, const Plan &p, bool inverse, bool in64, int mode,
                              int pass, hipStream_t s)
{
    const int *skip = pass >= 2 ? reinterpret_cast<const int *>(blob_ptr(p, p.lay.done)) : nullptr;
    constexpr int WM = 4, WN = 4;
    int wgn;
    dim3 grid;
    xgemm_grid(ss, p, wgn, grid);
    const b8 *qs = reinterpret_cast<const b8 *>(blob_ptr(p, inverse ? p.lay.sx_inv : p.lay.sx_fwd));
    // each refinement pass keeps its update partials in a region of its own
    const size_t slots = (size_t)grid.x * grid.y * grid.z;
    const size_t region = 2 * slots;
    if (mode == 2 && (size_t)pass * region > p.lay.red_count) return hipErrorInvalidValue;
    double *red = blob_mut(p, p.lay.red) + (mode == 2 ? (size_t)(pass - 1) * region : 0);
    if (in64) {
        if (mode != 0) return hipErrorInvalidValue;
        hipLaunchKernelGGL((split_xgemm_kernel<WM, WN, double, 0>), grid, dim3(512), 0, s, ss, p.nz,
                           p.nx, p.nx, qs, wgn, red, skip);
    } else if (mode == 0) {
        hipLaunchKernelGGL((split_xgemm_kernel<WM, WN, float, 0>), grid, dim3(512), 0, s, ss, p.nz,
                           p.nx, p.nx, qs, wgn, red, skip);
    } else if (mode == 1) {
        hipLaunchKernelGGL((split_xgemm_kernel<WM, WN, float, 1>), grid, dim3(512), 0, s, ss, p.nz,
                           p.nx, p.nx, qs, wgn, red, skip);
    } else {
        hipLaunchKernelGGL((split_xgemm_kernel<WM, WN, float, 2>), grid, dim3(512), 0, s, ss, p.nz,
                           p.nx, p.nx, qs, wgn, red, skip);
    }
    return hipGetLastError();
}

hipError_t launch_split_zgemm(const SplitSet &ss, const Plan &p, bool inverse, int pass, hipStream_t s)
{
    const int *skip = pass >= 2 ? reinterpret_cast<const int *>(blob_ptr(p, p.lay.done)) : nullptr;
    constexpr int WM = 4, WN = 4;
    const int M = p.nz;
    const int Ncol = max_rows(ss) * p.nx;
    const int nroww = M / (16 * WM);
    const int wgm = nroww >= 8 ? 8 : (nroww >= 4 ? 4 : (nroww >= 2 ? 2 : 1));
    const int wgn = 8 / wgm;
    dim3 grid((Ncol + 16 * WN * wgn - 1) / (16 * WN * wgn), (M + 16 * WM * wgm - 1) / (16 * WM * wgm),
              ss.n);
    const b8 *qs = reinterpret_cast<const b8 *>(blob_ptr(p, inverse ? p.lay.sz_inv : p.lay.sz_fwd));
    hipLaunchKernelGGL((split_zgemm_kernel<WM, WN>), grid, dim3(512), 0, s, ss, M, M, p.nx, qs, wgn, skip);
    return hipGetLastError();
}

hipError_t launch_residual_f32(const SplitSet &ss, const Plan &p, int pass, hipStream_t s)
{
    const int *skip = pass >= 2 ? reinterpret_cast<const int *>(blob_ptr(p, p.lay.done)) : nullptr;
    dim3 grid(XSUM_SLOTS, ss.n);
    hipLaunchKernelGGL(residual_f32_kernel, grid, dim3(256), 0, s, ss, p.nx, p.ny, p.nz,
                       1.0 / (p.hx * p.hx), 1.0 / (p.hz * p.hz), blob_ptr(p, p.lay.dyc),
                       blob_ptr(p, p.lay.dyf), blob_ptr(p, p.lay.bmean), blob_mut(p, p.lay.xsum),
                       skip);
    return hipGetLastError();
}

static size_t update_slots(const SplitSet &ss, const Plan &p)
{
    int wgn;
    dim3 grid;
    xgemm_grid(ss, p, wgn, grid);
    return (size_t)grid.x * grid.y * grid.z;
}

int max_refine_passes(const SplitSet &ss, const Plan &p)
{
    return (int)(p.lay.red_count / (2 * update_slots(ss, p))) + 1;
}

hipError_t launch_refine_check(const SplitSet &ss, const Plan &p, int pass, hipStream_t s)
{
    int wgn;
    dim3 grid;
    xgemm_grid(ss, p, wgn, grid);
    const int per_job = (int)(grid.x * grid.y);
    const size_t region = 2 * (size_t)grid.x * grid.y * grid.z;
    const double *red = blob_ptr(p, p.lay.red);
    const double *last = red + (size_t)(pass - 1) * region;
    const double *prev = pass >= 2 ? red + (size_t)(pass - 2) * region : nullptr;
    hipLaunchKernelGGL(refine_check_kernel, dim3(ss.n), dim3(256), 0, s, ss, last, prev, per_job,
                       pass, p.desc.tol, reinterpret_cast<int *>(blob_mut(p, p.lay.done)));
    return hipGetLastError();
}

}  // namespace ibs
