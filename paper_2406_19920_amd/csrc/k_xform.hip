// Eigen-transforms of the x and z directions as FP64 matrix-core GEMMs.
//
// The x transform contracts the innermost (x) index of every row of a
// [nz][rows][nx] field with an nx x nx matrix (forward: Q, inverse: Q^T);
// the z transform contracts the outermost (z) index, i.e. it multiplies the
// field viewed as an nz x (rows*nx) matrix from the left by an nz x nz matrix
// (forward: Q^T, inverse: Q).  These are the dense-matrix counterpart of the
// paper's 2-D FFT over the periodic directions (Section 2.3.3, items S1.1,
// S1.2, S2.1, S2.2); with walls in x, Q is the eigenbasis of the field's
// wall-bounded x operator (cosine or sine series), one matrix per job.
//
// Instruction: V_MFMA_F64_16X16X4_F64.  Per lane l of the 64-wide wave: A
// element (row l%16, k l/16), B element (k l/16, col l%16); result element q
// (q = 0..3) is row l/16 + 4q, column l%16 (checked on gfx950).  The K index inside a 16-deep chunk is
// permuted so that lane l feeds k = 4*(l/16) + t at step t = 0..3: then each
// lane reads four consecutive K values of its row (a 32-byte load).  The
// transform matrices are pre-swizzled on the host into exactly that order.
#include "ibs_internal.h"

namespace ibs {

typedef double d4 __attribute__((ext_vector_type(4)));

static __device__ __forceinline__ d4 mfma(double a, double b, d4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// x transform: for job q, C = A * B with A = in (M x K row-major, M = nz*rows),
// B = the job's swizzled K x N matrix (xq), C = out (M x N row-major).
// Workgroup of 4 waves laid out wgm x wgn; each wave owns a (16*WM) x
// (16*WN) tile.
template <int WM, int WN>
__global__ __launch_bounds__(256) void xgemm_f64_kernel(JobSet js, int nz, int K, int N, int wgn)
{
    const FieldJob &jb = js.j[blockIdx.z];
    const double *__restrict__ bs = static_cast<const double *>(jb.xq);
    const int skip = skip_first_row(jb.kind), trows = jb.rows - skip;
    const int M = nz * trows;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wgm = 4 / wgn;
    const int wm = wave / wgn, wn = wave % wgn;
    const int row0 = (blockIdx.x * wgm + wm) * (16 * WM);
    const int col0 = (blockIdx.y * wgn + wn) * (16 * WN);
    if (row0 >= M || col0 >= N) return;
    const int nrb = min(WM, (M - row0) >> 4);
    const int ncb = min(WN, (N - col0) >> 4);
    const int li = lane & 15, lg = lane >> 4;
    const double *__restrict__ A = jb.in;
    const int nb = N >> 4;
    d4 acc[WM][WN];
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j) acc[i][j] = (d4){0.0, 0.0, 0.0, 0.0};
    const double *arow[WM];
#pragma unroll
    for (int i = 0; i < WM; ++i)
        arow[i] = A + phys_row(row0 + 16 * i + (i < nrb ? li : 0), trows, skip) * K + 4 * lg;
    for (int kc = 0; kc < (K >> 4); ++kc) {
        d4 a[WM], b[WN];
#pragma unroll
        for (int i = 0; i < WM; ++i)
            a[i] = (i < nrb) ? *reinterpret_cast<const d4 *>(arow[i] + 16 * kc) : (d4){0, 0, 0, 0};
#pragma unroll
        for (int j = 0; j < WN; ++j)
            b[j] = (j < ncb) ? *reinterpret_cast<const d4 *>(
                                   bs + (((size_t)kc * nb + (col0 >> 4) + j) * 64 + lane) * 4)
                             : (d4){0, 0, 0, 0};
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int i = 0; i < WM; ++i)
#pragma unroll
                for (int j = 0; j < WN; ++j) acc[i][j] = mfma(a[i][t], b[j][t], acc[i][j]);
    }
    double *__restrict__ C = jb.out;
#pragma unroll
    for (int i = 0; i < WM; ++i) {
        if (i >= nrb) break;
#pragma unroll
        for (int j = 0; j < WN; ++j) {
            if (j >= ncb) break;
#pragma unroll
            for (int q = 0; q < 4; ++q)
                C[phys_row(row0 + 16 * i + lg + 4 * q, trows, skip) * N + col0 + 16 * j + li] = acc[i][j][q];
        }
    }
}

// z transform: for job q, C = As * B with As the swizzled M x K matrix
// (M = K = nz), B = in viewed as K x Ncol (Ncol = transform rows * nx, at
// plane stride rows * nx), C = out (M x Ncol).
// Registers held to two waves per SIMD (the 4 x 4 tile's accumulators
// then sit in the vector registers; unbounded, the allocation came to one
// wave per SIMD).
template <int WM, int WN>
__global__ __launch_bounds__(256, 2) void zgemm_f64_kernel(JobSet js, int M, int K, int nx, int wgn)
{
    const FieldJob &jb = js.j[blockIdx.z];
    const double *__restrict__ as = static_cast<const double *>(jb.zq);
    const int skip = skip_first_row(jb.kind);
    const int Ncol = (jb.rows - skip) * nx;
    const size_t ldp = (size_t)jb.rows * nx;   // plane stride
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wgm = 4 / wgn;
    const int wm = wave / wgn, wn = wave % wgn;
    const int row0 = (blockIdx.y * wgm + wm) * (16 * WM);
    const int col0 = (blockIdx.x * wgn + wn) * (16 * WN);
    if (row0 >= M || col0 >= Ncol) return;
    const int nrb = min(WM, (M - row0) >> 4);
    const int ncb = min(WN, (Ncol - col0) >> 4);
    const int li = lane & 15, lg = lane >> 4;
    const double *__restrict__ B = jb.in + skip * nx;
    const int mb = M >> 4;
    d4 acc[WM][WN];
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j) acc[i][j] = (d4){0.0, 0.0, 0.0, 0.0};
    for (int kc = 0; kc < (K >> 4); ++kc) {
        d4 a[WM], b[WN];
#pragma unroll
        for (int i = 0; i < WM; ++i)
            a[i] = (i < nrb) ? *reinterpret_cast<const d4 *>(
                                   as + (((size_t)kc * mb + (row0 >> 4) + i) * 64 + lane) * 4)
                             : (d4){0, 0, 0, 0};
        const double *brow = B + (size_t)(16 * kc + 4 * lg) * ldp + col0 + li;
#pragma unroll
        for (int j = 0; j < WN; ++j) {
            if (j < ncb) {
#pragma unroll
                for (int t = 0; t < 4; ++t) b[j][t] = brow[(size_t)t * ldp + 16 * j];
            } else {
                b[j] = (d4){0, 0, 0, 0};
            }
        }
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int i = 0; i < WM; ++i)
#pragma unroll
                for (int j = 0; j < WN; ++j) acc[i][j] = mfma(a[i][t], b[j][t], acc[i][j]);
    }
    double *__restrict__ C = jb.out + skip * nx;
#pragma unroll
    for (int i = 0; i < WM; ++i) {
        if (i >= nrb) break;
#pragma unroll
        for (int j = 0; j < WN; ++j) {
            if (j >= ncb) break;
#pragma unroll
            for (int q = 0; q < 4; ++q)
                C[(size_t)(row0 + 16 * i + lg + 4 * q) * ldp + col0 + 16 * j + li] = acc[i][j][q];
        }
    }
}

static int max_rows(const JobSet &js)   // transform rows per plane
{
    int r = 0;
    for (int q = 0; q < js.n; ++q) {
        const int t = js.j[q].rows - skip_first_row(js.j[q].kind);
        r = t > r ? t : r;
    }
    return r;
}

hipError_t launch_xgemm_f64(const JobSet &js_in, int nz, int K, int N, const double *const bs[NUM_XK],
                            hipStream_t s)
{
    JobSet js = js_in;
    for (int q = 0; q < js.n; ++q) js.j[q].xq = bs[js.j[q].xk];
    constexpr int WM = 4, WN = 4;
    const int M = nz * max_rows(js);
    // arrange the 4 waves over columns first (up to N/64 of them)
    const int nwave_cols = N / (16 * WN);
    int wgn = nwave_cols >= 4 ? 4 : (nwave_cols >= 2 ? 2 : 1);
    int wgm = 4 / wgn;
    dim3 grid((M + 16 * WM * wgm - 1) / (16 * WM * wgm), (N + 16 * WN * wgn - 1) / (16 * WN * wgn),
              js.n);
    hipLaunchKernelGGL((xgemm_f64_kernel<WM, WN>), grid, dim3(256), 0, s, js, nz, K, N, wgn);
    return hipGetLastError();
}

hipError_t launch_zgemm_f64(const JobSet &js_in, int M, int K, int nx, const double *const as[NUM_XK],
                            hipStream_t s)
{
    JobSet js = js_in;
    for (int q = 0; q < js.n; ++q) js.j[q].zq = as[js.j[q].zk];
    constexpr int WM = 4, WN = 4;
    const int Ncol = max_rows(js) * nx;
    int wgm = M >= 256 ? 4 : (M >= 128 ? 2 : 1);
    int wgn = 4 / wgm;
    dim3 grid((Ncol + 16 * WN * wgn - 1) / (16 * WN * wgn), (M + 16 * WM * wgm - 1) / (16 * WM * wgm),
              js.n);
    hipLaunchKernelGGL((zgemm_f64_kernel<WM, WN>), grid, dim3(256), 0, s, js, M, K, nx, wgn);
    return hipGetLastError();
}

}  // namespace ibs
