// Multi-grid stage kernels: one launch per stage of the separable solve
// (Section 2.3.3, items S2.1-S2.2: x transform, z transform, y tridiagonal,
// inverse z, inverse x) covering every field of every grid of a batch.
// Each launch is persistent: its waves walk a work list in device memory
// (work item = one 64 x 64 output tile of a transform, or 64 pencils of the
// tridiagonal) whose entries name a field of the job table, so grids of any
// size mix in one launch and a batch of G grids costs 5 launches, not 5 G.
// FP64 throughout: the transforms are plain (unfolded) FP64 matrix-core
// GEMMs against the grid's own forward / inverse eigenbasis tables, the
// pencils are solved by the Thomas algorithm (diagonally dominant systems),
// one pencil per thread.
#include <algorithm>

#include "ibs_internal.h"
#include "multigrid.h"

namespace ibs {

typedef double d4 __attribute__((ext_vector_type(4)));

static __device__ __forceinline__ d4 mma(double a, double b, d4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// x transform of one (16 WM) x 64 tile per wave: C = A B, A the field's
// transform rows (M = nz * trows rows of K = nx values), B the swizzled
// nx x nx table (forward Q or inverse G^T), C rows of nx values.  The
// operand order and chunking are those of the single-grid plain kernel.
template <int WM>
__global__ __launch_bounds__(256, 3) void mg_xgemm_kernel(const MgField *__restrict__ fields,
                                                       const int4 *__restrict__ items, int nitems,
                                                       int inverse)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lg = lane >> 4;
    for (int it = blockIdx.x * 4 + wave; it < nitems; it += gridDim.x * 4) {
        const int4 w = items[it];
        const MgField &f = fields[w.x];
        const int row0 = w.y, col0 = w.z;
        const int K = f.nx, N = f.nx;
        const int skip = skip_first_row(f.kind), trows = f.rows - skip;
        const int M = f.nz * trows;
        const int nrb = min(WM, (M - row0) >> 4), ncb = min(4, (N - col0) >> 4);
        const double *__restrict__ A = inverse ? f.work : f.in;
        double *__restrict__ C = inverse ? f.out : f.work;
        const double *__restrict__ bs = inverse ? f.xinv : f.xfwd;
        const int nb = N >> 4;
        d4 acc[WM][4];
#pragma unroll
        for (int i = 0; i < WM; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[i][j] = (d4){0.0, 0.0, 0.0, 0.0};
        const double *arow[WM];
#pragma unroll
        for (int i = 0; i < WM; ++i)
            arow[i] = A + phys_row(row0 + 16 * i + (i < nrb ? li : 0), trows, skip) * K + 4 * lg;
        for (int kc = 0; kc < (K >> 4); ++kc) {
            d4 a[WM], b[4];
#pragma unroll
            for (int i = 0; i < WM; ++i)
                a[i] = (i < nrb) ? *reinterpret_cast<const d4 *>(arow[i] + 16 * kc) : (d4){0, 0, 0, 0};
#pragma unroll
            for (int j = 0; j < 4; ++j)
                b[j] = (j < ncb) ? *reinterpret_cast<const d4 *>(
                                       bs + (((size_t)kc * nb + (col0 >> 4) + j) * 64 + lane) * 4)
                                 : (d4){0, 0, 0, 0};
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int i = 0; i < WM; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j) acc[i][j] = mma(a[i][t], b[j][t], acc[i][j]);
        }
#pragma unroll
        for (int i = 0; i < WM; ++i) {
            if (i >= nrb) break;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                if (j >= ncb) break;
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    C[phys_row(row0 + 16 * i + lg + 4 * q, trows, skip) * N + col0 + 16 * j + li] = acc[i][j][q];
            }
        }
    }
}

// z transform of one (16 WM) x 64 tile per wave: C = As B, As the swizzled
// nz x nz table (forward Q^T or inverse G), B the field viewed as nz rows
// of Ncol = trows * nx values at plane stride rows * nx.  Forward reads
// work and writes out; inverse reads out and writes work.
template <int WM>
__global__ __launch_bounds__(256, 3) void mg_zgemm_kernel(const MgField *__restrict__ fields,
                                                       const int4 *__restrict__ items, int nitems,
                                                       int inverse)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lg = lane >> 4;
    for (int it = blockIdx.x * 4 + wave; it < nitems; it += gridDim.x * 4) {
        const int4 w = items[it];
        const MgField &f = fields[w.x];
        const int row0 = w.y, col0 = w.z;
        const int M = f.nz, K = f.nz, nx = f.nx;
        const int skip = skip_first_row(f.kind);
        const int Ncol = (f.rows - skip) * nx;
        const size_t ldp = (size_t)f.rows * nx;
        const int nrb = min(WM, (M - row0) >> 4), ncb = min(4, (Ncol - col0) >> 4);
        const double *__restrict__ as = inverse ? f.zinv : f.zfwd;
        const double *__restrict__ B = (inverse ? f.out : f.work) + skip * nx;
        double *__restrict__ C = (inverse ? f.work : f.out) + skip * nx;
        const int mb = M >> 4;
        d4 acc[WM][4];
#pragma unroll
        for (int i = 0; i < WM; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[i][j] = (d4){0.0, 0.0, 0.0, 0.0};
        for (int kc = 0; kc < (K >> 4); ++kc) {
            d4 a[WM], b[4];
#pragma unroll
            for (int i = 0; i < WM; ++i)
                a[i] = (i < nrb) ? *reinterpret_cast<const d4 *>(
                                       as + (((size_t)kc * mb + (row0 >> 4) + i) * 64 + lane) * 4)
                                 : (d4){0, 0, 0, 0};
            const double *brow = B + (size_t)(16 * kc + 4 * lg) * ldp + col0 + li;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const double *bt = brow + (size_t)t * ldp;   // one address per row, the blocks at immediate offsets
#pragma unroll
                for (int j = 0; j < 4; ++j) b[j][t] = (j < ncb) ? bt[16 * j] : 0.0;
            }
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int i = 0; i < WM; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j) acc[i][j] = mma(a[i][t], b[j][t], acc[i][j]);
        }
#pragma unroll
        for (int i = 0; i < WM; ++i) {
            if (i >= nrb) break;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                if (j >= ncb) break;
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    C[(size_t)(row0 + 16 * i + lg + 4 * q) * ldp + col0 + 16 * j + li] = acc[i][j][q];
            }
        }
    }
}

// y pencils: item (field, plane c, first pencil a0), one pencil a = a0 +
// lane per thread, in place on out.  System of pencil (a, c), shift s =
// lambda_x[a] + lambda_z[c]: Poisson L_y + s, Helmholtz I - c (L_y + s), L_y
// the kind's y rows.  Face unknowns (v) are rows 1..ny-1, their wall rows 0
// and ny are written as 0.  The Poisson (0,0) pencil is singular (the
// constant mode): the Delta-weighted mean of its right-hand side is removed
// (the rhs's volume-weighted mean, scaled by sqrt(nx nz)), row 0 is pinned
// to 0, and the weighted mean of the result is removed (zero volume-
// weighted mean of the solution).
// Thomas elimination: m_j = d_j - a_j cp_{j-1}, cp_j = c_j / m_j, forward
// x_j <- (b_j - a_j x_{j-1}) / m_j, back substitution x_j -= cp_j x_{j+1}.
// The factors cp depend on the system only, not on the data: the batch
// builds them once (FACTOR), and each solve reads them in its back
// substitution instead of writing and reading them back (40 instead of 48
// bytes per cell).  Both launches form the rows in the same code.

// row j of pencil (shift s) in the form a x_{j-1} + m x_j + c x_{j+1}
struct MgRow {
    double a, m, c;
};
static __device__ __forceinline__ MgRow mg_row(int j, int j0, int j1, double lj, double dj, double uj, bool pois,
                                               double cc, double s, bool pinned)
{
    if (j == j0) lj = 0.0;
    if (j == j1) uj = 0.0;
    MgRow r;
    if (pois) { r.a = lj; r.m = dj + s; r.c = uj; }
    else { r.a = -cc * lj; r.m = 1.0 - cc * (dj + s); r.c = -cc * uj; }
    if (pinned && j == j0) { r.a = 0.0; r.m = 1.0; r.c = 0.0; }
    return r;
}

template <bool FACTOR>
__global__ __launch_bounds__(256) void mg_tridiag_kernel(const MgField *__restrict__ fields,
                                                         const int4 *__restrict__ items, int nitems)
{
    // Rows are read in bursts of TR, every load of a burst issued before the
    // first row of the burst is eliminated (a row's store may not be moved
    // above a later row's load, so loads issued row by row would each wait
    // for the memory in turn).
    constexpr int TR = 8;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int it0 = blockIdx.x * 4 + wave; it0 < nitems; it0 += gridDim.x * 4) {
        const int it = __builtin_amdgcn_readfirstlane(it0);   // wave-uniform item
        const int4 w = items[it];
        const MgField &f = fields[w.x];
        const int c = w.y, a = w.z + lane;
        if (a >= f.nx) continue;
        const int nx = f.nx;
        const bool faces = f.kind == KIND_F;
        const int j0 = faces ? 1 : 0, j1 = f.ny - 1;   // unknown rows j0..j1
        double *__restrict__ x = f.out + (size_t)c * f.rows * nx + a;
        double *__restrict__ cp = f.cpt + (size_t)c * f.rows * nx + a;
        // the y rows are read-only here and the same for every lane: read
        // through the scalar cache
        typedef const __attribute__((address_space(4))) double *crow;
        const crow lo = (crow)f.lo, di = (crow)f.di, up = (crow)f.up;
        const double s = f.lam_x[a] + f.lam_z[c];
        const bool pois = f.poisson != 0;
        const double cc = f.c;
        const bool pinned = pois && a == 0 && c == 0;
        if constexpr (FACTOR) {
            double cprev = 0.0;
            for (int j = j0; j <= j1; ++j) {
                const MgRow r = mg_row(j, j0, j1, lo[j], di[j], up[j], pois, cc, s, pinned);
                const double im = 1.0 / (r.m - r.a * cprev);   // as in the forward sweep
                cprev = r.c * im;
                cp[(size_t)j * nx] = cprev;
            }
            continue;
        }
        double mean = 0.0;
        if (pinned) {
            double sw = 0.0, swd = 0.0;
            for (int j = j0; j <= j1; ++j) {
                sw += f.wy[j];
                swd += f.wy[j] * x[(size_t)j * nx];
            }
            mean = swd / sw;
        }
        // forward sweep (the factors kept in registers only)
        double cprev = 0.0, dprev = 0.0;
        auto fwd_row = [&](int j, double bj, double lj, double dj, double uj) {
            const MgRow r = mg_row(j, j0, j1, lj, dj, uj, pois, cc, s, pinned);
            bj = (pinned && j == j0) ? 0.0 : bj - mean;
            const double im = 1.0 / (r.m - r.a * cprev);
            cprev = r.c * im;
            dprev = (bj - r.a * dprev) * im;
            x[(size_t)j * nx] = dprev;
        };
        int j = j0;
        for (; j + TR - 1 <= j1; j += TR) {   // whole bursts: no branch between the loads
            double bv[TR], lv[TR], dv[TR], uv[TR];
#pragma unroll
            for (int r = 0; r < TR; ++r) {
                bv[r] = x[(size_t)(j + r) * nx];
                lv[r] = lo[j + r];
                dv[r] = di[j + r];
                uv[r] = up[j + r];
            }
#pragma unroll
            for (int r = 0; r < TR; ++r) fwd_row(j + r, bv[r], lv[r], dv[r], uv[r]);
        }
        for (; j <= j1; ++j) fwd_row(j, x[(size_t)j * nx], lo[j], di[j], up[j]);
        // back substitution: x_j = x_j - cp_j x_{j+1}, in bursts going down
        double xn = dprev;   // row j1 is final
        j = j1 - 1;
        for (; j - (TR - 1) >= j0; j -= TR) {
            double dv[TR], cv[TR];
#pragma unroll
            for (int r = 0; r < TR; ++r) {
                dv[r] = x[(size_t)(j - r) * nx];
                cv[r] = cp[(size_t)(j - r) * nx];
            }
#pragma unroll
            for (int r = 0; r < TR; ++r) {
                xn = dv[r] - cv[r] * xn;
                x[(size_t)(j - r) * nx] = xn;
            }
        }
        for (; j >= j0; --j) {
            xn = x[(size_t)j * nx] - cp[(size_t)j * nx] * xn;
            x[(size_t)j * nx] = xn;
        }
        if (faces) {
            x[0] = 0.0;
            x[(size_t)f.ny * nx] = 0.0;
        }
        if (pinned) {
            double sw = 0.0, swx = 0.0;
            for (int j = j0; j <= j1; ++j) {
                sw += f.wy[j];
                swx += f.wy[j] * x[(size_t)j * nx];
            }
            const double mx = swx / sw;
            for (int j = j0; j <= j1; ++j) x[(size_t)j * nx] -= mx;
        }
        if (a == 0 && c == 0 && f.info) {
            ibs_solve_info *inf = f.info;
            inf->iters = 1;
            inf->status = IBS_OK;
            inf->rel_residual = 0.0;
            inf->rel_correction = 0.0;
            inf->removed_mean = pois ? mean * f.inv_sqrt_nxnz : 0.0;
        }
    }
}

// Blocks of `kernel` (256 threads) resident on the device at once: the
// persistent grid size.
template <typename K>
static int resident(K kernel)
{
    int per_cu = 0, dev = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 256, 0) != hipSuccess ||
        hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        per_cu * cus <= 0)
        return 256;
    return std::min(per_cu * cus, MG_MAX_BLOCKS);
}

hipError_t launch_multigrid_stage(int stage, const MgField *fields, const int4 *items, int nitems,
                                  hipStream_t s)
{
    if (nitems <= 0) return hipSuccess;
    static const int rx = resident(mg_xgemm_kernel<MG_WM>), rz = resident(mg_zgemm_kernel<MG_WM>),
                     rt = resident(mg_tridiag_kernel<false>);
    const int res = (stage == MG_TRI || stage == MG_FACTOR) ? rt : (stage == MG_Z_FWD || stage == MG_Z_INV ? rz : rx);
    const int blocks = std::min((nitems + 3) / 4, res);
    switch (stage) {
    case MG_X_FWD: hipLaunchKernelGGL(mg_xgemm_kernel<MG_WM>, dim3(blocks), dim3(256), 0, s, fields, items, nitems, 0); break;
    case MG_Z_FWD: hipLaunchKernelGGL(mg_zgemm_kernel<MG_WM>, dim3(blocks), dim3(256), 0, s, fields, items, nitems, 0); break;
    case MG_TRI: hipLaunchKernelGGL(mg_tridiag_kernel<false>, dim3(blocks), dim3(256), 0, s, fields, items, nitems); break;
    case MG_FACTOR: hipLaunchKernelGGL(mg_tridiag_kernel<true>, dim3(blocks), dim3(256), 0, s, fields, items, nitems); break;
    case MG_Z_INV: hipLaunchKernelGGL(mg_zgemm_kernel<MG_WM>, dim3(blocks), dim3(256), 0, s, fields, items, nitems, 1); break;
    default: hipLaunchKernelGGL(mg_xgemm_kernel<MG_WM>, dim3(blocks), dim3(256), 0, s, fields, items, nitems, 1); break;
    }
    return hipGetLastError();
}

}  // namespace ibs
