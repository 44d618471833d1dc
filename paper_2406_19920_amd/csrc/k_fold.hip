// Folded eigen-transforms of the periodic directions (FP64 matrix cores).
//
// The real Fourier basis Q (Appendix A: cos and sin modes, plus the mean
// and the alternating Nyquist mode) has a mirror symmetry in the grid
// index: with H = N/2, Q[N-i][a] = Q[i][a] for the cos, mean and Nyquist
// columns and Q[N-i][a] = -Q[i][a] for the sin columns.  So, per row,
//   forward:  E[i] = X[i] + X[N-i],  O[i] = X[i] - X[N-i]   (1 <= i < H)
//             cos outputs  = E Qc (+ the X[H] term),
//             sin outputs  = O Qs,
//   inverse:  U = Xc Qc^T (+ the Nyquist term),  V = Xs Qs^T,
//             X[i] = U[i] + V[i],  X[N-i] = U[i] - V[i],
// which are two H x H products instead of one N x N product: half the
// matrix-core work of the plain transform.  The odd cases are the four
// self-mirrored points: X[0] (the E slot 0), X[H] (carried in the unused
// O slot 0), the Nyquist output of the forward transform and the X[H]
// output of the inverse (both alternating sums, done on the vector units
// while the K loop runs).
//
// Spectral layout (as for the plain transform): index a < H is cos mode a
// (a = 0 the mean), a = H the Nyquist mode, H + k (1 <= k < H) sin mode k.
// Instruction layout as in the plain kernels: lane l feeds A(row l%16,
// k 4(l/16)+t) and B(k 4(l/16)+t, col l%16), t = 0..3; result element q
// is row l/16 + 4q, column l%16.  Requires H a multiple of 16.
#include "ibs_internal.h"

// No implicit multiply-add fusion in this file: every rounding is written
// out (fma() where wanted), so that all tile shapes give the same bits.
#pragma clang fp contract(off)

namespace ibs {

typedef double d4 __attribute__((ext_vector_type(4)));

static __device__ __forceinline__ d4 mfma(double a, double b, d4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// x transform of every row of a [nz][rows][N] field.  Forward: the
// physical row -> spectral row; inverse: spectral -> physical.  bc, bs:
// the two H x H factors, swizzled as B operands.  A wave owns WM row
// blocks and WN column blocks of both factors.
// Waves per SIMD the register allocation is held to, where the tile fits
// without spilling: three for the small tiles (the memory latency then has
// a third wave to hide behind), two for the tiles that load ahead (left
// alone they took one), else what the tile needs.
template <int WM, int WN, bool PF>
constexpr int xf_waves() { return (!PF && WM * WN <= 4 && WM <= 2) ? 3 : (PF ? 2 : 1); }
template <int WM, int WN, bool PF>
constexpr int zf_waves() { return (!PF && WM * WN <= 4 && WN <= 2) ? 3 : ((PF && WN <= 2) ? 2 : 1); }

template <int WM, int WN, bool INV, bool PF>
__global__ __launch_bounds__(256, (xf_waves<WM, WN, PF>())) void xfold_f64_kernel(JobSet js, int nz, int N,
                                                        const double *__restrict__ bc,
                                                        const double *__restrict__ bs, int wgn,
                                                        double s0, double s1)
{
    const FieldJob &jb = js.j[blockIdx.z];
    const int skip = skip_first_row(jb.kind), trows = jb.rows - skip;
    const int M = nz * trows;
    const int H = N >> 1, HB = H >> 4;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wgm = 4 / wgn;
    const int wm = wave / wgn, wn = wave % wgn;
    const int row0 = (blockIdx.x * wgm + wm) * (16 * WM);
    const int cb0 = (blockIdx.y * wgn + wn) * WN;
    if (row0 >= M || cb0 >= HB) return;
    const int nrb = min(WM, (M - row0) >> 4);
    const int ncb = min(WN, HB - cb0);
    const int li = lane & 15, lg = lane >> 4;
    const double *__restrict__ A = jb.in;
    double *__restrict__ C = jb.out;

    d4 acc_c[WM][WN], acc_s[WM][WN];
    double nyq[WM];
#pragma unroll
    for (int i = 0; i < WM; ++i) {
        nyq[i] = 0.0;
#pragma unroll
        for (int j = 0; j < WN; ++j) {
            acc_c[i][j] = (d4){0.0, 0.0, 0.0, 0.0};
            acc_s[i][j] = (d4){0.0, 0.0, 0.0, 0.0};
        }
    }
    const double *arow[WM];
#pragma unroll
    for (int i = 0; i < WM; ++i) arow[i] = A + phys_row(row0 + 16 * i + (i < nrb ? li : 0), trows, skip) * N;

    // raw operands of one 16-deep chunk: the row data (forward: X[k] and
    // X[mirror k]; inverse: cos and sin inputs) and both factors' fragments.
    // The next chunk's are loaded while the current chunk is multiplied.
    // forward: ma holds the mirrored run X[N-k0-3 .. N-k0] as loaded (one
    // 4-wide load), reversed where it is used; kk = 0 pairs with X[H]
    // instead, so lanes with k0 = 0 load the run N-4 .. N-1 and xh = X[H]
    d4 pa[WM], ma[WM], fc[WN], fs[WN];
    double xh[WM];
    auto load = [&](int kc) {
        const int k0 = 16 * kc + 4 * lg;
#pragma unroll
        for (int i = 0; i < WM; ++i) {
            if (i < nrb) {   // wave-uniform
                pa[i] = *reinterpret_cast<const d4 *>(arow[i] + k0);
                if (!INV) {
                    __builtin_memcpy(&ma[i], arow[i] + (k0 == 0 ? N - 4 : N - k0 - 3), sizeof(d4));
                    if (kc == 0) xh[i] = arow[i][H];   // wave-uniform
                } else {
                    ma[i] = *reinterpret_cast<const d4 *>(arow[i] + H + k0);
                }
            } else {
                pa[i] = (d4){0, 0, 0, 0};
                ma[i] = (d4){0, 0, 0, 0};
                xh[i] = 0.0;
            }
        }
#pragma unroll
        for (int j = 0; j < WN; ++j) {
            if (j < ncb) {
                const size_t o = (((size_t)kc * HB + cb0 + j) * 64 + lane) * 4;
                fc[j] = *reinterpret_cast<const d4 *>(bc + o);
                fs[j] = *reinterpret_cast<const d4 *>(bs + o);
            } else {
                fc[j] = (d4){0, 0, 0, 0};
                fs[j] = (d4){0, 0, 0, 0};
            }
        }
    };
    if (PF) load(0);
    for (int kc = 0; kc < HB; ++kc) {
        const int k0 = 16 * kc + 4 * lg;
        if (!PF) load(kc);   // no prefetch: fewer registers, more waves
        d4 xc[WM], xs[WM];   // forward: E, O; inverse: cos and sin inputs
#pragma unroll
        for (int i = 0; i < WM; ++i) {
            if (!INV) {
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const bool self = k0 + t == 0;
                    const double m = k0 == 0 ? (t == 0 ? xh[i] : ma[i][4 - t]) : ma[i][3 - t];
                    xc[i][t] = self ? pa[i][t] : pa[i][t] + m;
                    xs[i][t] = self ? m : pa[i][t] - m;
                }
                // Nyquist output: sum of (-1)^i E[i]
                nyq[i] += (xc[i][0] - xc[i][1]) + (xc[i][2] - xc[i][3]);
            } else {
                xc[i] = pa[i];
                xs[i] = ma[i];
                // physical point H: sum of Q[H][a] Xc[a], Q[H][a] = w_a (-1)^a
                nyq[i] = fma(k0 == 0 ? s0 : s1, xc[i][0], nyq[i]);
                nyq[i] = fma(-s1, xc[i][1], nyq[i]);
                nyq[i] = fma(s1, xc[i][2], nyq[i]);
                nyq[i] = fma(-s1, xc[i][3], nyq[i]);
            }
        }
        d4 b_c[WN], b_s[WN];
#pragma unroll
        for (int j = 0; j < WN; ++j) { b_c[j] = fc[j]; b_s[j] = fs[j]; }
        if (PF && kc + 1 < HB) load(kc + 1);
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int i = 0; i < WM; ++i)
#pragma unroll
                for (int j = 0; j < WN; ++j) {
                    acc_c[i][j] = mfma(xc[i][t], b_c[j][t], acc_c[i][j]);
                    acc_s[i][j] = mfma(xs[i][t], b_s[j][t], acc_s[i][j]);
                }
    }

    const double sH = (H & 1) ? -s0 : s0;   // Q[H][H]
#pragma unroll
    for (int i = 0; i < WM; ++i) {
        if (i >= nrb) break;
        double ny = nyq[i];
        ny += __shfl_xor(ny, 16, 64);
        ny += __shfl_xor(ny, 32, 64);   // every lane of row li holds its sum
        const int rb = row0 + 16 * i;
        size_t orow[4];                 // physical output rows of the lane
        double ah[4];                   // A[row][H] of those rows
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            orow[q] = phys_row(rb + lg + 4 * q, trows, skip) * N;
            ah[q] = A[orow[q] + H];
        }
        if (!INV) {
            double nyr[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) nyr[q] = __shfl(ny, lg + 4 * q, 64);
#pragma unroll
            for (int j = 0; j < WN; ++j) {
                if (j >= ncb) break;
                const int a = 16 * (cb0 + j) + li;
                const double wa = (a == 0 ? s0 : s1) * ((a & 1) ? -1.0 : 1.0);   // Q[H][a]
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const size_t o = orow[q];
                    C[o + a] = fma(ah[q], wa, acc_c[i][j][q]);
                    double sv = acc_s[i][j][q];
                    if (a == 0) sv = fma(s0, nyr[q], sv);   // spectral index H: Nyquist
                    C[o + H + a] = sv;
                }
            }
        } else {
            if (cb0 == 0 && lg == 0) {   // physical point H of row li
                const size_t r = phys_row(rb + li, trows, skip) * N;
                C[r + H] = fma(A[r + H], sH, ny);
            }
#pragma unroll
            for (int j = 0; j < WN; ++j) {
                if (j >= ncb) break;
                const int ii = 16 * (cb0 + j) + li;
                const double sg = (ii & 1) ? -s0 : s0;   // Q[ii][H]
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const size_t o = orow[q];
                    const double u = fma(ah[q], sg, acc_c[i][j][q]), v = acc_s[i][j][q];
                    C[o + ii] = u + v;
                    if (ii != 0) C[o + N - ii] = u - v;
                }
            }
        }
    }
}

// z transform: the field viewed as N x Ncol (N = nz planes, Ncol =
// rows*nx), multiplied from the left.  ac, as: the two H x H factors,
// swizzled as A operands.  A wave owns WM row blocks (of both factors) and
// WN column blocks.
template <int WM, int WN, bool INV, bool PF>
__global__ __launch_bounds__(256, (zf_waves<WM, WN, PF>())) void zfold_f64_kernel(JobSet js, int N, int nx,
                                                        const double *__restrict__ ac,
                                                        const double *__restrict__ as, int wgn,
                                                        double s0, double s1)
{
    const FieldJob &jb = js.j[blockIdx.z];
    const int skip = skip_first_row(jb.kind);
    const int Ncol = (jb.rows - skip) * nx;
    const size_t ldp = (size_t)jb.rows * nx;   // plane stride
    const int H = N >> 1, HB = H >> 4;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wgm = 4 / wgn;
    const int wm = wave / wgn, wn = wave % wgn;
    const int rb0 = (blockIdx.y * wgm + wm) * WM;
    const int col0 = (blockIdx.x * wgn + wn) * (16 * WN);
    if (rb0 >= HB || col0 >= Ncol) return;
    const int nrb = min(WM, HB - rb0);
    const int ncb = min(WN, (Ncol - col0) >> 4);
    const int li = lane & 15, lg = lane >> 4;
    const double *__restrict__ B = jb.in + skip * nx;
    double *__restrict__ C = jb.out + skip * nx;

    d4 acc_c[WM][WN], acc_s[WM][WN];
    double nyq[WN];
#pragma unroll
    for (int j = 0; j < WN; ++j) {
        nyq[j] = 0.0;
#pragma unroll
        for (int i = 0; i < WM; ++i) {
            acc_c[i][j] = (d4){0.0, 0.0, 0.0, 0.0};
            acc_s[i][j] = (d4){0.0, 0.0, 0.0, 0.0};
        }
    }
    // raw operands of one 16-deep chunk (both factors' fragments; the
    // column data: forward X[k] and X[mirror k], inverse cos and sin planes);
    // the next chunk's are loaded while the current chunk is multiplied
    d4 fa[WM], fb[WM], pa[WN], ma[WN];
    auto load = [&](int kc) {
        const int k0 = 16 * kc + 4 * lg;
#pragma unroll
        for (int i = 0; i < WM; ++i) {
            if (i < nrb) {
                const size_t o = (((size_t)kc * HB + rb0 + i) * 64 + lane) * 4;
                fa[i] = *reinterpret_cast<const d4 *>(ac + o);
                fb[i] = *reinterpret_cast<const d4 *>(as + o);
            } else {
                fa[i] = (d4){0, 0, 0, 0};
                fb[i] = (d4){0, 0, 0, 0};
            }
        }
#pragma unroll
        for (int j = 0; j < WN; ++j) {
            if (j < ncb) {
                const double *col = B + col0 + 16 * j + li;
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int kk = k0 + t;
                    pa[j][t] = col[(size_t)kk * ldp];
                    ma[j][t] = col[(size_t)(INV ? H + kk : (kk == 0 ? H : N - kk)) * ldp];
                }
            } else {
                pa[j] = (d4){0, 0, 0, 0};
                ma[j] = (d4){0, 0, 0, 0};
            }
        }
    };
    if (PF) load(0);
    for (int kc = 0; kc < HB; ++kc) {
        const int k0 = 16 * kc + 4 * lg;
        if (!PF) load(kc);   // no prefetch: fewer registers, more waves
        d4 a_c[WM], a_s[WM];
#pragma unroll
        for (int i = 0; i < WM; ++i) { a_c[i] = fa[i]; a_s[i] = fb[i]; }
        d4 xc[WN], xs[WN];
#pragma unroll
        for (int j = 0; j < WN; ++j) {
            if (!INV) {
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const bool self = k0 + t == 0;
                    xc[j][t] = self ? pa[j][t] : pa[j][t] + ma[j][t];
                    xs[j][t] = self ? ma[j][t] : pa[j][t] - ma[j][t];
                }
                nyq[j] += (xc[j][0] - xc[j][1]) + (xc[j][2] - xc[j][3]);
            } else {
                xc[j] = pa[j];
                xs[j] = ma[j];
                nyq[j] = fma(k0 == 0 ? s0 : s1, xc[j][0], nyq[j]);
                nyq[j] = fma(-s1, xc[j][1], nyq[j]);
                nyq[j] = fma(s1, xc[j][2], nyq[j]);
                nyq[j] = fma(-s1, xc[j][3], nyq[j]);
            }
        }
        if (PF && kc + 1 < HB) load(kc + 1);
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int i = 0; i < WM; ++i)
#pragma unroll
                for (int j = 0; j < WN; ++j) {
                    acc_c[i][j] = mfma(a_c[i][t], xc[j][t], acc_c[i][j]);
                    acc_s[i][j] = mfma(a_s[i][t], xs[j][t], acc_s[i][j]);
                }
    }

    const double sH = (H & 1) ? -s0 : s0;
#pragma unroll
    for (int j = 0; j < WN; ++j) {
        if (j >= ncb) break;
        const size_t cc = (size_t)(col0 + 16 * j + li);
        double ny = nyq[j];
        ny += __shfl_xor(ny, 16, 64);
        ny += __shfl_xor(ny, 32, 64);   // every lane of column li holds its sum
        const double bh = B[(size_t)H * ldp + cc];
        if (INV && rb0 == 0 && lg == 0) C[(size_t)H * ldp + cc] = fma(bh, sH, ny);
#pragma unroll
        for (int i = 0; i < WM; ++i) {
            if (i >= nrb) break;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int r = 16 * (rb0 + i) + lg + 4 * q;   // 0 <= r < H
                if (!INV) {
                    const double wr = (r == 0 ? s0 : s1) * ((r & 1) ? -1.0 : 1.0);   // Q[H][r]
                    C[(size_t)r * ldp + cc] = fma(bh, wr, acc_c[i][j][q]);
                    double sv = acc_s[i][j][q];
                    if (r == 0) sv = fma(s0, ny, sv);   // plane H: Nyquist
                    C[(size_t)(H + r) * ldp + cc] = sv;
                } else {
                    const double u = fma(bh, (r & 1) ? -s0 : s0, acc_c[i][j][q]), v = acc_s[i][j][q];
                    C[(size_t)r * ldp + cc] = u + v;
                    if (r != 0) C[(size_t)(N - r) * ldp + cc] = u - v;
                }
            }
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

// can_fold() is defined with the plan builder (host code).

// Tile candidates (row blocks x column blocks per wave, and whether the next
// chunk's operands are loaded ahead at the cost of registers).  Every
// candidate sums each output element in the same order, so the choice
// changes only the speed, never the result.
static constexpr int XF_WM[] = {2, 4, 4, 1, 2, 1, 2, 1};
static constexpr int XF_WN[] = {2, 1, 2, 4, 2, 4, 1, 2};
static constexpr int ZF_WM[] = {2, 1, 2, 4, 2, 1, 2, 1};
static constexpr int ZF_WN[] = {2, 4, 4, 1, 2, 4, 1, 2};
static constexpr bool F_PF[] = {false, false, false, false, true, true, true, true};
int fold_candidates() { return 8; }

template <int WM, int WN, bool PF>
static hipError_t xfold_launch(const JobSet &js, const Plan &p, bool inverse, hipStream_t s)
{
    const int N = p.nx, HB = N / 32;
    const int M = p.nz * max_rows(js);
    const int nwave_cols = (HB + WN - 1) / WN;
    const int wgn = nwave_cols >= 4 ? 4 : (nwave_cols >= 2 ? 2 : 1);
    const int wgm = 4 / wgn;
    dim3 grid((M + 16 * WM * wgm - 1) / (16 * WM * wgm), (nwave_cols + wgn - 1) / wgn, js.n);
    const double *bc = blob_ptr(p, inverse ? p.lay.fx_inv_c : p.lay.fx_fwd_c);
    const double *bs = blob_ptr(p, inverse ? p.lay.fx_inv_s : p.lay.fx_fwd_s);
    const double s0 = 1.0 / std::sqrt((double)N), s1 = std::sqrt(2.0 / (double)N);
    if (inverse)
        hipLaunchKernelGGL((xfold_f64_kernel<WM, WN, true, PF>), grid, dim3(256), 0, s, js, p.nz, N, bc, bs,
                           wgn, s0, s1);
    else
        hipLaunchKernelGGL((xfold_f64_kernel<WM, WN, false, PF>), grid, dim3(256), 0, s, js, p.nz, N, bc,
                           bs, wgn, s0, s1);
    return hipGetLastError();
}

template <int WM, int WN, bool PF>
static hipError_t zfold_launch(const JobSet &js, const Plan &p, bool inverse, hipStream_t s)
{
    const int N = p.nz, HB = N / 32;
    const int Ncol = max_rows(js) * p.nx;
    const int nwave_rows = (HB + WM - 1) / WM;
    const int wgm = nwave_rows >= 4 ? 4 : (nwave_rows >= 2 ? 2 : 1);
    const int wgn = 4 / wgm;
    dim3 grid((Ncol + 16 * WN * wgn - 1) / (16 * WN * wgn), (nwave_rows + wgm - 1) / wgm, js.n);
    const double *ac = blob_ptr(p, inverse ? p.lay.fz_inv_c : p.lay.fz_fwd_c);
    const double *as = blob_ptr(p, inverse ? p.lay.fz_inv_s : p.lay.fz_fwd_s);
    const double s0 = 1.0 / std::sqrt((double)N), s1 = std::sqrt(2.0 / (double)N);
    if (inverse)
        hipLaunchKernelGGL((zfold_f64_kernel<WM, WN, true, PF>), grid, dim3(256), 0, s, js, N, p.nx, ac, as,
                           wgn, s0, s1);
    else
        hipLaunchKernelGGL((zfold_f64_kernel<WM, WN, false, PF>), grid, dim3(256), 0, s, js, N, p.nx, ac,
                           as, wgn, s0, s1);
    return hipGetLastError();
}

#define IBS_FOLD_CASE(F, T, c) \
    case c: return F<T##_WM[c], T##_WN[c], F_PF[c]>(js, p, inverse, s);

hipError_t launch_xfold_f64(const JobSet &js, const Plan &p, bool inverse, hipStream_t s)
{
    switch (p.tune[TUNE_XFOLD] < 0 ? 0 : p.tune[TUNE_XFOLD]) {
        IBS_FOLD_CASE(xfold_launch, XF, 0) IBS_FOLD_CASE(xfold_launch, XF, 1)
        IBS_FOLD_CASE(xfold_launch, XF, 2) IBS_FOLD_CASE(xfold_launch, XF, 3)
        IBS_FOLD_CASE(xfold_launch, XF, 4) IBS_FOLD_CASE(xfold_launch, XF, 5)
        IBS_FOLD_CASE(xfold_launch, XF, 6) IBS_FOLD_CASE(xfold_launch, XF, 7)
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_zfold_f64(const JobSet &js, const Plan &p, bool inverse, hipStream_t s)
{
    switch (p.tune[TUNE_ZFOLD] < 0 ? 0 : p.tune[TUNE_ZFOLD]) {
        IBS_FOLD_CASE(zfold_launch, ZF, 0) IBS_FOLD_CASE(zfold_launch, ZF, 1)
        IBS_FOLD_CASE(zfold_launch, ZF, 2) IBS_FOLD_CASE(zfold_launch, ZF, 3)
        IBS_FOLD_CASE(zfold_launch, ZF, 4) IBS_FOLD_CASE(zfold_launch, ZF, 5)
        IBS_FOLD_CASE(zfold_launch, ZF, 6) IBS_FOLD_CASE(zfold_launch, ZF, 7)
    default: return hipErrorInvalidValue;
    }
}
#undef IBS_FOLD_CASE

}  // namespace ibs
