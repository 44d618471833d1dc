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

#include <algorithm>
#include <type_traits>

namespace ibs {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 b8 __attribute__((ext_vector_type(8)));
typedef float fv8 __attribute__((ext_vector_type(8)));
typedef double dv4 __attribute__((ext_vector_type(4)));

// Inverse x transform epilogues.  MODE 1 stores the iterate x = C (FP64);
// MODE 3 stores it in FP32 in the job's stored-iterate field xs (the first
// pass of a multi-pass solve: its result is only FP32-accurate, and the next
// pass rewrites x); MODE 2 updates x += C from the FP64 x; MODE 4 writes
// x = xs + C from the FP32 xs.  Modes 2 and 4 also sum C^2 and x^2.
template <int MODE> struct XStore {
    static constexpr bool store = MODE == 1 || MODE == 3;
    static constexpr bool update = MODE == 2 || MODE == 4;
    // the skipped wall rows are zeroed by the first pass: in x (MODE 1), or
    // in both xs and x (MODE 3; MODE 4 then writes the transform rows only)
    static constexpr bool zero_walls = MODE == 1 || MODE == 3;
    typedef typename std::conditional<MODE >= 3, float, double>::type T;   // stored iterate
};
template <int MODE>
static __device__ __forceinline__ typename XStore<MODE>::T *stored_iterate(const SplitJob &jb)
{
    if constexpr (MODE >= 3) return static_cast<float *>(jb.xs);
    else return jb.x;
}
// where the epilogue writes: xs for MODE 3, x otherwise
template <int MODE>
static __device__ __forceinline__ typename std::conditional<MODE == 3, float, double>::type *
xdest(const SplitJob &jb)
{
    if constexpr (MODE == 3) return static_cast<float *>(jb.xs);
    else return jb.x;
}

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

// The six partial products of a three-term split, small ones first.
static constexpr int TA_[6] = {2, 0, 1, 1, 0, 0};
static constexpr int TB_[6] = {0, 2, 1, 0, 1, 0};

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

// ---------------------------------------------------------------------------
// Transform kernels.  Both keep the streamed field in registers: every data
// element is loaded from HBM and split by exactly one wave.  The transform
// matrix is shared: per 32-deep K chunk, the workgroup copies the chunk of
// the pre-split, pre-swizzled matrix (NBT 16-blocks x 3 terms x 64 lanes x
// 16 bytes) into LDS (double-buffered when it fits), and every wave reads
// its fragments from there.  The next chunk's matrix and data are loaded
// while the current chunk is multiplied.
// ---------------------------------------------------------------------------

// Copy `cnt` 16-byte fragments (global, contiguous; cnt a multiple of 64)
// straight into LDS: each wave issues whole 64-fragment slices, lane l's
// fragment landing at slice + 16 l bytes (checked on gfx950).  Completion is
// awaited with s_waitcnt vmcnt before the barrier that publishes the data.
static __device__ __forceinline__ void q_dma(const b8 *__restrict__ src, b8 *dst, int cnt)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int base = wave * 64; base < cnt; base += 512)
        __builtin_amdgcn_global_load_lds(static_cast<const void *>(src + base + lane),
                                         (__attribute__((address_space(3))) void *)(dst + base), 16, 0, 0);
}
static __device__ __forceinline__ void wait_vm() { __builtin_amdgcn_s_waitcnt(0); }

// The refinement updates write their partial sums (sum of d^2, sum of x^2)
// per wave: slot (block slot * UPD_WAVES + wave), no LDS reduction.
constexpr int UPD_WAVES = 8;

// Copy `cnt` 16-byte fragments (global, contiguous) into registers / LDS.
template <int PER>
static __device__ __forceinline__ void q_load(const b8 *__restrict__ src, int cnt, b8 (&r)[PER])
{
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int idx = threadIdx.x + u * 512;
        if (idx < cnt) r[u] = src[idx];
    }
}
template <int PER>
static __device__ __forceinline__ void q_store(b8 *__restrict__ dst, int cnt, const b8 (&r)[PER])
{
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int idx = threadIdx.x + u * 512;
        if (idx < cnt) dst[idx] = r[u];
    }
}

// x transform: C = A B, A = the field's rows (M = nz*rows, K = nx), B the
// split swizzled nx x nx matrix.  A wave owns WM row blocks (16 rows each)
// and all N = 16 NB columns (NB <= NBT).  MODE 0: FP32 out; MODE 1..4 as
// in XStore (per-block sums of C^2 and x^2 into red for the updates).
template <int NBT, int WM, typename Tin, int MODE>
__global__ __launch_bounds__(512) void split_xgemm_kernel(SplitSet ss, int nz, int K, int N,
                                                          const b8 *__restrict__ qs,
                                                          double *__restrict__ red,
                                                          const int *__restrict__ skip,
                                                          const double *__restrict__ scale)
{
    constexpr int QCNT = NBT * 3 * 64;                // fragments per chunk
    constexpr bool DB = 2 * QCNT * 16 <= 144 * 1024;  // double buffer if it fits
    constexpr int QPER = (QCNT + 511) / 512;
    __shared__ b8 sq[(DB ? 2 : 1) * QCNT];
    if (skip && skip[blockIdx.z]) return;   // this job has already converged
    const SplitJob &jb = ss.j[blockIdx.z];
    // update modes: the residual was stored scaled by sigma (a power of
    // two), so the correction is scaled back exactly
    const double isg = (XStore<MODE>::update && scale) ? 1.0 / scale[blockIdx.z] : 1.0;
    // the job's own matrix when the jobs' x operators differ (walls in x)
    const b8 *__restrict__ qj = jb.xq ? static_cast<const b8 *>(jb.xq) : qs;
    const int rskip = skip_first_row(jb.kind), trows = jb.rows - rskip;
    const int M = nz * trows;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lg = lane >> 4;
    const int NB = N >> 4;
    const int qcnt = NB * 3 * 64;
    const int row0 = (blockIdx.x * 8 + wave) * (16 * WM);
    const int nrb = row0 < M ? min(WM, (M - row0) >> 4) : 0;
    const Tin *__restrict__ A = static_cast<const Tin *>(jb.in);
    const int KC = K >> 5;

    f4 acc[WM][NBT];
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < NBT; ++j) acc[i][j] = (f4){0.f, 0.f, 0.f, 0.f};

    float dcur[WM][8], dnext[WM][8];
    auto load_data = [&](int kc, float (&d)[WM][8]) {
#pragma unroll
        for (int i = 0; i < WM; ++i) {
            if (i < nrb) {
                load8<Tin>(A + phys_row(row0 + 16 * i + li, trows, rskip) * K + 32 * kc + 8 * lg, d[i]);
            } else {
#pragma unroll
                for (int e = 0; e < 8; ++e) d[i][e] = 0.f;
            }
        }
    };
    b8 qreg[QPER];
    q_load<QPER>(qj, qcnt, qreg);
    q_store<QPER>(sq, qcnt, qreg);
    load_data(0, dcur);
    for (int kc = 0; kc < KC; ++kc) {
        __syncthreads();
        const b8 *cur = sq + (DB ? (kc & 1) * QCNT : 0);
        const bool more = kc + 1 < KC;
        if (more) {
            q_load<QPER>(qj + (size_t)(kc + 1) * qcnt, qcnt, qreg);
            load_data(kc + 1, dnext);
        }
        b8 a[WM][3];
#pragma unroll
        for (int i = 0; i < WM; ++i) split8(dcur[i], a[i]);
        if (nrb > 0) {
            // groups of G column blocks: the six term products are the outer
            // loop, so consecutive MFMAs update G*WM independent accumulators
            // (blocks beyond NB read unused LDS and are never stored)
            constexpr int G = (NBT >= 4 && WM == 1) ? 4 : 2;
#pragma unroll
            for (int jg = 0; jg < NBT; jg += G) {
                b8 b[G][3];
#pragma unroll
                for (int jj = 0; jj < G; ++jj)
#pragma unroll
                    for (int t = 0; t < 3; ++t) b[jj][t] = cur[((jg + jj) * 3 + t) * 64 + lane];
#pragma unroll
                for (int pr = 0; pr < 6; ++pr)
#pragma unroll
                    for (int jj = 0; jj < G; ++jj)
#pragma unroll
                        for (int i = 0; i < WM; ++i)
                            acc[i][jg + jj] = mma(a[i][TA_[pr]], b[jj][TB_[pr]], acc[i][jg + jj]);
            }
        }
        if (more) {
            if (!DB) __syncthreads();
            q_store<QPER>(sq + (DB ? ((kc + 1) & 1) * QCNT : 0), qcnt, qreg);
#pragma unroll
            for (int i = 0; i < WM; ++i)
#pragma unroll
                for (int e = 0; e < 8; ++e) dcur[i][e] = dnext[i][e];
        }
    }
    double sd = 0.0, sx = 0.0;
#pragma unroll
    for (int i = 0; i < WM; ++i) {
        if (i < nrb) {
            size_t orow[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int t = row0 + 16 * i + 4 * lg + q;
                orow[q] = phys_row(t, trows, rskip) * N;
                // the skipped wall row before each plane's first transform
                // row holds zeros in the result
                if constexpr (MODE != 0 && XStore<MODE>::zero_walls)
                    if (rskip && t % trows == 0)
                        for (int c = li; c < N; c += 16) {
                            xdest<MODE>(jb)[orow[q] - N + c] = 0;
                            if (MODE == 3) jb.x[orow[q] - N + c] = 0.0;
                        }
            }
#pragma unroll
            for (int j = 0; j < NBT; ++j) {
                if (j < NB) {
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const size_t o = orow[q] + 16 * j + li;
                        if constexpr (MODE == 0) {
                            jb.out[o] = acc[i][j][q];
                        } else if constexpr (XStore<MODE>::store) {
                            xdest<MODE>(jb)[o] = acc[i][j][q];
                        } else {
                            // the correction of the sigma-scaled residual, unscaled
                            const double d = (double)acc[i][j][q] * isg;
                            const double xn = (double)stored_iterate<MODE>(jb)[o] + d;
                            jb.x[o] = xn;
                            sd += d * d;
                            sx += xn * xn;
                        }
                    }
                }
            }
        }
    }
    if (MODE == 2 || MODE == 4) {
        sd = wave_sum(sd);
        sx = wave_sum(sx);
        if (lane == 0) {
            const size_t slot = ((size_t)blockIdx.z * gridDim.x + blockIdx.x) * UPD_WAVES + wave;
            red[2 * slot] = sd;
            red[2 * slot + 1] = sx;
        }
    }
}

// z transform: C = A B, A the split swizzled nz x nz matrix (M = K = nz =
// 16 MB, MB <= MBT), B the field viewed as nz x (rows*nx), FP32 in and out.
// A wave owns all M rows and WN column blocks (16 columns each).
template <int MBT, int WN>
__global__ __launch_bounds__(512) void split_zgemm_kernel(SplitSet ss, int M, int K, int nx,
                                                          const b8 *__restrict__ qs,
                                                          const int *__restrict__ skip)
{
    constexpr int QCNT = MBT * 3 * 64;
    constexpr bool DB = 2 * QCNT * 16 <= 144 * 1024;
    constexpr int QPER = (QCNT + 511) / 512;
    __shared__ b8 sq[(DB ? 2 : 1) * QCNT];
    if (skip && skip[blockIdx.z]) return;
    const SplitJob &jb = ss.j[blockIdx.z];
    // the job's own matrix when the jobs' z operators differ (walls in z)
    const b8 *__restrict__ qj = jb.zq ? static_cast<const b8 *>(jb.zq) : qs;
    const int rskip = skip_first_row(jb.kind);
    const int Ncol = (jb.rows - rskip) * nx;
    const size_t ldp = (size_t)jb.rows * nx;   // plane stride
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lg = lane >> 4;
    const int MB = M >> 4;
    const int qcnt = MB * 3 * 64;
    const int col0 = (blockIdx.x * 8 + wave) * (16 * WN);
    const int ncb = col0 < Ncol ? min(WN, (Ncol - col0) >> 4) : 0;
    const float *__restrict__ B = static_cast<const float *>(jb.in) + rskip * nx;
    float *__restrict__ C = jb.out + rskip * nx;
    const int KC = K >> 5;

    f4 acc[MBT][WN];
#pragma unroll
    for (int i = 0; i < MBT; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j) acc[i][j] = (f4){0.f, 0.f, 0.f, 0.f};

    float dcur[WN][8], dnext[WN][8];
    auto load_data = [&](int kc, float (&d)[WN][8]) {
        const float *brow = B + (size_t)(32 * kc + 8 * lg) * ldp + col0 + li;
#pragma unroll
        for (int j = 0; j < WN; ++j)
#pragma unroll
            for (int e = 0; e < 8; ++e) d[j][e] = (j < ncb) ? brow[(size_t)e * ldp + 16 * j] : 0.f;
    };
    b8 qreg[QPER];
    q_load<QPER>(qj, qcnt, qreg);
    q_store<QPER>(sq, qcnt, qreg);
    load_data(0, dcur);
    for (int kc = 0; kc < KC; ++kc) {
        __syncthreads();
        const b8 *cur = sq + (DB ? (kc & 1) * QCNT : 0);
        const bool more = kc + 1 < KC;
        if (more) {
            q_load<QPER>(qj + (size_t)(kc + 1) * qcnt, qcnt, qreg);
            load_data(kc + 1, dnext);
        }
        b8 b[WN][3];
#pragma unroll
        for (int j = 0; j < WN; ++j) split8(dcur[j], b[j]);
        if (ncb > 0) {
            constexpr int G = (MBT >= 4 && WN == 1) ? 4 : 2;
#pragma unroll
            for (int ig = 0; ig < MBT; ig += G) {
                b8 a[G][3];
#pragma unroll
                for (int ii = 0; ii < G; ++ii)
#pragma unroll
                    for (int t = 0; t < 3; ++t) a[ii][t] = cur[((ig + ii) * 3 + t) * 64 + lane];
#pragma unroll
                for (int pr = 0; pr < 6; ++pr)
#pragma unroll
                    for (int ii = 0; ii < G; ++ii)
#pragma unroll
                        for (int j = 0; j < WN; ++j)
                            acc[ig + ii][j] = mma(a[ii][TA_[pr]], b[j][TB_[pr]], acc[ig + ii][j]);
            }
        }
        if (more) {
            if (!DB) __syncthreads();
            q_store<QPER>(sq + (DB ? ((kc + 1) & 1) * QCNT : 0), qcnt, qreg);
#pragma unroll
            for (int j = 0; j < WN; ++j)
#pragma unroll
                for (int e = 0; e < 8; ++e) dcur[j][e] = dnext[j][e];
        }
    }
#pragma unroll
    for (int i = 0; i < MBT; ++i) {
        if (i < MB) {
#pragma unroll
            for (int j = 0; j < WN; ++j) {
                if (j < ncb) {
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        C[(size_t)(16 * i + 4 * lg + q) * ldp + col0 + 16 * j + li] = acc[i][j][q];
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Folded transforms (n % 64 == 0).  The real Fourier basis is even or odd
// under i -> n - i, so a length-n transform is two half-length products:
//   forward: E[i] = X[i] + X[n-i], O[i] = X[i] - X[n-i] (E[0] = X[0],
//            O[0] = X[H]); cos outputs = E Fc (+ X[H] Q[H][a]), sin and
//            Nyquist outputs = O Fs (+ the alternating sum of E at H)
//   inverse: U = Xc Fc (+ X[H] Q[i][H]), V = Xs Fs; X[i] = U + V,
//            X[n-i] = U - V, X[H] = the alternating sum of Xc (+ X[H] Q[H][H])
// (H = n/2).  Half the matrix-core work of the plain transform; the four
// self-mirrored points are handled on the vector units.  The chunk of both
// factors (2 x HB 16-blocks x 3 terms) is staged through LDS as above.
// ---------------------------------------------------------------------------

// x transform, a wave owning WM row blocks and all columns of both factors.
// MODE as for the plain kernel (0: FP32 out, forward; 1..4 as in XStore).
// Persistent like the z kernel: block b takes row tiles b, b + G, ... over
// the jobs still running as one pipeline of 32-deep chunks.  MODE 2 writes
// the update sums of tile rt of job q to slot q * tiles_per_job + rt.
template <int HBT, int WM, typename Tin, int MODE, bool INV, int FS>
__global__ __launch_bounds__(512) void split_xfold_kernel(SplitSet ss, int nz, int N,
                                                          const b8 *__restrict__ qs,
                                                          double *__restrict__ red,
                                                          const int *__restrict__ skip, double s0,
                                                          double s1, int tiles_per_job,
                                                          const double *__restrict__ scale)
{
    // FS = 1: a pipeline step is one 32-deep chunk of both factors; FS = 2
    // (large n): one factor at a time, so a double-buffered step fits LDS
    constexpr int QCNT = (FS == 1 ? 2 : 1) * HBT * 3 * 64;
    static_assert(2 * QCNT * 16 <= 144 * 1024, "double-buffered factor chunk must fit LDS");
    __shared__ b8 sq[2 * QCNT];
    // jobs not yet converged (block-uniform), packed 8 bits each so that no
    // private array is indexed at run time
    int live = 0, nlive = 0;
    for (int q = 0; q < ss.n; ++q)
        if (!(skip && skip[q])) live |= q << (8 * nlive++);
    const int ntiles = nlive * tiles_per_job;
    const int G = gridDim.x;
    const int my_tiles = (int)blockIdx.x < ntiles ? (ntiles - 1 - (int)blockIdx.x) / G + 1 : 0;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lg = lane >> 4;
    const int H = N >> 1, HB = H >> 4;
    const int qcnt = (FS == 1 ? 2 : 1) * HB * 3 * 64;
    const int KC = H >> 5;
    const int nsteps = my_tiles * KC * FS;
    const double sH = (H & 1) ? -s0 : s0;

    struct TileRef { int job, rt, rskip, trows, row0, nrb; const SplitJob *jb; };
    auto tile_ref = [&](int i) {
        const int t = (int)blockIdx.x + i * G;
        TileRef r;
        r.job = (live >> (8 * (t / tiles_per_job))) & 0xff;
        r.rt = t % tiles_per_job;
        r.jb = &ss.j[r.job];
        r.rskip = skip_first_row(r.jb->kind);
        r.trows = r.jb->rows - r.rskip;
        const int M = nz * r.trows;
        r.row0 = (r.rt * 8 + wave) * (16 * WM);
        r.nrb = r.row0 < M ? min(WM, (M - r.row0) >> 4) : 0;
        return r;
    };

    f4 acc[WM][2][HBT];
    double nyq[WM];
    auto clear = [&]() {
#pragma unroll
        for (int i = 0; i < WM; ++i) {
            nyq[i] = 0.0;
#pragma unroll
            for (int f = 0; f < 2; ++f)
#pragma unroll
                for (int j = 0; j < HBT; ++j) acc[i][f][j] = (f4){0.f, 0.f, 0.f, 0.f};
        }
    };
    // forward: p = X[k], m = X[mirror k]; inverse: p = cos inputs, m = sin
    // inputs.  The next chunk is loaded, raw, into the same registers once
    // the current one has been split; nothing reads them before the step's
    // closing wait, so the loads run under the products.
    Tin rp[WM][8], rm[WM][8], rxh[WM];
    auto load_data = [&](int chunk) {   // chunk = tile * KC + kc
        const TileRef r = tile_ref(chunk / KC);
        const Tin *A = static_cast<const Tin *>(r.jb->in);
        const int k0 = 32 * (chunk % KC) + 8 * lg;
#pragma unroll
        for (int i = 0; i < WM; ++i) {
            if (i < r.nrb) {   // wave-uniform
                const Tin *arow = A + phys_row(r.row0 + 16 * i + li, r.trows, r.rskip) * N;
                __builtin_memcpy(rp[i], arow + k0, sizeof(rp[i]));
                if (!INV) {
                    // mirrored points N - kk (kk = k0 .. k0+7) as one 8-wide
                    // run, reversed at the split; kk = 0 pairs with point H
                    // instead, so lanes with k0 = 0 read the run N-8 .. N-1
                    __builtin_memcpy(rm[i], arow + (k0 == 0 ? N - 8 : N - k0 - 7), sizeof(rm[i]));
                    if (chunk % KC == 0) rxh[i] = arow[H];   // wave-uniform: once per tile
                } else {
                    __builtin_memcpy(rm[i], arow + H + k0, sizeof(rm[i]));
                }
            } else {
#pragma unroll
                for (int e = 0; e < 8; ++e) { rp[i][e] = 0; rm[i][e] = 0; }
                rxh[i] = 0;
            }
        }
    };
    if (nsteps == 0) return;
    clear();
    q_dma(qs, sq, qcnt);
    load_data(0);
    wait_vm();
    b8 ae[WM][3], ao[WM][3];   // split E and O of the current chunk
    // X[H] of the tile's output rows (and, inverse, of rows li), loaded at
    // the start of the tile's last step so that the epilogue does not wait
    Tin ahp[WM][4], xhp[WM];
    typename XStore<MODE>::T xhold[WM];   // update modes: old iterate at point H of rows li
    // one chunk per iteration; its FS steps unrolled, so that the factor
    // of a step is known at compile time and the data loads of a chunk go
    // straight into the registers the next chunk reads
    for (int step0 = 0; step0 < nsteps; step0 += FS) {
#pragma unroll
        for (int f = 0; f < FS; ++f) {   // f: factor of this step (FS = 2)
        const int step = step0 + f, chunk = step / FS;
        const int kc = chunk % KC;
        const bool last = kc == KC - 1 && f == FS - 1;   // the tile completes this step
        __syncthreads();
        const b8 *cur = sq + (step & 1) * QCNT;
        const bool more = step + 1 < nsteps;
        // the next step's factors go to the other LDS buffer, at the step
        // start (the copy runs under the products).  No other LDS object
        // or barrier may appear in the loop: with one, the compiler made the
        // products' LDS reads wait for this copy (and, the memory counter
        // being in order, for the data loads after it)
        if (more) q_dma(qs + (size_t)((step + 1) % (KC * FS)) * qcnt, sq + ((step + 1) & 1) * QCNT, qcnt);
        if (last) {
            const TileRef r = tile_ref(chunk / KC);
            const Tin *A = static_cast<const Tin *>(r.jb->in);
#pragma unroll
            for (int i = 0; i < WM; ++i) {
                if (i >= r.nrb) continue;   // wave-uniform
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    ahp[i][q] = A[phys_row(r.row0 + 16 * i + 4 * lg + q, r.trows, r.rskip) * N + H];
                if (INV) xhp[i] = A[phys_row(r.row0 + 16 * i + li, r.trows, r.rskip) * N + H];
                if constexpr (XStore<MODE>::update)
                    xhold[i] = stored_iterate<MODE>(*r.jb)[phys_row(r.row0 + 16 * i + li, r.trows, r.rskip) * N + H];
            }
        }
        const int k0 = 32 * kc + 8 * lg;
        if (f == 0) {
#pragma unroll
            for (int i = 0; i < WM; ++i) {
                float ev[8], ov[8], pc[8], mc[8];
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    pc[e] = (float)rp[i][e];
                    if (INV) mc[e] = (float)rm[i][e];
                    else if (k0 == 0) mc[e] = (float)(e == 0 ? rxh[i] : rm[i][8 - e]);
                    else mc[e] = (float)rm[i][7 - e];
                }
                if (!INV) {
#pragma unroll
                    for (int e = 0; e < 8; ++e) {
                        const bool self = k0 + e == 0;
                        ev[e] = self ? pc[e] : pc[e] + mc[e];
                        ov[e] = self ? mc[e] : pc[e] - mc[e];
                        nyq[i] += (e & 1) ? -(double)ev[e] : (double)ev[e];
                    }
                } else {
#pragma unroll
                    for (int e = 0; e < 8; ++e) {
                        ev[e] = pc[e];
                        ov[e] = mc[e];
                        const double w = (k0 + e == 0) ? s0 : s1;
                        nyq[i] += (e & 1) ? -w * (double)ev[e] : w * (double)ev[e];
                    }
                }
                split8(ev, ae[i]);
                split8(ov, ao[i]);
            }
            if (chunk + 1 < my_tiles * KC) load_data(chunk + 1);
        }
        {
            constexpr int GR = (HBT >= 6 || WM >= 2) ? 1 : 2;   // register budget
#pragma unroll
            for (int jg = 0; jg < HBT; jg += GR) {
                if (FS == 1) {
                    b8 bc[GR][3], bs[GR][3];
#pragma unroll
                    for (int jj = 0; jj < GR; ++jj)
#pragma unroll
                        for (int t = 0; t < 3; ++t) {
                            bc[jj][t] = cur[((jg + jj) * 3 + t) * 64 + lane];
                            bs[jj][t] = cur[((HB + jg + jj) * 3 + t) * 64 + lane];
                        }
#pragma unroll
                    for (int pr = 0; pr < 6; ++pr)
#pragma unroll
                        for (int jj = 0; jj < GR; ++jj)
#pragma unroll
                            for (int i = 0; i < WM; ++i) {
                                acc[i][0][jg + jj] = mma(ae[i][TA_[pr]], bc[jj][TB_[pr]], acc[i][0][jg + jj]);
                                acc[i][1][jg + jj] = mma(ao[i][TA_[pr]], bs[jj][TB_[pr]], acc[i][1][jg + jj]);
                            }
                } else {
                    // one factor per step: cos (E) on even steps, sin (O) on odd
                    b8 bf[GR][3];
#pragma unroll
                    for (int jj = 0; jj < GR; ++jj)
#pragma unroll
                        for (int t = 0; t < 3; ++t) bf[jj][t] = cur[((jg + jj) * 3 + t) * 64 + lane];
                    if (f == 0) {
#pragma unroll
                        for (int pr = 0; pr < 6; ++pr)
#pragma unroll
                            for (int jj = 0; jj < GR; ++jj)
#pragma unroll
                                for (int i = 0; i < WM; ++i)
                                    acc[i][0][jg + jj] = mma(ae[i][TA_[pr]], bf[jj][TB_[pr]], acc[i][0][jg + jj]);
                    } else {
#pragma unroll
                        for (int pr = 0; pr < 6; ++pr)
#pragma unroll
                            for (int jj = 0; jj < GR; ++jj)
#pragma unroll
                                for (int i = 0; i < WM; ++i)
                                    acc[i][1][jg + jj] = mma(ao[i][TA_[pr]], bf[jj][TB_[pr]], acc[i][1][jg + jj]);
                    }
                }
            }
        }
        // next step's factors and data, and this tile's X[H] values, have
        // landed (the epilogue's stores below are left in flight)
        if (more || last) wait_vm();
        if (last) {   // the tile is complete: store it
            const TileRef r = tile_ref(chunk / KC);
            const SplitJob &jb = *r.jb;
            // update modes: the residual was stored scaled by sigma (a power
            // of two), so the correction is scaled back exactly
            const double isg = (XStore<MODE>::update && scale) ? 1.0 / scale[r.job] : 1.0;
            double sd = 0.0, sx = 0.0;
#pragma unroll
            for (int i = 0; i < WM; ++i) {
                if (i >= r.nrb) continue;
                double ny = nyq[i];
                ny += __shfl_xor(ny, 16, 64);
                ny += __shfl_xor(ny, 32, 64);   // every lane of row li holds its sum
                size_t orow[4];
                double ah[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int t = r.row0 + 16 * i + 4 * lg + q;
                    orow[q] = phys_row(t, r.trows, r.rskip) * N;
                    ah[q] = (double)ahp[i][q];   // X[H] of the output row
                    // the skipped wall row before each plane's first row
                    // holds zeros in the result
                    if constexpr (MODE != 0 && XStore<MODE>::zero_walls)
                        if (r.rskip && t % r.trows == 0)
                            for (int c = li; c < N; c += 16) {
                                xdest<MODE>(jb)[orow[q] - N + c] = 0;
                                if (MODE == 3) jb.x[orow[q] - N + c] = 0.0;
                            }
                }
                if (!INV) {
                    double nyr[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) nyr[q] = __shfl(ny, 4 * lg + q, 64);
#pragma unroll
                    for (int j = 0; j < HBT; ++j) {
                        if (j >= HB) continue;
                        const int a = 16 * j + li;
                        const double wa = (a == 0 ? s0 : s1) * ((a & 1) ? -1.0 : 1.0);   // Q[H][a]
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            jb.out[orow[q] + a] = (float)fma(ah[q], wa, (double)acc[i][0][j][q]);
                            double sv = (double)acc[i][1][j][q];
                            if (a == 0) sv = fma(s0, nyr[q], sv);   // spectral index H
                            jb.out[orow[q] + H + a] = (float)sv;
                        }
                    }
                } else {
                    // destination and stored iterate held in registers: the
                    // job record is not reloaded after each store
                    auto *const xd = xdest<MODE>(jb);
                    const auto *const xold = stored_iterate<MODE>(jb);
                    if (lg == 0) {   // physical point H of row li
                        const size_t rr = phys_row(r.row0 + 16 * i + li, r.trows, r.rskip) * N;
                        const double xh = fma((double)xhp[i], sH, ny);
                        if constexpr (XStore<MODE>::store) {
                            xd[rr + H] = xh;
                        } else {
                            const double dh = xh * isg, xn = (double)xhold[i] + dh;
                            xd[rr + H] = xn;
                            sd += dh * dh;
                            sx += xn * xn;
                        }
                    }
                    // the rows' old values first, eight column blocks and (an
                    // FP32 iterate) all four rows at a time (all loads in
                    // flight together; every position is distinct), then the
                    // updates
                    typedef typename XStore<MODE>::T Tx;   // kept in its stored type
                    constexpr int JG = HBT < 8 ? HBT : 8;
                    constexpr int QG = (XStore<MODE>::update && sizeof(Tx) == 4 && HBT <= 8) ? 4 : 1;
#pragma unroll
                    for (int q0 = 0; q0 < 4; q0 += QG) {
#pragma unroll
                        for (int j0 = 0; j0 < HBT; j0 += JG) {
                            Tx xo[QG][2][JG];
                            if constexpr (XStore<MODE>::update) {
                                // a position the row lacks is neither read
                                // nor used (its store below is skipped too)
#pragma unroll
                                for (int qq = 0; qq < QG; ++qq)
#pragma unroll
                                    for (int jj = 0; jj < JG; ++jj) {
                                        const int ii = 16 * (j0 + jj) + li;
                                        const bool ok = j0 + jj < HB;
                                        if (ok) xo[qq][0][jj] = xold[orow[q0 + qq] + ii];
                                        if (ok && ii != 0) xo[qq][1][jj] = xold[orow[q0 + qq] + N - ii];
                                    }
                                // all of them have landed before the first
                                // store (else each later use would wait on
                                // the stores issued meanwhile)
                                wait_vm();
                            }
#pragma unroll
                            for (int qq = 0; qq < QG; ++qq) {
                                const int q = q0 + qq;
#pragma unroll
                                for (int jj = 0; jj < JG; ++jj) {
                                    const int j = j0 + jj;
                                    if (j >= HB) continue;
                                    const int ii = 16 * j + li;
                                    const double sg = (ii & 1) ? -s0 : s0;   // Q[ii][H]
                                    const double u = fma(ah[q], sg, (double)acc[i][0][j][q]);
                                    const double v = (double)acc[i][1][j][q];
                                    const size_t o1 = orow[q] + ii, o2 = orow[q] + N - ii;
                                    if constexpr (XStore<MODE>::store) {
                                        xd[o1] = u + v;
                                        if (ii != 0) xd[o2] = u - v;
                                    } else {
                                        const double d1 = (u + v) * isg, x1 = xo[qq][0][jj] + d1;
                                        xd[o1] = x1;
                                        sd += d1 * d1;
                                        sx += x1 * x1;
                                        if (ii != 0) {
                                            const double d2 = (u - v) * isg, x2 = xo[qq][1][jj] + d2;
                                            xd[o2] = x2;
                                            sd += d2 * d2;
                                            sx += x2 * x2;
                                        }
                                    }
                                }
                            }
                        }
                    }
                }
            }
            if (XStore<MODE>::update) {
                sd = wave_sum(sd);
                sx = wave_sum(sx);
                if (lane == 0) {
                    const size_t slot = ((size_t)r.job * tiles_per_job + r.rt) * UPD_WAVES + wave;
                    red[2 * slot] = sd;
                    red[2 * slot + 1] = sx;
                }
            }
            clear();
        }
        }
    }
}

// z transform, a wave owning all output rows of both factors and WN
// column blocks; FP32 in and out.  Persistent: block b takes column tiles
// b, b + G, ... (G = gridDim.x) over the jobs still running, and streams
// their 32-deep chunks as one pipeline, so the next tile's first chunk is
// loaded while the current tile's last chunk is multiplied.
template <int HBT, int WN, bool INV, int FS>
__global__ __launch_bounds__(512) void split_zfold_kernel(SplitSet ss, int N, int nx,
                                                          const b8 *__restrict__ qs,
                                                          const int *__restrict__ skip, double s0,
                                                          double s1, int tiles_per_job)
{
    // FS = 1: a pipeline step is one 32-deep chunk of both factors; FS = 2
    // (large n): one factor at a time, so a double-buffered step fits LDS
    constexpr int QCNT = (FS == 1 ? 2 : 1) * HBT * 3 * 64;
    static_assert(2 * QCNT * 16 <= 144 * 1024, "double-buffered factor chunk must fit LDS");
    __shared__ b8 sq[2 * QCNT];
    // jobs not yet converged (block-uniform), packed 8 bits each so that no
    // private array is indexed at run time
    int live = 0, nlive = 0;
    for (int q = 0; q < ss.n; ++q)
        if (!(skip && skip[q])) live |= q << (8 * nlive++);
    const int ntiles = nlive * tiles_per_job;
    const int G = gridDim.x;
    const int my_tiles = (int)blockIdx.x < ntiles ? (ntiles - 1 - (int)blockIdx.x) / G + 1 : 0;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lg = lane >> 4;
    const int H = N >> 1, HB = H >> 4;
    const int qcnt = (FS == 1 ? 2 : 1) * HB * 3 * 64;
    const int KC = H >> 5;
    const int nsteps = my_tiles * KC * FS;
    const double sH = (H & 1) ? -s0 : s0;

    // tile -> job record and this wave's first column
    struct TileRef { const SplitJob *jb; int rskip, Ncol, col0, ncb; size_t ldp; };
    auto tile_ref = [&](int i) {
        const int t = (int)blockIdx.x + i * G;
        TileRef r;
        r.jb = &ss.j[(live >> (8 * (t / tiles_per_job))) & 0xff];
        r.rskip = skip_first_row(r.jb->kind);
        r.Ncol = (r.jb->rows - r.rskip) * nx;
        r.ldp = (size_t)r.jb->rows * nx;
        r.col0 = ((t % tiles_per_job) * 8 + wave) * (16 * WN);
        r.ncb = r.col0 < r.Ncol ? min(WN, (r.Ncol - r.col0) >> 4) : 0;
        return r;
    };

    f4 acc[2][HBT][WN];
    double nyq[WN];
    auto clear = [&]() {
#pragma unroll
        for (int j = 0; j < WN; ++j) {
            nyq[j] = 0.0;
#pragma unroll
            for (int f = 0; f < 2; ++f)
#pragma unroll
                for (int i = 0; i < HBT; ++i) acc[f][i][j] = (f4){0.f, 0.f, 0.f, 0.f};
        }
    };
    float pc[WN][8], mc[WN][8];   // the chunk being split; then the next one
    auto load_data = [&](int chunk) {   // chunk = tile * KC + kc
        const TileRef r = tile_ref(chunk / KC);
        const int k0 = 32 * (chunk % KC) + 8 * lg;
        const float *B = static_cast<const float *>(r.jb->in) + r.rskip * nx;
#pragma unroll
        for (int j = 0; j < WN; ++j) {
            const float *col = B + r.col0 + 16 * j + li;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int kk = k0 + e;
                const bool ok = j < r.ncb;
                pc[j][e] = ok ? col[(size_t)kk * r.ldp] : 0.f;
                mc[j][e] = ok ? col[(size_t)(INV ? H + kk : (kk == 0 ? H : N - kk)) * r.ldp] : 0.f;
            }
        }
    };
    if (nsteps == 0) return;
    clear();
    q_dma(qs, sq, qcnt);
    load_data(0);
    wait_vm();
    b8 be[WN][3], bo[WN][3];   // split E and O of the current chunk
    float bhp[WN];   // plane H of the tile's columns, loaded at its last step
    // one chunk per iteration; its FS steps unrolled, so that the factor
    // of a step is known at compile time and the data loads of a chunk go
    // straight into the registers the next chunk reads
    for (int step0 = 0; step0 < nsteps; step0 += FS) {
#pragma unroll
        for (int f = 0; f < FS; ++f) {   // f: factor of this step (FS = 2)
        const int step = step0 + f, chunk = step / FS;
        const int kc = chunk % KC;
        const bool last = kc == KC - 1 && f == FS - 1;   // the tile completes this step
        __syncthreads();
        const b8 *cur = sq + (step & 1) * QCNT;
        const bool more = step + 1 < nsteps;
        // the next step's factors go to the other LDS buffer, at the step
        // start (the copy runs under the products)
        if (more) q_dma(qs + (size_t)((step + 1) % (KC * FS)) * qcnt, sq + ((step + 1) & 1) * QCNT, qcnt);
        if (last) {
            const TileRef r = tile_ref(chunk / KC);
            const float *B = static_cast<const float *>(r.jb->in) + r.rskip * nx;
#pragma unroll
            for (int j = 0; j < WN; ++j)
                if (j < r.ncb) bhp[j] = B[(size_t)H * r.ldp + r.col0 + 16 * j + li];   // wave-uniform
        }
        const int k0 = 32 * kc + 8 * lg;
        if (f == 0) {
#pragma unroll
            for (int j = 0; j < WN; ++j) {
                float ev[8], ov[8];
                if (!INV) {
#pragma unroll
                    for (int e = 0; e < 8; ++e) {
                        const bool self = k0 + e == 0;
                        ev[e] = self ? pc[j][e] : pc[j][e] + mc[j][e];
                        ov[e] = self ? mc[j][e] : pc[j][e] - mc[j][e];
                        nyq[j] += (e & 1) ? -(double)ev[e] : (double)ev[e];
                    }
                } else {
#pragma unroll
                    for (int e = 0; e < 8; ++e) {
                        ev[e] = pc[j][e];
                        ov[e] = mc[j][e];
                        const double w = (k0 + e == 0) ? s0 : s1;
                        nyq[j] += (e & 1) ? -w * (double)ev[e] : w * (double)ev[e];
                    }
                }
                split8(ev, be[j]);
                split8(ov, bo[j]);
            }
            if (chunk + 1 < my_tiles * KC) load_data(chunk + 1);
        }
        {
            constexpr int GR = HBT >= 6 ? 1 : 2;   // register budget
#pragma unroll
            for (int ig = 0; ig < HBT; ig += GR) {
                if (FS == 1) {
                    b8 ac[GR][3], as[GR][3];
#pragma unroll
                    for (int ii = 0; ii < GR; ++ii)
#pragma unroll
                        for (int t = 0; t < 3; ++t) {
                            ac[ii][t] = cur[((ig + ii) * 3 + t) * 64 + lane];
                            as[ii][t] = cur[((HB + ig + ii) * 3 + t) * 64 + lane];
                        }
#pragma unroll
                    for (int pr = 0; pr < 6; ++pr)
#pragma unroll
                        for (int ii = 0; ii < GR; ++ii)
#pragma unroll
                            for (int j = 0; j < WN; ++j) {
                                acc[0][ig + ii][j] = mma(ac[ii][TA_[pr]], be[j][TB_[pr]], acc[0][ig + ii][j]);
                                acc[1][ig + ii][j] = mma(as[ii][TA_[pr]], bo[j][TB_[pr]], acc[1][ig + ii][j]);
                            }
                } else {
                    // one factor per step: cos (E) on even steps, sin (O) on odd
                    b8 af[GR][3];
#pragma unroll
                    for (int ii = 0; ii < GR; ++ii)
#pragma unroll
                        for (int t = 0; t < 3; ++t) af[ii][t] = cur[((ig + ii) * 3 + t) * 64 + lane];
                    if (f == 0) {
#pragma unroll
                        for (int pr = 0; pr < 6; ++pr)
#pragma unroll
                            for (int ii = 0; ii < GR; ++ii)
#pragma unroll
                                for (int j = 0; j < WN; ++j)
                                    acc[0][ig + ii][j] = mma(af[ii][TA_[pr]], be[j][TB_[pr]], acc[0][ig + ii][j]);
                    } else {
#pragma unroll
                        for (int pr = 0; pr < 6; ++pr)
#pragma unroll
                            for (int ii = 0; ii < GR; ++ii)
#pragma unroll
                                for (int j = 0; j < WN; ++j)
                                    acc[1][ig + ii][j] = mma(af[ii][TA_[pr]], bo[j][TB_[pr]], acc[1][ig + ii][j]);
                    }
                }
            }
        }
        // next step's factors and data, and this tile's plane-H values, have
        // landed (the epilogue's stores below are left in flight)
        if (more || last) wait_vm();
        if (last) {   // the tile is complete: store it
            const TileRef r = tile_ref(chunk / KC);
            float *C = r.jb->out + r.rskip * nx;
#pragma unroll
            for (int j = 0; j < WN; ++j) {
                if (j >= r.ncb) continue;
                const size_t cc = (size_t)(r.col0 + 16 * j + li);
                double ny = nyq[j];
                ny += __shfl_xor(ny, 16, 64);
                ny += __shfl_xor(ny, 32, 64);   // every lane of column li holds its sum
                const double bh = (double)bhp[j];
                if (INV && lg == 0) C[(size_t)H * r.ldp + cc] = (float)fma(bh, sH, ny);
#pragma unroll
                for (int i = 0; i < HBT; ++i) {
                    if (i >= HB) continue;
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int rr = 16 * i + 4 * lg + q;   // 0 <= rr < H
                        if (!INV) {
                            const double wr = (rr == 0 ? s0 : s1) * ((rr & 1) ? -1.0 : 1.0);   // Q[H][rr]
                            C[(size_t)rr * r.ldp + cc] = (float)fma(bh, wr, (double)acc[0][i][j][q]);
                            double sv = (double)acc[1][i][j][q];
                            if (rr == 0) sv = fma(s0, ny, sv);   // plane H: Nyquist
                            C[(size_t)(H + rr) * r.ldp + cc] = (float)sv;
                        } else {
                            const double u = fma(bh, (rr & 1) ? -s0 : s0, (double)acc[0][i][j][q]);
                            const double v = (double)acc[1][i][j][q];
                            C[(size_t)rr * r.ldp + cc] = (float)(u + v);
                            if (rr != 0) C[(size_t)(N - rr) * r.ldp + cc] = (float)(u - v);
                        }
                    }
                }
            }
            clear();
        }
        }
    }
}

// FP32 residual r = b - A x of the stored iterate xs (FP64, or FP32 after
// the first pass; either way evaluated in FP64) with the 7-point stencils of
// Section 2.1.  For the pressure problem the weighted mean of b (recorded
// by the first pass) is subtracted first: that constant lies in the null
// space of every correction, and left in r its FP32 rounding would swamp the
// shrinking residual.  The same pass sums Delta_j x per block (fixed block
// layout and order), so the next correction can also remove the weighted
// mean that x has picked up from the FP32 transforms.
// A block owns RB whole rows (RB = 256 / (nx/4): a thread takes 4
// consecutive points of a row, a row's threads its whole width, so the x
// neighbours, periodic ones included, are in the row's own lines) of rz
// consecutive z planes and marches along z, keeping x at k-1, k, k+1 in
// registers (each x value is read from HBM about once; y neighbours come
// from the same or adjacent blocks' rows).  grid: (tiles per job, jobs),
// the same tile count for all jobs.
// ST: a stretched wall-bounded x and/or z (sgx / sgz the per-index
// geometry, StretchSlot layout, null for a uniform axis): the x and z rows
// take their per-index coefficients, and the weighted sums Delta_j x
// become W x with the cells' x and z shares of the volume weight.
template <typename Tx, bool ST>
__global__ __launch_bounds__(256) void residual_f32_kernel(SplitSet ss, int nx, int ny, int nz,
                                                           double ihx2, double ihz2,
                                                           const double *__restrict__ dyc,
                                                           const double *__restrict__ dyf,
                                                           const double *__restrict__ bmean,
                                                           double *__restrict__ xsum,
                                                           const int *__restrict__ skip, int rb_rows,
                                                           int tiles_y, int rz, int py, int wxw, int wzw,
                                                           const double *__restrict__ sgx,
                                                           const double *__restrict__ sgz,
                                                           const double *__restrict__ scale)
{
    typedef Tx tx4 __attribute__((ext_vector_type(4)));
    typedef double dv4_ __attribute__((ext_vector_type(4)));
    typedef float fv4 __attribute__((ext_vector_type(4)));
    const int job = blockIdx.y;
    if (skip && skip[job]) return;
    const SplitJob &jb = ss.j[job];
    const int op = jb.op, rows = jb.rows;
    const size_t plane = (size_t)rows * nx;
    const Tx *__restrict__ x = static_cast<const Tx *>(jb.xs);
    const double bm = (op == IBS_OP_POISSON) ? bmean[job] : 0.0;
    const double sg = scale[job];   // power of two: the stored residual is r sigma
    const int kz = blockIdx.x / tiles_y, ty = blockIdx.x - kz * tiles_y;
    const int k0 = kz * rz, k1 = min(nz, k0 + rz);
    const int tr = nx >> 2;                       // threads per row
    const int t = threadIdx.x % tr, rb = threadIdx.x / tr;
    const int j = ty * rb_rows + rb, i0 = 4 * t;
    double wx = 0.0;
    if (rb < rb_rows && j < rows) {
        const bool wall = !py && op == IBS_OP_HELMHOLTZ_V && (j == 0 || j == ny);
        const int iw = (i0 == 0) ? nx - 1 : i0 - 1, ie = (i0 + 4 == nx) ? 0 : i0 + 4;
        const size_t o = (size_t)j * nx;          // row start within a plane
        // y part in difference form, cu (x_up - x) - cl (x - x_lo); a missing
        // neighbour is the boundary ghost g x (g = 1 Neumann, -1 mirror, 0 wall)
        double D = 0.0, cu = 0.0, cl = 0.0, gu = 0.0, gl = 0.0;
        bool ru = false, rl = false;
        if (py) {
            // periodic y: interior formulas everywhere, neighbours wrapping
            // (delta_0 = delta_ny is the distance across the wrap)
            if (op != IBS_OP_HELMHOLTZ_V) {
                D = dyc[j];
                cu = 1.0 / (dyf[j + 1] * D);
                cl = 1.0 / (dyf[j] * D);
            } else {
                cu = 1.0 / (dyc[j] * dyf[j]);
                cl = 1.0 / (dyc[j == 0 ? ny - 1 : j - 1] * dyf[j]);
            }
            ru = true;
            rl = true;
        } else if (op != IBS_OP_HELMHOLTZ_V) {
            D = dyc[j];
            const double gb = (op == IBS_OP_POISSON) ? 1.0 : -1.0;
            ru = j + 1 < ny;
            cu = ru ? 1.0 / (dyf[j + 1] * D) : 1.0 / (D * D);
            gu = gb;
            rl = j > 0;
            cl = rl ? 1.0 / (dyf[j] * D) : 1.0 / (D * D);
            gl = gb;
        } else if (!wall) {
            cu = 1.0 / (dyc[j] * dyf[j]);
            cl = 1.0 / (dyc[j - 1] * dyf[j]);
            ru = j + 1 <= ny - 1;
            rl = j - 1 >= 1;
        }
        // branch-free body (every load unconditional and in range, a missing
        // neighbour reads the row itself), so unrolled iterations' loads can
        // all be in flight together
        // (periodic y: the neighbour of the last row is row 0, of row 0 the last)
        const int wrapoff = -(rows - 1) * nx;
        const int du = ru ? (py && j + 1 == rows ? wrapoff : nx) : 0;
        const int dl = rl ? (py && j == 0 ? wrapoff : nx) : 0;
        const double wu = ru ? 1.0 : gu, wl = rl ? 1.0 : gl;
        const bool pois = op == IBS_OP_POISSON;
        const double cj = jb.c;
        const double wD = (op != IBS_OP_HELMHOLTZ_V) ? D : 0.0;
        const double *__restrict__ bb = jb.b;
        float *__restrict__ rr = jb.r;
        // walls in x: the ghost beyond a wall is gx x (1 pressure, -1 v and
        // w, 0 u); u's slot 0 is the wall face itself (residual 0) and the
        // west neighbour of slot 1 that wall (0)
        const bool xw_u = wxw && op == IBS_OP_HELMHOLTZ_U;
        const double gx = pois ? 1.0 : (op == IBS_OP_HELMHOLTZ_U ? 0.0 : -1.0);
        // walls in z: the same along z, w the face-normal component
        const bool zw_w = wzw && op == IBS_OP_HELMHOLTZ_W;
        const double gz = pois ? 1.0 : (op == IBS_OP_HELMHOLTZ_W ? 0.0 : -1.0);
        auto ld4 = [&](size_t at) { return *reinterpret_cast<const tx4 *>(x + at); };
        // stretched: this thread's x coefficients and volume shares
        const int xkd = pois ? XK_P : (op == IBS_OP_HELMHOLTZ_U ? XK_F : XK_C);
        const int zkd = pois ? XK_P : (op == IBS_OP_HELMHOLTZ_W ? XK_F : XK_C);
        double aex[4], awx[4], wnx[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            aex[e] = awx[e] = ihx2;
            wnx[e] = 1.0;
            if constexpr (ST) {
                if (sgx) {
                    aex[e] = sgx[(size_t)sg_ae(xkd) * nx + i0 + e];
                    awx[e] = sgx[(size_t)sg_aw(xkd) * nx + i0 + e];
                    wnx[e] = sgx[(size_t)SG_WN * nx + i0 + e];
                }
            }
        }
        tx4 xm = ld4((size_t)(k0 == 0 ? nz - 1 : k0 - 1) * plane + o + i0);
        tx4 xc = ld4((size_t)k0 * plane + o + i0);
#pragma unroll 2
        for (int k = k0; k < k1; ++k) {
            const size_t c = (size_t)k * plane + o;   // this row of plane k
            const tx4 xp = ld4((size_t)(k + 1 == nz ? 0 : k + 1) * plane + o + i0);
            const tx4 xu = ld4((size_t)((ptrdiff_t)c + du + i0)), xl = ld4((size_t)((ptrdiff_t)c - dl + i0));
            const double xwe = (double)x[c + iw], xee = (double)x[c + ie];
            const dv4_ bv = *reinterpret_cast<const dv4_ *>(bb + c + i0);
            double aez = ihz2, awz = ihz2, wnz = 1.0;
            if constexpr (ST) {
                if (sgz) {
                    aez = sgz[(size_t)sg_ae(zkd) * nz + k];
                    awz = sgz[(size_t)sg_aw(zkd) * nz + k];
                    wnz = sgz[(size_t)SG_WN * nz + k];
                }
            }
            fv4 rv;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const double xcc = (double)xc[e];
                double xw = e == 0 ? xwe : (double)xc[e - 1];
                double xe = e == 3 ? xee : (double)xc[e + 1];
                bool xwall = false;
                if (wxw) {
                    const int i = i0 + e;
                    if (i == 0) xw = gx * xcc;
                    if (i + 1 == nx) xe = gx * xcc;
                    if (xw_u && i == 1) xw = 0.0;
                    xwall = xw_u && i == 0;
                }
                double zp = (double)xp[e], zm = (double)xm[e];
                if (wzw) {
                    if (k == 0) zm = gz * xcc;
                    if (k + 1 == nz) zp = gz * xcc;
                    if (zw_w && k == 1) zm = 0.0;
                    xwall = xwall || (zw_w && k == 0);
                }
                double lap;
                if constexpr (ST)
                    lap = (xe - xcc) * aex[e] - (xcc - xw) * awx[e] + (zp - xcc) * aez - (xcc - zm) * awz;
                else
                    lap = ((xe - xcc) - (xcc - xw)) * ihx2 + ((zp - xcc) - (xcc - zm)) * ihz2;
                lap += cu * (wu * (double)xu[e] - xcc) - cl * (xcc - wl * (double)xl[e]);
                const double ax = pois ? lap : xcc - cj * lap;
                rv[e] = (wall || xwall) ? 0.f : (float)(sg * ((bv[e] - bm) - ax));
                if constexpr (ST) wx += wD * wnx[e] * wnz * xcc;
                else wx += wD * xcc;
            }
            *reinterpret_cast<fv4 *>(rr + c + i0) = rv;
            xm = xc;
            xc = xp;
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
    const SplitJob &jb = ss.j[job];
    if (pass == 0) {
        // one pass only: no correction was measured, so no error estimate
        // exists; the report says NOT_CONVERGED with unknown (NaN) error
        if (threadIdx.x == 0) {
            done[job] = 0;
            if (jb.info) {
                ibs_solve_info *inf = static_cast<ibs_solve_info *>(jb.info);
                inf->iters = 1;
                inf->rel_correction = __builtin_nan("");
                inf->rel_residual = __builtin_nan("");
                if (inf->status == IBS_OK) inf->status = IBS_ERR_NOT_CONVERGED;
            }
        }
        return;
    }
    if (pass >= 2 && done[job]) return;     // stopped earlier: report stands
    const size_t off = (size_t)job * slots_per_job * 2;
    const double2 last = sum_pairs(red_last + off, slots_per_job);
    double rprev = 1.0;
    if (red_prev) {
        const double2 prev = sum_pairs(red_prev + off, slots_per_job);
        rprev = !(isfinite(prev.x) && isfinite(prev.y)) ? __builtin_nan("")
                                                        : (prev.y > 0.0 ? sqrt(prev.x / prev.y) : 0.0);
    }
    if (threadIdx.x == 0) {
        // a non-finite norm (a NaN or infinity in the data) predicts NaN,
        // which never meets tol
        const bool finite = isfinite(last.x) && isfinite(last.y) && isfinite(rprev);
        const double rc = !finite ? __builtin_nan("") : (last.y > 0.0 ? sqrt(last.x / last.y) : 0.0);
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

static int max_rows(const SplitSet &ss)   // transform rows per plane
{
    int r = 0;
    for (int q = 0; q < ss.n; ++q) {
        const int t = ss.j[q].rows - skip_first_row(ss.j[q].kind);
        r = t > r ? t : r;
    }
    return r;
}

// x transform tiling: a wave owns WM row blocks and all columns (NB <= NBT
// column blocks); at most 128 accumulator registers, and the data of the
// current and next chunk must stay in registers too.
static int x_nbt(int N) { return N <= 64 ? 4 : (N <= 128 ? 8 : (N <= 256 ? 16 : 32)); }
static constexpr int x_wm(int nbt) { return nbt == 4 ? 4 : (nbt == 32 ? 1 : 2); }

// folded x tiling: HBT 16-blocks per factor (HB = nx/32 <= HBT), WM row
// blocks per wave, at most 32 accumulator tiles per wave
static int xf_hbt(int nx)
{
    const int hb = nx / 32;
    return hb <= 2 ? 2 : hb <= 4 ? 4 : hb <= 6 ? 6 : hb <= 8 ? 8 : hb <= 12 ? 12 : 16;
}
static constexpr int xf_wm(int hbt) { return hbt <= 4 ? 2 : 1; }
static constexpr int f_steps(int hbt) { return hbt <= 8 ? 1 : 2; }   // factors per pipeline step: 2 / 1

static void xgemm_grid(const SplitSet &ss, const Plan &p, dim3 &grid)
{
    const int wm = x_folds_split(p) ? xf_wm(xf_hbt(p.nx)) : x_wm(x_nbt(p.nx));
    const int M = p.nz * max_rows(ss);
    grid = dim3((M + 8 * 16 * wm - 1) / (8 * 16 * wm), 1, ss.n);
}

// Workgroups of `kernel` (block size 512) resident on the device at once.
template <typename K>
static int resident_blocks(K kernel)
{
    int per_cu = 0, dev = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 512, 0) != hipSuccess ||
        hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        per_cu * cus <= 0)
        return 256;
    return per_cu * cus;
}

template <int HBT, typename Tin, int MODE, bool INV>
static void launch_xf(const SplitSet &ss, const Plan &p, const b8 *qs, double *red, const int *skip,
                      const double *scale,
                      dim3 grid, hipStream_t s)
{
    static const int resident =
        resident_blocks(split_xfold_kernel<HBT, xf_wm(HBT), Tin, MODE, INV, f_steps(HBT)>);
    const int tiles_per_job = (int)grid.x;
    const int ntiles = tiles_per_job * ss.n;
    const int g = ntiles < resident ? ntiles : resident;
    const double s0 = 1.0 / std::sqrt((double)p.nx), s1 = std::sqrt(2.0 / (double)p.nx);
    hipLaunchKernelGGL((split_xfold_kernel<HBT, xf_wm(HBT), Tin, MODE, INV, f_steps(HBT)>), dim3(g), dim3(512), 0, s,
                       ss, p.nz, p.nx, qs, red, skip, s0, s1, tiles_per_job, scale);
}

template <typename Tin, int MODE, bool INV>
static void launch_xf_hb(const SplitSet &ss, const Plan &p, const b8 *qs, double *red, const int *skip,
                      const double *scale,
                         dim3 grid, hipStream_t s)
{
    switch (xf_hbt(p.nx)) {
    case 2: launch_xf<2, Tin, MODE, INV>(ss, p, qs, red, skip, scale, grid, s); break;
    case 4: launch_xf<4, Tin, MODE, INV>(ss, p, qs, red, skip, scale, grid, s); break;
    case 6: launch_xf<6, Tin, MODE, INV>(ss, p, qs, red, skip, scale, grid, s); break;
    case 8: launch_xf<8, Tin, MODE, INV>(ss, p, qs, red, skip, scale, grid, s); break;
    case 12: launch_xf<12, Tin, MODE, INV>(ss, p, qs, red, skip, scale, grid, s); break;
    default: launch_xf<16, Tin, MODE, INV>(ss, p, qs, red, skip, scale, grid, s); break;
    }
}

template <int NBT, typename Tin, int MODE>
static void launch_x(const SplitSet &ss, const Plan &p, const b8 *qs, double *red, const int *skip,
                      const double *scale,
                     dim3 grid, hipStream_t s)
{
    hipLaunchKernelGGL((split_xgemm_kernel<NBT, x_wm(NBT), Tin, MODE>), grid, dim3(512), 0, s, ss,
                       p.nz, p.nx, p.nx, qs, red, skip, scale);
}

template <typename Tin, int MODE>
static void launch_x_nb(const SplitSet &ss, const Plan &p, const b8 *qs, double *red, const int *skip,
                      const double *scale,
                        dim3 grid, hipStream_t s)
{
    switch (x_nbt(p.nx)) {
    case 4: launch_x<4, Tin, MODE>(ss, p, qs, red, skip, scale, grid, s); break;
    case 8: launch_x<8, Tin, MODE>(ss, p, qs, red, skip, scale, grid, s); break;
    case 16: launch_x<16, Tin, MODE>(ss, p, qs, red, skip, scale, grid, s); break;
    default: launch_x<32, Tin, MODE>(ss, p, qs, red, skip, scale, grid, s); break;
    }
}

static size_t update_slots(const SplitSet &ss, const Plan &p);

hipError_t launch_split_xgemm(const SplitSet &ss, const Plan &p, const State &st, bool inverse, bool in64,
                              int mode, int pass, hipStream_t s)
{
    // the caller (run_refined) has checked the mode, pass and state size
    const int *skip = pass >= 2 ? st.done : nullptr;
    dim3 grid;
    xgemm_grid(ss, p, grid);
    // each refinement pass keeps its update partials in a region of its own
    const size_t region = update_region(p, ss.n);
    const bool upd = mode == 2 || mode == 4;
    double *red = st.red + (upd ? (size_t)(pass - 1) * region : 0);
    const double *scale = upd ? st.scale : nullptr;   // the residuals' sigma
    if (x_folds_split(p)) {
        const b8 *qs = reinterpret_cast<const b8 *>(blob_ptr(p, inverse ? p.lay.sxf_inv : p.lay.sxf_fwd));
        switch (in64 ? -1 : mode) {
        case -1: launch_xf_hb<double, 0, false>(ss, p, qs, red, skip, scale, grid, s); break;
        case 0: launch_xf_hb<float, 0, false>(ss, p, qs, red, skip, scale, grid, s); break;
        case 1: launch_xf_hb<float, 1, true>(ss, p, qs, red, skip, scale, grid, s); break;
        case 2: launch_xf_hb<float, 2, true>(ss, p, qs, red, skip, scale, grid, s); break;
        case 3: launch_xf_hb<float, 3, true>(ss, p, qs, red, skip, scale, grid, s); break;
        default: launch_xf_hb<float, 4, true>(ss, p, qs, red, skip, scale, grid, s); break;
        }
        return hipGetLastError();
    }
    const size_t *tab = inverse ? p.lay.sx_inv : p.lay.sx_fwd;
    const b8 *qs = reinterpret_cast<const b8 *>(blob_ptr(p, tab[XK_P]));
    SplitSet sj = ss;   // each job's matrix for its x operator
    for (int q = 0; q < sj.n; ++q) sj.j[q].xq = blob_ptr(p, tab[sj.j[q].xk]);
    switch (in64 ? -1 : mode) {
    case -1: launch_x_nb<double, 0>(sj, p, qs, red, skip, scale, grid, s); break;
    case 0: launch_x_nb<float, 0>(sj, p, qs, red, skip, scale, grid, s); break;
    case 1: launch_x_nb<float, 1>(sj, p, qs, red, skip, scale, grid, s); break;
    case 2: launch_x_nb<float, 2>(sj, p, qs, red, skip, scale, grid, s); break;
    case 3: launch_x_nb<float, 3>(sj, p, qs, red, skip, scale, grid, s); break;
    default: launch_x_nb<float, 4>(sj, p, qs, red, skip, scale, grid, s); break;
    }
    return hipGetLastError();
}

// z transform tiling: a wave owns all M = nz rows (MB <= MBT row blocks)
// and WN column blocks.

template <int HBT, int WN, bool INV>
static void launch_zf_dir(const SplitSet &ss, const Plan &p, const b8 *qs, const int *skip, hipStream_t s)
{
    static const int resident = resident_blocks(split_zfold_kernel<HBT, WN, INV, f_steps(HBT)>);
    const int Ncol = max_rows(ss) * p.nx;
    const int tiles_per_job = (Ncol + 8 * 16 * WN - 1) / (8 * 16 * WN);
    const int ntiles = tiles_per_job * ss.n;
    const int grid = ntiles < resident ? ntiles : resident;
    const double s0 = 1.0 / std::sqrt((double)p.nz), s1 = std::sqrt(2.0 / (double)p.nz);
    hipLaunchKernelGGL((split_zfold_kernel<HBT, WN, INV, f_steps(HBT)>), dim3(grid), dim3(512), 0, s, ss, p.nz, p.nx, qs,
                       skip, s0, s1, tiles_per_job);
}

template <int HBT, int WN>
static void launch_zf(const SplitSet &ss, const Plan &p, bool inverse, const b8 *qs, const int *skip,
                      hipStream_t s)
{
    if (inverse) launch_zf_dir<HBT, WN, true>(ss, p, qs, skip, s);
    else launch_zf_dir<HBT, WN, false>(ss, p, qs, skip, s);
}

hipError_t launch_split_zgemm(const SplitSet &ss, const Plan &p, const State &st, bool inverse, int pass,
                              hipStream_t s)
{
    const int *skip = pass >= 2 ? st.done : nullptr;
    if (z_folds_split(p)) {
        // folded: HBT 16-blocks per factor (HB = nz/32), WN column blocks per wave
        const b8 *qs = reinterpret_cast<const b8 *>(blob_ptr(p, inverse ? p.lay.szf_inv : p.lay.szf_fwd));
        const int hb = p.nz / 32;
        if (hb <= 2) launch_zf<2, 2>(ss, p, inverse, qs, skip, s);
        else if (hb <= 4) launch_zf<4, 1>(ss, p, inverse, qs, skip, s);
        else if (hb <= 6) launch_zf<6, 1>(ss, p, inverse, qs, skip, s);
        else if (hb <= 8) launch_zf<8, 1>(ss, p, inverse, qs, skip, s);
        else if (hb <= 12) launch_zf<12, 1>(ss, p, inverse, qs, skip, s);
        else launch_zf<16, 1>(ss, p, inverse, qs, skip, s);
        return hipGetLastError();
    }
    const int M = p.nz;
    const int Ncol = max_rows(ss) * p.nx;
    const size_t *tab = inverse ? p.lay.sz_inv : p.lay.sz_fwd;
    const b8 *qs = reinterpret_cast<const b8 *>(blob_ptr(p, tab[XK_P]));
    SplitSet sj = ss;   // each job's matrix for its z operator
    for (int q = 0; q < sj.n; ++q) sj.j[q].zq = blob_ptr(p, tab[sj.j[q].zk]);
    const int mbt = M <= 64 ? 4 : (M <= 128 ? 8 : (M <= 256 ? 16 : (M <= 384 ? 24 : 32)));
    const int wn = mbt == 4 ? 4 : (mbt <= 16 ? 2 : 1);
    dim3 grid((Ncol + 8 * 16 * wn - 1) / (8 * 16 * wn), 1, ss.n);
    switch (mbt) {
    case 4: hipLaunchKernelGGL((split_zgemm_kernel<4, 4>), grid, dim3(512), 0, s, sj, M, M, p.nx, qs, skip); break;
    case 8: hipLaunchKernelGGL((split_zgemm_kernel<8, 2>), grid, dim3(512), 0, s, sj, M, M, p.nx, qs, skip); break;
    case 16: hipLaunchKernelGGL((split_zgemm_kernel<16, 2>), grid, dim3(512), 0, s, sj, M, M, p.nx, qs, skip); break;
    case 24: hipLaunchKernelGGL((split_zgemm_kernel<24, 1>), grid, dim3(512), 0, s, sj, M, M, p.nx, qs, skip); break;
    default: hipLaunchKernelGGL((split_zgemm_kernel<32, 1>), grid, dim3(512), 0, s, sj, M, M, p.nx, qs, skip); break;
    }
    return hipGetLastError();
}

// Residual tiling: groups of rb_rows whole rows (256 threads, 4 points per
// thread) times z chunks of rz planes, with at most XSUM_SLOTS blocks per
// job (one x-sum partial each).
static void residual_tiling(const Plan &p, int &rb_rows, int &tiles_y, int &rz, int &tiles)
{
    rb_rows = std::max(1, 256 / (p.nx / 4));
    tiles_y = (p.ny + 1 + rb_rows - 1) / rb_rows;
    const int chunks = std::max(1, std::min((p.nz + 7) / 8, XSUM_SLOTS / tiles_y));
    rz = (p.nz + chunks - 1) / chunks;
    tiles = tiles_y * ((p.nz + rz - 1) / rz);
}

int residual_tiles(const Plan &p)
{
    int rb, ty, rz, t;
    residual_tiling(p, rb, ty, rz, t);
    return t;
}

// Power-of-two scale sigma of each job's FP32 residuals (refinement
// passes): from the largest magnitude of the first pass's pencil data (the
// block maxima its tridiagonal launches recorded; an orthonormal transform
// of the rhs, within a factor sqrt(n) of its largest entry), sigma =
// 2^-e with 2^e <= that maximum < 2^(e+1), so the residuals, about the
// first pass's relative error times the rhs, stay far inside the FP32 and
// bfloat16 exponent range whatever the rhs's own magnitude.  Scaling by a
// power of two is exact: it changes no rounding unless a value would
// otherwise leave that range.  One block per job, a fixed reduction order.
__global__ __launch_bounds__(256) void residual_scale_kernel(const double *__restrict__ bmax,
                                                             double *__restrict__ scale)
{
    __shared__ double sm[4];
    const int job = blockIdx.x;
    double m = 0.0;
    for (int q = threadIdx.x; q < BMAX_SLOTS; q += blockDim.x) m = fmax(m, bmax[(size_t)job * BMAX_SLOTS + q]);
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) m = fmax(m, __shfl_xor(m, d, 64));
    if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        m = fmax(fmax(sm[0], sm[1]), fmax(sm[2], sm[3]));
        double sg = 1.0;
        if (m > 0.0 && m <= 1.7976931348623157e308) {
            const int e = max(-120, min(120, ilogb(m)));
            sg = ldexp(1.0, -e);
        }
        scale[job] = sg;
    }
}

hipError_t launch_residual_scale(const SplitSet &ss, const State &st, hipStream_t s)
{
    hipLaunchKernelGGL(residual_scale_kernel, dim3(ss.n), dim3(256), 0, s, st.bmax, st.scale);
    return hipGetLastError();
}

hipError_t launch_residual_f32(const SplitSet &ss, const Plan &p, const State &st, int pass, bool x32,
                               hipStream_t s)
{
    // the tiling fits XSUM_SLOTS and nx / 4 <= 256 threads per row for
    // every grid the refined plan accepts (nx % 32 == 0, nx <= 512; checked
    // when the plan is built)
    const int *skip = pass >= 2 ? st.done : nullptr;
    int rb_rows, tiles_y, rz, tiles;
    residual_tiling(p, rb_rows, tiles_y, rz, tiles);
    dim3 grid(tiles, ss.n);
    auto go = [&](auto kernel) {
        hipLaunchKernelGGL(kernel, grid, dim3(256), 0, s, ss, p.nx, p.ny, p.nz, 1.0 / (p.hx * p.hx),
                           1.0 / (p.hz * p.hz), blob_ptr(p, p.lay.dyc), blob_ptr(p, p.lay.dyf),
                           st.bmean, st.xsum, skip, rb_rows, tiles_y, rz, p.py ? 1 : 0, p.wx ? 1 : 0,
                           p.wz ? 1 : 0, p.sx ? blob_ptr(p, p.lay.sgx) : nullptr,
                           p.sz ? blob_ptr(p, p.lay.sgz) : nullptr, st.scale);
    };
    const bool st_ = p.sx || p.sz;
    if (x32) st_ ? go(residual_f32_kernel<float, true>) : go(residual_f32_kernel<float, false>);
    else st_ ? go(residual_f32_kernel<double, true>) : go(residual_f32_kernel<double, false>);
    return hipGetLastError();
}

// Rows of the transform tiling are those of every component (ny; the v
// component's first wall row is left out), so the update partials depend
// only on the grid and the component count.
size_t update_region(const Plan &p, int ncomp)
{
    SplitSet ss{};
    ss.n = ncomp;
    for (int q = 0; q < ncomp; ++q) { ss.j[q].rows = p.ny; ss.j[q].kind = KIND_C; }
    dim3 grid;
    xgemm_grid(ss, p, grid);
    return 2 * (size_t)grid.x * grid.y * grid.z * UPD_WAVES;
}

hipError_t launch_refine_check(const SplitSet &ss, const Plan &p, const State &st, int pass, hipStream_t s)
{
    dim3 grid;
    xgemm_grid(ss, p, grid);
    const int per_job = (int)(grid.x * grid.y) * UPD_WAVES;
    const size_t region = update_region(p, ss.n);
    const double *last = pass >= 1 ? st.red + (size_t)(pass - 1) * region : nullptr;
    const double *prev = pass >= 2 ? st.red + (size_t)(pass - 2) * region : nullptr;
    hipLaunchKernelGGL(refine_check_kernel, dim3(ss.n), dim3(256), 0, s, ss, last, prev, per_job,
                       pass, p.desc.tol, st.done);
    return hipGetLastError();
}

}  // namespace ibs
