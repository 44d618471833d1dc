// Tridiagonal solves along y, one system per (x-mode a, z-mode c) pencil.
//
// After the x and z transforms every pencil is decoupled (Section 2.3.3,
// items S1.1 and S2.1; Appendix B gives the matrices on a uniform grid).
// Row j of pencil (a, c), with T the y part of the Laplacian (lo, di, up)
// and s = lambda_x[a] + lambda_z[c] (minus the transverse modified
// wavenumber squared, Appendix A):
//   Poisson   : lo_j x_{j-1} + (di_j + s) x_j + up_j x_{j+1} = b_j
//   Helmholtz : -c lo_j x_{j-1} + (1 - c s - c di_j) x_j - c up_j x_{j+1} = r_j
// The Neumann (0,0) pressure pencil is singular: its right-hand side is
// first made compatible (its volume-weighted mean removed), its first point
// is pinned to zero (as in Section 2.3.3, item S2.1), and after the solve
// the weighted mean is removed, which fixes the null mode at zero mean.
//
// Layout and parallel scheme (an MI355X design, not the paper's
// thread-per-pencil Thomas sweep): a tile is 16 (8 or 32, by arithmetic
// type) consecutive x-modes of one z-plane, all rows.  Persistent workgroups walk the tiles in
// adjacent pairs; each tile is read row by row into registers while the
// previous tile is being solved, then staged through LDS.  Each pencil is
// split into P (16 or 32) chunks of M consecutive rows, one lane per chunk.
// Every lane eliminates its chunk with two local sweeps (down and up),
// leaving one equation per lane that couples the last unknowns of
// neighbouring chunks; that reduced tridiagonal system of P equations is
// solved by parallel cyclic reduction with wavefront shuffles; the lanes
// then back-substitute their interiors.  Rows beyond the system size are
// identity rows.  The arithmetic is FP64, or FP32 for Helmholtz launches
// whose pencil condition numbers are provably small (refined path).
#pragma once
#include "ibs_internal.h"

#include <algorithm>
#include <cmath>

namespace ibs {

// 1/d from the hardware reciprocal estimate refined by two Newton steps
// (d is a normal, finite FP64 number here: diagonally dominant pivots).
static __device__ __forceinline__ double rcp64(double d)
{
    double x = __builtin_amdgcn_rcp(d);
    double e = fma(-d, x, 1.0);
    x = fma(x, e, x);
    e = fma(-d, x, 1.0);
    return fma(x, e, x);
}

// Raw buffer access with the hardware range check: offsets at or beyond the
// resource's byte count load 0 and drop stores.  The whole offset goes in
// the vector operand (the scalar offset is outside the range check).
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
template <typename T>
static __device__ __forceinline__ T buf_load(__amdgpu_buffer_rsrc_t rs, uint32_t voff, uint32_t soff);
template <>
__device__ __forceinline__ double buf_load<double>(__amdgpu_buffer_rsrc_t rs, uint32_t voff, uint32_t soff)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, voff, soff, 0));
}
template <>
__device__ __forceinline__ float buf_load<float>(__amdgpu_buffer_rsrc_t rs, uint32_t voff, uint32_t soff)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, voff, soff, 0));
}
static __device__ __forceinline__ void buf_store_raw(double v, __amdgpu_buffer_rsrc_t rs, uint32_t voff, uint32_t soff)
{
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), rs, voff, soff, 0);
}
static __device__ __forceinline__ void buf_store_raw(float v, __amdgpu_buffer_rsrc_t rs, uint32_t voff, uint32_t soff)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), rs, voff, soff, 0);
}
template <typename T>
static __device__ __forceinline__ void buf_store(T v, __amdgpu_buffer_rsrc_t rs, uint32_t voff, uint32_t soff)
{
    buf_store_raw(v, rs, voff, soff);
}

// 1/d in the arithmetic type: FP64 as above; FP32 from the hardware
// estimate and one Newton step.
static __device__ __forceinline__ double rcpr(double d) { return rcp64(d); }
static __device__ __forceinline__ float rcpr(float d)
{
    const float x = __builtin_amdgcn_rcpf(d);
    return fmaf(x, fmaf(-d, x, 1.0f), x);
}

// Largest pencil condition number solved in FP32 arithmetic (refined path).
constexpr double FP32_KAPPA = 16.0;

struct TriParams {
    const double *lam_x[NUM_XK], *lam_z[NUM_XK];   // per x / z kind of the job
    const double *lo[NUM_KINDS], *di[NUM_KINDS], *up[NUM_KINDS];
    const double *wy;   // Delta_j: weights of the pressure unknowns
    double *bmean;      // per job: weighted mean removed from the rhs (Poisson)
    const double *xsum; // per job: nxsum partial sums of Delta_j x (stride XSUM_SLOTS), or null
    int nxsum;
    int record_mean;    // write bmean (first pass of a solve)
    const int *skip;    // per job: refinement already stopped (later passes), or null
    double wsum_y;      // sum of Delta_j
    int nx, nz;
    int poisson;
    double inv_sqrt_nxnz;
    // pressure pencils of the refined path: the plan lists the 32-wide
    // x-tiles (per z-mode) holding a pencil too ill-conditioned for FP32
    // arithmetic (the FP64 lane).  lane_mode 0: every tile; 1: every tile
    // but the FP64-lane ones (FP32 arithmetic); 2: only the FP64-lane tiles.
    const unsigned *lane_mask;   // per z-mode: bit t = x-tile [32t, 32t+32) is in the FP64 lane
    const int *lane_list;        // FP64-lane tiles as (c << 8) | t
    int lane_len;
    int lane_mode;
    // refined path: the first pass's launches record per-job partial maxima
    // of their pencil data (BMAX_SLOTS per job, one per block: the FP32
    // tiles' launch the first half, the FP64 lane's the second), from which
    // the refinement passes take the power of two sigma that scales their
    // FP32 residuals; those passes then steer the mean in sigma units
    double *bmax;          // first pass: partial maxima, or null
    const double *scale;   // later passes: per job sigma, or null (1)
};

// T: storage type of the field (double, or float on the refined path);
// R: arithmetic type (double; float only for well-conditioned Helmholtz
// systems of the refined path, whose refinement absorbs FP32 rounding).
// CYC: cyclic systems (periodic y: row 0 couples to row n-1 and row n-1 to
// row 0 through the operator's corner coefficients lo[0], up[n-1]); the
// system then fills the P chunks exactly (n = P M, no padding rows) and the
// reduced system of the chunk ends is itself cyclic: its parallel cyclic
// reduction takes the neighbours at distance d modulo P, and after the last
// step (d = P/2, where both neighbours are the lane itself) each equation
// reads (EA + EB + EC) z = ED.
// BMX: this launch records the partial maxima (the refined path's first
// pass); a separate instantiation, so that no other launch carries the
// tracking.
// Registers: FP32 arithmetic is held to four waves per SIMD up to 9 rows per
// lane, and up to 13 for the non-cyclic systems (a few registers spill
// there, but two 8-wave blocks per CU instead of one: the 384-row pencils
// of 512x384x384 run 4 % faster); the rest is left to the compiler.
template <typename T, typename R, int P, int M, int TA, bool CYC = false, bool BMX = false>
__global__ __launch_bounds__(TA * P, (sizeof(R) == 4 && (M <= 9 || (!CYC && M <= 13))) ? 4 : 1) void tridiag_kernel(JobSet js, TriParams tp, int ntx,
                                                         int ntiles)
{
    // TA: pencils per tile
    constexpr int NT = TA * P;             // threads
    constexpr int NR = P * M;              // padded rows
    // LDS row of system row j: for even M each chunk of M rows is followed
    // by one unused row, so the P lanes of a pencil, which walk rows M
    // apart, hit distinct banks
    constexpr int MS = M + (M % 2 == 0 ? 1 : 0);
    constexpr int NRS = P * MS;            // LDS rows
    auto lr = [](int j) {
        if constexpr (MS == M) return j;
        else return (j / M) * MS + j % M;
    };
    constexpr int LDR = TA + 1;            // LDS row stride (elements)
    // Two staging buffers (alternate tiles) where they fit: a tile's
    // staging then needs no barrier against the previous tile's write-back,
    // which reads the other buffer (the barriers of the tile in between
    // order it after the write-back of the tile before).
    constexpr bool DB = P == 32 && M <= 9;
    __shared__ R sx[(DB ? 2 : 1) * NRS * LDR];
    __shared__ R slo[NRS], sdi[NRS], sup[NRS], sw[NRS];
    __shared__ double xs_sm[NT / 64];   // per-wave sums of the x-sum partials

    const int tid = threadIdx.x;
    const int nx = tp.nx;
    // staging role: thread loads rows lrow + P*r (r < M) of column lcol
    const int lcol = tid % TA, lrow = tid / TA;
    // solving role: pencil p (column), chunk k of M rows
    const int p = tid / P, k = tid % P;
    const int s = k * M;
    const bool pois = tp.poisson != 0;
    const uint32_t row_bytes = (uint32_t)nx * sizeof(T);

    // converged jobs (later refinement passes): read once, block-uniform
    int skipmask = 0;
    if (tp.skip)
        for (int q = 0; q < js.n; ++q) skipmask |= tp.skip[q] ? (1 << q) : 0;

    // Every fetch issues the same M + 2 loads and every write-back the same
    // M stores, whatever the tile: rows beyond the system, tiles beyond the
    // last and tiles of converged jobs are handled by the buffer range check
    // (loads return 0, stores are dropped).  With no loads or stores under
    // branches, the wait before a tile is used covers only that tile's data
    // and leaves the next tile's loads in flight.
    auto plane_rsrc = [&](int job, int c, bool live) {
        const FieldJob &jb = js.j[job];
        const T *base = reinterpret_cast<const T *>(jb.out) + (size_t)c * jb.rows * nx;
        return __builtin_amdgcn_make_buffer_rsrc(const_cast<T *>(base), (short)0,
                                                 live ? (int)(jb.rows * row_bytes) : 0, 0x00020000);
    };
    auto decode = [&](int tile, int &job, int &c, int &a0) {
        if (tp.lane_mode == 2) {
            // the listed 32-wide tiles, each as 32 / TA tiles of TA pencils
            constexpr int per = 32 / TA;
            const int per_job = tp.lane_len * per;
            job = tile / per_job;
            const int rem = tile - job * per_job;
            const int e = tp.lane_list[rem / per];
            c = e >> 8;
            a0 = (e & 0xff) * 32 + (rem % per) * TA;
        } else {
            job = tile / (tp.nz * ntx);
            const int rem = tile - job * tp.nz * ntx;
            c = rem / ntx;
            a0 = (rem - c * ntx) * TA;
        }
    };
    // maxima of |staged value| per job (BMX): each thread keeps a running
    // maximum for the job of its current tiles and folds it into the job's
    // LDS slot when the job changes (rarely: tiles run job by job) and at
    // the end, by an integer max on the bit patterns (non-negative floats
    // order as their patterns do)
    __shared__ unsigned bmx_sm[BMX ? STATE_JOBS : 1];
    float tmax = 0.f;
    int tjob = -1;
    if constexpr (BMX) {
        if (tid < STATE_JOBS) bmx_sm[tid] = 0u;
        __syncthreads();
    }
    // tiles left to the FP64 lane (lane_mode 1): block-uniform
    auto lane_skipped = [&](int c, int a0) {
        return tp.lane_mode == 1 && ((tp.lane_mask[c] >> (a0 >> 5)) & 1u);
    };
    // raw values only: conversion and wall rows are applied when the tile is
    // staged, so that nothing here waits for the loads
    auto fetch = [&](int tile, T (&pf)[M], double &plx, double &plz) {
        int job, c, a0;
        decode(tile < ntiles ? tile : ntiles - 1, job, c, a0);
        const bool live = tile < ntiles && !((skipmask >> job) & 1) && !lane_skipped(c, a0);
        plx = tp.lam_x[js.j[job].xk][a0 + p];
        plz = tp.lam_z[js.j[job].zk][c];
        const auto rs = plane_rsrc(job, c, live);
        const uint32_t sys0 = skip_first_row(js.j[job].kind);   // first row of the system
        const uint32_t voff = (uint32_t)(a0 + lcol) * sizeof(T) + (lrow + sys0) * row_bytes;
#pragma unroll
        for (int r = 0; r < M; ++r) pf[r] = buf_load<T>(rs, voff + r * P * row_bytes, 0);
    };

    // two register buffers: the tile two steps ahead is in flight while the
    // current one is solved (HBM latency is long next to one tile's work)
    T pfa[M], pfb[M];
    double lxa, lza, lxb, lzb;
    int cur_job = -1;
    auto process = [&](const int tile, T (&pf)[M], double &plx, double &plz, R *sx) {
        int job, c, a0;
        decode(tile, job, c, a0);
        const FieldJob &jb = js.j[job];
        // the v systems leave out the first wall row (kept at zero below)
        const int kind = jb.kind, sys0 = skip_first_row(kind), n = jb.rows - sys0;
        const bool live = !((skipmask >> job) & 1) && !lane_skipped(c, a0);   // block-uniform
        // the previous tile's staging buffer is no longer read (the
        // coefficient rows below are free once its solve, which ends with a
        // barrier, is done)
        if constexpr (!DB) __syncthreads();
        if (live && job != cur_job) {
            // rows of the job's operator without the pencil shift:
            // Poisson (lo, di, up); Helmholtz (-c lo, 1 - c di, -c up)
            const R cj = (R)jb.c;
            for (int j = tid; j < NR; j += NT) {
                const bool real = j < n;
                const R lo = real ? (R)tp.lo[kind][j + sys0] : R(0);
                const R di = real ? (R)tp.di[kind][j + sys0] : R(0);
                const R up = real ? (R)tp.up[kind][j + sys0] : R(0);
                slo[lr(j)] = pois ? lo : -cj * lo;
                sdi[lr(j)] = pois ? di : R(1) - cj * di;
                sup[lr(j)] = pois ? up : -cj * up;
                sw[lr(j)] = (real && pois) ? (R)tp.wy[j] : R(0);
            }
            cur_job = job;
        }
        const bool walls = kind == KIND_F;
#pragma unroll
        for (int r = 0; r < M; ++r) {
            const int j = lrow + P * r;
            sx[lr(j) * LDR + lcol] = (walls && j == n - 1) ? R(0) : (R)pf[r];
        }
        if constexpr (BMX) {
            if (live) {   // block-uniform
                if (job != tjob) {
                    if (tjob >= 0) atomicMax(&bmx_sm[tjob], __float_as_uint(tmax));
                    tjob = job;
                    tmax = 0.f;
                }
#pragma unroll
                for (int r = 0; r < M; ++r) {
                    const int j = lrow + P * r;
                    if (!(walls && j == n - 1)) tmax = fmaxf(tmax, fabsf((float)pf[r]));
                }
            }
        }
        const R sh = (R)(plx + plz);
        if (live && tp.xsum && pois && a0 == 0 && c == 0) {
            // refinement passes: the residual's partial sums of Delta_j x,
            // summed by the whole block for the pinned pencil (fixed order:
            // strided per thread, a butterfly per wave, the waves in order)
            const double *xsp = tp.xsum + (size_t)job * XSUM_SLOTS;
            double part = 0.0;
            for (int q = tid; q < tp.nxsum; q += NT) part += xsp[q];
#pragma unroll
            for (int d = 32; d >= 1; d >>= 1) part += __shfl_xor(part, d, 64);
            if ((tid & 63) == 0) xs_sm[tid >> 6] = part;
        }
        __syncthreads();
        fetch(tile + 2 * (int)gridDim.x, pf, plx, plz);  // this buffer's next tile
        if (live) {
            const int a = a0 + p;
            const R sadd = pois ? sh : -(R)jb.c * sh;   // pencil shift of the diagonal
            const bool pinned = pois && a == 0 && c == 0;

            R r[M];
#pragma unroll
            for (int t = 0; t < M; ++t) r[t] = sx[(k * MS + t) * LDR + p];

            R removed = 0.0;
            if (pinned) {
                // compatibility: remove the volume-weighted mean of this pencil's rhs
                R swr = 0.0, sww = 0.0;
#pragma unroll
                for (int t = 0; t < M; ++t) {
                    swr += sw[k * MS + t] * r[t];
                    sww += sw[k * MS + t];
                }
#pragma unroll
                for (int d = 1; d < P; d <<= 1) {
                    swr += __shfl_xor(swr, d, P);
                    sww += __shfl_xor(sww, d, P);
                }
                const R mean = swr / sww;
                removed = mean;
#pragma unroll
                for (int t = 0; t < M; ++t)
                    if (s + t < n) r[t] -= mean;
                if (k == 0) r[0] = 0.0;  // pin the first point
            }

            auto coef = [&](int j, R &A, R &B, R &C) {
                const bool real = j < n && !(pinned && j == 0);
                A = real ? slo[lr(j)] : 0.0;
                B = real ? sdi[lr(j)] + sadd : 1.0;
                C = real ? sup[lr(j)] : 0.0;
            };

            // down-sweep: rows s+1 .. s+M-1 in the form al x_s + x_j + ga x_{j+1} = rho
            R al[M], ga[M];
            {
                R A, B, C;
                coef(s + 1, A, B, C);
                R inv = rcpr(B);
                al[1] = A * inv; ga[1] = C * inv; r[1] = r[1] * inv;
#pragma unroll
                for (int t = 2; t < M; ++t) {
                    coef(s + t, A, B, C);
                    inv = rcpr(B - A * ga[t - 1]);
                    al[t] = -A * al[t - 1] * inv;
                    ga[t] = C * inv;
                    r[t] = (r[t] - A * r[t - 1]) * inv;
                }
            }
            // interior rows in terms of the chunk ends, x_j = bp + bq x_s + br x_e,
            // by back-substitution (no divisions), then the top row
            //   lam x_{s-1} + x_s + mu x_e = sig
            R lam_u, mu_u, sig_u;
            {
                R bp = r[M - 2], bq = -al[M - 2], br = -ga[M - 2];
#pragma unroll
                for (int t = M - 3; t >= 1; --t) {
                    bp = r[t] - ga[t] * bp;
                    bq = -al[t] - ga[t] * bq;
                    br = -ga[t] * br;
                }
                R A, B, C;
                coef(s, A, B, C);
                const R inv = rcpr(B + C * bq);
                lam_u = A * inv;
                mu_u = C * br * inv;
                sig_u = (r[0] - C * bp) * inv;
            }

            // reduced system in z_k = x_{last row of chunk k}
            R lam1, mu1, sig1;
            if constexpr (CYC) {
                const int kn = (k + 1) % P;   // chunk 0 follows chunk P-1
                lam1 = __shfl(lam_u, kn, P);
                mu1 = __shfl(mu_u, kn, P);
                sig1 = __shfl(sig_u, kn, P);
            } else {
                lam1 = __shfl_down(lam_u, 1, P);
                mu1 = __shfl_down(mu_u, 1, P);
                sig1 = __shfl_down(sig_u, 1, P);
                if (k == P - 1) { lam1 = 0.0; mu1 = 0.0; sig1 = 0.0; }
            }
            const R ae = al[M - 1], ge = ga[M - 1], re = r[M - 1];
            R EA = -ae * lam_u;
            R EB = 1.0 - ae * mu_u - ge * lam1;
            R EC = -ge * mu1;
            R ED = re - ae * sig_u - ge * sig1;
#pragma unroll
            for (int d = 1; d < P; d <<= 1) {
                // each lane scales its row to a unit diagonal (one division)
                // and the neighbours at distance d eliminate with it: three
                // values cross lanes each way instead of four
                const R ib = rcpr(EB);
                const R ua = EA * ib, uc = EC * ib, ud = ED * ib;
                R am, cm, dm, ap, cp, dp;
                if constexpr (CYC) {
                    const int km = (k - d + P) % P, kp = (k + d) % P;
                    am = __shfl(ua, km, P); cm = __shfl(uc, km, P); dm = __shfl(ud, km, P);
                    ap = __shfl(ua, kp, P); cp = __shfl(uc, kp, P); dp = __shfl(ud, kp, P);
                } else {
                    am = __shfl_up(ua, d, P); cm = __shfl_up(uc, d, P); dm = __shfl_up(ud, d, P);
                    ap = __shfl_down(ua, d, P); cp = __shfl_down(uc, d, P); dp = __shfl_down(ud, d, P);
                    if (k < d) { am = 0.0; cm = 0.0; dm = 0.0; }
                    if (k + d >= P) { ap = 0.0; cp = 0.0; dp = 0.0; }
                }
                const R nA = -EA * am, nC = -EC * cp;
                const R nB = EB - EA * cm - EC * ap;
                const R nD = ED - EA * dm - EC * dp;
                EA = nA; EB = nB; EC = nC; ED = nD;
            }
            R z, zm;
            if constexpr (CYC) {
                z = ED * rcpr(EA + EB + EC);
                zm = __shfl(z, (k - 1 + P) % P, P);
            } else {
                z = ED * rcpr(EB);
                zm = __shfl_up(z, 1, P);
                if (k == 0) zm = 0.0;
            }
            const R xs = sig_u - lam_u * zm - mu_u * z;

            // interior back-substitution, in place: r[t] becomes x[t]
            r[M - 1] = z;
#pragma unroll
            for (int t = M - 2; t >= 1; --t) r[t] = r[t] - al[t] * xs - ga[t] * r[t + 1];
            r[0] = xs;

            if (pinned) {
                // null mode: zero volume-weighted mean
                R swx = 0.0, sww = 0.0;
#pragma unroll
                for (int t = 0; t < M; ++t) {
                    swx += sw[k * MS + t] * r[t];
                    sww += sw[k * MS + t];
                }
#pragma unroll
                for (int d = 1; d < P; d <<= 1) {
                    swx += __shfl_xor(swx, d, P);
                    sww += __shfl_xor(sww, d, P);
                }
                R mx = swx / sww;
                if (tp.xsum) {
                    // refinement: steer the correction so that x + d has zero
                    // weighted mean (in this pencil's normalisation)
                    double part = 0.0;
#pragma unroll
                    for (int w = 0; w < NT / 64; ++w) part += xs_sm[w];
                    const double sgj = tp.scale ? tp.scale[job] : 1.0;
                    mx += sgj * part * tp.inv_sqrt_nxnz / tp.wsum_y;
                }
#pragma unroll
                for (int t = 0; t < M; ++t)
                    if (s + t < n) r[t] -= mx;
            }
#pragma unroll
            for (int t = 0; t < M; ++t) sx[(k * MS + t) * LDR + p] = r[t];

            if (pinned && k == 0 && tp.record_mean) tp.bmean[job] = removed * tp.inv_sqrt_nxnz;
            if (a0 == 0 && c == 0 && tid == 0 && jb.info) {
                ibs_solve_info *inf = static_cast<ibs_solve_info *>(jb.info);
                const double rm = removed * tp.inv_sqrt_nxnz;
                inf->iters = 1;
                inf->status = IBS_OK;
                inf->rel_residual = 0.0;
                inf->rel_correction = 0.0;
                inf->removed_mean = pois ? rm : 0.0;
            }
        }  // live
        __syncthreads();
        const auto rs = plane_rsrc(job, c, live);
        const uint32_t voff = (uint32_t)(a0 + lcol) * sizeof(T) + (lrow + sys0) * row_bytes;
#pragma unroll
        for (int r2 = 0; r2 < M; ++r2)
            buf_store<T>((T)sx[lr(lrow + P * r2) * LDR + lcol], rs, voff + r2 * P * row_bytes, 0);
        // the left-out wall row holds zeros (an offset past the range drops
        // the store of every other lane)
        buf_store<T>(T(0), rs, (sys0 && lrow == 0) ? (uint32_t)(a0 + lcol) * sizeof(T) : 0xFFFFFFF0u, 0);
    };
    // A block takes tiles in adjacent pairs (2b, 2b+1: neighbouring x-modes
    // of one z-plane), so the two halves of each 128-byte line of a 4-byte
    // field are read by the same block, back to back, through one L2.
    const int G = gridDim.x;
    fetch(2 * blockIdx.x, pfa, lxa, lza);
    fetch(2 * blockIdx.x + 1, pfb, lxb, lzb);
    for (int tile = 2 * blockIdx.x; tile < ntiles; tile += 2 * G) {
        process(tile, pfa, lxa, lza, sx);
        if (tile + 1 < ntiles) process(tile + 1, pfb, lxb, lzb, DB ? sx + NRS * LDR : sx);
    }
    if constexpr (BMX) {
        // block maxima per job, written to slot blockIdx.x of this launch's
        // half (the FP64 lane's launch: the second); the block also zeroes
        // its other slots of the half (blockIdx.x + k G), and a launch of
        // the first half the same slots of the second, which the lane's
        // launch, if any, then fills
        if (tjob >= 0) atomicMax(&bmx_sm[tjob], __float_as_uint(tmax));
        __syncthreads();
        constexpr int HALF = BMAX_SLOTS / 2;
        const int base = tp.lane_mode == 2 ? HALF : 0;
        for (int q = 0; q < js.n; ++q) {
            const double m = (double)__uint_as_float(bmx_sm[q]);
            double *dst = tp.bmax + (size_t)q * BMAX_SLOTS;
            for (int sl = (int)blockIdx.x + G * tid; sl < HALF; sl += G * NT) {
                dst[base + sl] = sl == (int)blockIdx.x ? m : 0.0;
                if (tp.lane_mode != 2) dst[HALF + sl] = 0.0;
            }
        }
    }
}

template <typename T, typename R, int P, int M, bool CYC, bool BMX>
static hipError_t launch_pm_k(const JobSet &js, const TriParams &tp, hipStream_t s)
{
    // pencils per tile: 16; 8 for FP32 data with FP64 arithmetic, whose
    // registers allow fewer waves per SIMD (blocks of 4 waves then still
    // fill them; with FP64 data the 16-wide tiles measured as fast with
    // less traffic); 32 for FP32 arithmetic over 32 lanes of up to 9 rows
    // (a tile row is one whole 128-byte line; 16-wave blocks, 5 % faster)
    constexpr int TA = sizeof(R) == 8 && sizeof(T) == 4 && P == 32 ? 8
                       : (sizeof(R) == 4 && P == 32 && M <= 9) ? 32 : 16;
    // persistent blocks walk the tiles (job, z-mode, TA x-modes) in order;
    // as many blocks as are resident at once, so that every block's tiles
    // run back to back
    static const int resident = [] {
        int per_cu = 0, dev = 0, cus = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, tridiag_kernel<T, R, P, M, TA, CYC, BMX>, TA * P, 0) !=
                hipSuccess ||
            hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            return 1024;
        return per_cu * cus > 0 ? per_cu * cus : 1024;
    }();
    static_assert(32 % TA == 0, "FP64-lane tiles are 32 pencils wide");
    const int ntx = tp.nx / TA;
    const int ntiles = tp.lane_mode == 2 ? js.n * tp.lane_len * (32 / TA) : ntx * tp.nz * js.n;
    if (ntiles == 0) return hipSuccess;
    const int pairs = (ntiles + 1) / 2;
    int grid = pairs < resident ? pairs : resident;
    if (BMX && grid > BMAX_SLOTS / 2) grid = BMAX_SLOTS / 2;   // one slot per block
    hipLaunchKernelGGL((tridiag_kernel<T, R, P, M, TA, CYC, BMX>), dim3(grid), dim3(TA * P), 0, s, js, tp, ntx,
                       ntiles);
    return hipGetLastError();
}

template <typename T, typename R, int P, int M, bool CYC = false>
static hipError_t launch_pm(const JobSet &js, const TriParams &tp, hipStream_t s)
{
    if constexpr (sizeof(T) == 4)
        if (tp.bmax) return launch_pm_k<T, R, P, M, CYC, true>(js, tp, s);
    return launch_pm_k<T, R, P, M, CYC, false>(js, tp, s);
}

}  // namespace ibs

namespace ibs {
// Cyclic launches (periodic y), k_tridiag_cyc.hip: n must be one of the
// sizes cyclic_rows_supported() accepts (n = P M exactly).
hipError_t launch_cyclic_dd(const JobSet &js, const TriParams &tp, int n, hipStream_t s);
hipError_t launch_cyclic_fd(const JobSet &js, const TriParams &tp, int n, hipStream_t s);
hipError_t launch_cyclic_ff(const JobSet &js, const TriParams &tp, int n, hipStream_t s);
}  // namespace ibs
