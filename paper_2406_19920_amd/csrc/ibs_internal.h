// Internal declarations shared by the host runtime and the kernel launchers.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/ibsolve.h"

namespace ibs {

// Kinds of y operator (rows of the tridiagonal systems, Appendix B):
//   KIND_P: pressure, cell centres, homogeneous Neumann walls (n = ny rows)
//   KIND_C: u and w, cell-centre height, Dirichlet wall by mirror ghost
//   KIND_F: v, y faces incl. the two wall faces as identity rows (n = ny+1)
//   KIND_PF: v when y is periodic (the triply periodic branch): ny faces,
//            no walls, cyclic.  With periodic y, KIND_P and KIND_C hold
//            the cyclic cell-centre operator (the same for p, u and w).
enum { KIND_P = 0, KIND_C = 1, KIND_F = 2, KIND_PF = 3, NUM_KINDS = 4 };

// Kinds of x operator (the eigenbasis of a field's x transform).  Periodic
// x: one real Fourier basis serves every field (the tables of kinds 1 and 2
// alias those of kind 0).  Walls in x (bc_x = IBS_DIRICHLET):
//   XK_P: pressure, cell centres, homogeneous Neumann (cosine series)
//   XK_C: v and w, cell centres, Dirichlet by mirror ghost (sine series)
//   XK_F: u, x faces; slot 0 is the wall face x = 0 and face nx is not
//         stored; the basis has a zero column 0 (and zero row 0), so the
//         wall slot transforms to zero both ways (sine series on 1..nx-1)
// Walls in z (bc_z = IBS_DIRICHLET) take the same three kinds along z, w
// being the face-normal component (plane 0 the wall face z = 0).
enum { XK_P = 0, XK_C = 1, XK_F = 2, NUM_XK = 3 };

// Byte offsets of the tables inside the device constant blob.
struct BlobLayout {
    size_t bx_fwd[NUM_XK], bx_inv[NUM_XK];   // x transform per x kind, B operand of C = A B,
                                             // swizzled (unfolded x: nx % 32 != 0 or walls)
    size_t az_fwd[NUM_XK], az_inv[NUM_XK];   // z transform per z kind, A operand of C = A B,
                                             // swizzled (unfolded z: nz % 32 != 0 or walls)
    // folded transforms (n % 32 == 0): the two H x H factors (H = n/2)
    size_t fx_fwd_c, fx_fwd_s, fx_inv_c, fx_inv_s;   // B-operand swizzle
    size_t fz_fwd_c, fz_fwd_s, fz_inv_c, fz_inv_s;   // A-operand swizzle
    size_t lam_x[NUM_XK], lam_z[NUM_XK];   // eigenvalues (double) per x / z kind
    size_t lo[NUM_KINDS], di[NUM_KINDS], up[NUM_KINDS];  // y operator rows
    size_t wy;               // Delta_j (pressure weights), ny doubles
    size_t dyc, dyf;         // cell heights [ny], centre distances [ny+1]
    size_t sx_fwd[NUM_XK], sx_inv[NUM_XK];   // x transform per x kind, bf16x3 split, B-operand
                                             // swizzle (unfolded x: nx % 64 != 0 or walls)
    size_t sz_fwd[NUM_XK], sz_inv[NUM_XK];   // z transform per z kind, bf16x3 split, A-operand
                                             // swizzle (unfolded z: nz % 64 != 0 or walls)
    size_t sxf_fwd, sxf_inv; // folded x transform factors, bf16x3 split (nx % 64 == 0)
    size_t szf_fwd, szf_inv; // folded z transform factors, bf16x3 split (nz % 64 == 0)
    size_t lane_mask;        // refined: per z-mode bit mask of FP64-lane x-tiles (uint32 [nz])
    size_t lane_list;        // refined: FP64-lane tiles, (c << 8) | t (int [lane_len])
    size_t sgx, sgz;         // stretched wall-bounded x / z: SG_SLOTS arrays of n doubles
                             // each (StretchSlot), else empty
    size_t total;
};

// Per-call mutable state of a solve, kept in the caller's workspace after
// the work fields (the plan's device blob is read-only once uploaded, so
// calls on one plan may run concurrently on different streams when each
// brings its own workspace).
constexpr int STATE_JOBS = 4;        // jobs (components) per call
constexpr int XSUM_SLOTS = 4096;     // max residual blocks per job (fixed order: deterministic sums)
constexpr int COMPAT_SLOTS = 2048;   // max blocks of the compatibility reduction
constexpr int RESID_SLOTS = 4096;    // max blocks of the residual() norm reduction
constexpr int MAX_PASSES = 8;        // most refinement passes a solve may take (max_iter)
constexpr int MAX_PLANES = 1024;     // largest nz a plan accepts
constexpr int BMAX_SLOTS = 2048;     // partial maxima per job (two halves of 1024 blocks)
// Smallest cell width a plan accepts, as a fraction of the domain length
// along that axis.  The operators' condition numbers grow as the inverse
// square of it: below about 1e-7 (tanh stretching beyond beta = 8 at 64
// cells) FP64 itself no longer resolves the solution (measured on
// manufactured solutions at beta = 10: errors of 1e-8 on the FP64 path and
// 1e-7 on the refined one, whose FP64 residuals then cannot tell it), so
// such grids are refused instead of solved to an accuracy no report shows.
constexpr double MIN_CELL_FRACTION = 1e-7;
// Refined path: pressure pencils whose condition bound 1 + g/|s| (g the
// Gershgorin bound of the y operator, s the pencil's transverse eigenvalue)
// exceeds this are solved with FP64 arithmetic (the FP64 lane); the rest in
// FP32, whose rounding the refinement then removes.
constexpr double LANE64_KAPPA = 1000.0;
// Cyclic pencils (periodic y) lose more to FP32 rounding at the same bound
// (the reduced system's last step divides by EA + EB + EC, which cancels
// towards the near-null constant mode): measured 1e-10 after two passes at
// a bound of 935 on a 96 x 96 x 64 grid; their lane takes bounds above 100.
constexpr double LANE64_KAPPA_CYCLIC = 100.0;
struct State {
    double *bmean = nullptr;   // per job: weighted mean of the Poisson rhs
    double *xsum = nullptr;    // per job: partial sums of Delta_j x (XSUM_SLOTS each)
    int *done = nullptr;       // per job: refinement stop flags
    int *incompat = nullptr;   // per job: strict compatibility check failed
    double *compat = nullptr;  // compatibility partials (2 per block)
    double *red = nullptr;     // refinement update partials, then residual() partials
    size_t red_count = 0;      // doubles in red
    double *bmax = nullptr;    // per job: partial maxima of the first pass's pencil data
                               // (BMAX_SLOTS each: the FP32 tiles' blocks, then the FP64 lane's)
    double *scale = nullptr;   // per job: power of two sigma the refinement passes scale
                               // their FP32 residuals by
};

// Kernel classes for the optional live profile (HIP events around launches).
enum {
    PK_XGEMM = 0, PK_ZGEMM, PK_TRIDIAG, PK_DIVERGENCE, PK_CORRECT, PK_RESIDUAL,
    PK_XGEMM_SPLIT, PK_ZGEMM_SPLIT, PK_TRIDIAG_F32, PK_UPDATE, PK_EXPLICIT, PK_IBM, NUM_PK
};

struct ProfRec {
    int kid;
    hipEvent_t start, stop;
    double flops, bytes;
};

struct Profile {
    bool on = false;
    std::vector<ProfRec> recs;
    std::vector<hipEvent_t> pool;
    double ms[NUM_PK] = {};
    double flops[NUM_PK] = {};
    double bytes[NUM_PK] = {};
    long long launches[NUM_PK] = {};
};

// Tunable launch shapes (results do not depend on the choice).
enum { TUNE_XFOLD = 0, TUNE_ZFOLD, NUM_TUNE };
static_assert(NUM_TUNE == IBS_NUM_TUNE, "tuning knobs and the ABI disagree");

// Per-index geometry of a stretched wall-bounded axis (n cells, widths
// Delta_i, centre distances delta_i), SG_SLOTS consecutive arrays of n
// doubles.  The 3-point rows along the axis are ae[i] (x_{i+1} - x_i) -
// aw[i] (x_i - x_{i-1}), a missing neighbour being the wall ghost (x_i for
// the pressure, -x_i for the mirror kind, 0 for the face kind), per kind:
//   XK_P cells: ae = 1/(delta_{i+1} Delta_i), aw = 1/(delta_i Delta_i)
//   XK_C cells: the same, the wall ones 1/Delta^2 (mirror ghost)
//   XK_F faces 1..n-1: ae = 1/(Delta_i delta_i), aw = 1/(Delta_{i-1} delta_i)
// (slots not used by a row hold 0).  rc = 1/Delta_i (divergence), rf =
// 1/delta_i (gradient; rf[0] = 0), wn = Delta_i / hbar (the cell's share
// of the volume weight, hbar the mean width).
enum StretchSlot { SG_RC = 0, SG_RF = 1, SG_WN = 2, SG_AE = 3, SG_AW = 4, SG_SLOTS = 3 + 2 * NUM_XK };
__host__ __device__ inline int sg_ae(int xk) { return SG_AE + 2 * xk; }
__host__ __device__ inline int sg_aw(int xk) { return SG_AW + 2 * xk; }

struct Plan {
    ibs_grid_desc desc;
    bool py = false;                               // y periodic (no walls)
    bool wx = false;                               // walls at x = 0 and x = lx
    bool wz = false;                               // walls at z = 0 and z = lz
    bool sx = false, sz = false;                   // stretched (wall-bounded) x / z
    int tune[NUM_TUNE] = {-1, -1};   // candidate index per knob; -1 = default
    int nx, ny, nz;
    double hx, hz;
    std::vector<double> yf, yc, dyc, dyf;          // grid
    std::vector<double> xf, zf;                    // x / z faces [n+1] (uniform: i h)
    std::vector<double> qx[NUM_XK], qz[NUM_XK];    // Q[i][a], row-major n x n, per x / z kind
                                                   // (forward: xhat_a = sum_i Q[i][a] x_i)
    std::vector<double> gx[NUM_XK], gz[NUM_XK];    // inverse bases: x_i = sum_a G[i][a] xhat_a
                                                   // (G = Q unless stretched)
    std::vector<double> lam_x[NUM_XK], lam_z[NUM_XK];
    std::vector<double> lo[NUM_KINDS], di[NUM_KINDS], up[NUM_KINDS];
    int rows[NUM_KINDS];
    BlobLayout lay;
    int lane_len = 0;                              // FP64-lane tiles (refined pressure pencils)
    std::vector<unsigned char> blob;               // host image of the blob
    void *dev_const = nullptr;
    Profile prof;
};

// Rows of a plane that the x and z transforms visit.  The v component
// (KIND_F) has ny + 1 rows per plane whose first and last are the wall
// faces; its first row is left out of the transforms (the tridiagonal step
// writes its zeros), so every component has ny transform rows per plane
// and a batch of components splits into equal tiles.  Transform row t of a
// [planes][rows][n] field is physical row phys_row(t).
__host__ __device__ inline int skip_first_row(int kind) { return kind == KIND_F ? 1 : 0; }
__host__ __device__ inline size_t phys_row(int t, int trows, int skip)
{
    return skip ? (size_t)t + (size_t)(t / trows) + 1 : (size_t)t;
}

// Per-component record for batched launches (passed by value).
// The refined path reuses it with float work arrays (cast through the
// pointers) and x the FP64 iterate.
struct FieldJob {
    const double *in;   // input field
    double *out;        // output field
    int rows;           // rows per z-plane (ny or ny+1)
    int kind;           // KIND_*
    int xk;             // XK_* (x operator)
    const void *xq;     // x transform matrix of this job (set by the x launchers)
    int zk;             // XK_* kind of the z operator
    const void *zq;     // z transform matrix of this job (set by the z launchers)
    double c;           // Helmholtz coefficient (Poisson: unused)
    void *info;         // ibs_solve_info* or null
};
struct JobSet {
    FieldJob j[4];
    int n;
};

// Error reporting
void set_error(const std::string &msg);

// Row counts the cyclic tridiagonal (periodic y) is built for.
bool cyclic_rows_supported(int n);
// y rows of a component's field: v (comp 1) has ny + 1 with walls, ny
// when y is periodic; u, w, p have ny.
inline int comp_rows(const Plan &p, int comp) { return comp == 1 && !p.py ? p.ny + 1 : p.ny; }
inline int comp_kind(const Plan &p, int comp)
{
    return comp == 1 ? (p.py ? KIND_PF : KIND_F) : KIND_C;
}
// x kind of a component (u 0, v 1, w 2); the pressure is XK_P.
inline int comp_xkind(const Plan &p, int comp)
{
    return !p.wx ? XK_P : (comp == 0 ? XK_F : XK_C);
}
// z kind of a component: w is the face-normal one.
inline int comp_zkind(const Plan &p, int comp)
{
    return !p.wz ? XK_P : (comp == 2 ? XK_F : XK_C);
}

// Workspace of one solve call: the work fields and the state after them.
size_t field_bytes_for(const Plan &p, int op, int ncomp);
size_t state_bytes_for(const Plan &p, int op, int ncomp);
size_t work_bytes_for(const Plan &p, int op, int ncomp);
State state_in(const Plan &p, void *work, int op, int ncomp);

// ---- kernel launchers (return hipError_t of the launch) --------------------
// C[M x N] = A[M x K] * Bs, A row-major (lda), Bs the swizzled K x N matrix
// of the job's x kind (bs[js.j[q].xk]); batched over the jobs of js
// (A = js.j[q].in, C = js.j[q].out, M = nz*rows).
hipError_t launch_xgemm_f64(const JobSet &js, int nz, int K, int N,
                            const double *const bs[NUM_XK], hipStream_t s);
// C[M x Ncol] = As * B, As the swizzled M x K matrix, B row-major (K x Ncol),
// Ncol = rows * nx per job.
// Folded FP64 transforms (valid when can_fold(n)).
bool can_fold(int n);
int fold_candidates();
// Folded split transforms: the half length must hold whole 32-deep chunks.
inline bool can_fold_split(int n) { return n % 64 == 0; }
// The folds use the Fourier basis's mirror symmetry: a direction folds only
// when it is periodic.
inline bool x_folds(const Plan &p) { return !p.wx && can_fold(p.nx); }
inline bool x_folds_split(const Plan &p) { return !p.wx && can_fold_split(p.nx); }
inline bool z_folds(const Plan &p) { return !p.wz && can_fold(p.nz); }
inline bool z_folds_split(const Plan &p) { return !p.wz && can_fold_split(p.nz); }
hipError_t launch_xfold_f64(const JobSet &js, const Plan &p, bool inverse, hipStream_t s);
hipError_t launch_zfold_f64(const JobSet &js, const Plan &p, bool inverse, hipStream_t s);
hipError_t launch_zgemm_f64(const JobSet &js, int M, int K, int nx,
                            const double *const as[NUM_XK], hipStream_t s);
// Tridiagonal pencils along y, in place on js.j[q].out ([nz][rows][nx]).
// poisson: pressure operator (pin + weighted-mean handling of pencil 0,0).
hipError_t launch_tridiag_f64(const JobSet &js, const Plan &p, const State &st, bool poisson,
                              hipStream_t s);
hipError_t launch_divergence(const Plan &p, const double *u, const double *v,
                             const double *w, double *b, double scale, hipStream_t s);
hipError_t launch_correct(const Plan &p, const double *phi, double *u, double *v,
                          double *w, double g, double *pr, const double *lap,
                          double cp, hipStream_t s);
hipError_t launch_residual(const Plan &p, int op, double c, const double *x,
                           const double *b, double *r, double *norms2, double *red, hipStream_t s);
// One Runge-Kutta sub-step around the solves (explicit estimate, immersed
// boundary forcing): the fields and coefficients its kernels take.
struct FsStage {
    double alpha, beta, gamma, zeta, dt, re;
    const double *u, *v, *w, *p;          // u^{n-1}, p^{n-1}
    double *nu, *nv, *nw;                 // in: N of the stage before (zeta != 0); out: N(u^{n-1})
    double *ue, *ve, *we;                 // u^e (eq. a)
    double *ru, *rv, *rw;                 // Helmholtz right-hand sides (eq. e)
    const double *markers, *ud, *dvol;    // immersed boundary: X_eta, U^d, dV_eta
    double *force;                        // F at the markers, or null
    int nmarkers;
};
hipError_t launch_explicit(const Plan &p, const FsStage &s, hipStream_t st);
hipError_t launch_ibm(const Plan &p, const FsStage &s, hipStream_t st);

// rhs += the contribution of inhomogeneous wall data lo, hi ([nz][nx]).
hipError_t launch_wall_data(const Plan &p, int op, double c, const double *lo, const double *hi,
                            double *rhs, hipStream_t s);
// Strict compatibility check of a Poisson rhs in FP64 (weighted mean against
// weighted rms, on b itself): partial sums, then the verdict per job, which
// sets st.incompat and, through the job's report, IBS_ERR_INCOMPATIBLE_RHS.
hipError_t launch_compat_partials(const Plan &p, const double *const *b, int njobs, const State &st,
                                  hipStream_t s);
hipError_t launch_compat_final(const Plan &p, void *const *info, int njobs, const State &st,
                               hipStream_t s);
int compat_blocks(const Plan &p);

// ---- refined (split-precision) path ---------------------------------------
struct SplitJob {
    const void *in;     // x transforms: FP64 (first pass) or FP32 input rows
    float *out;         // FP32 output (forward passes, z passes)
    double *x;          // x inverse: FP64 iterate (store or += update)
    void *xs;           // stored iterate the residual and the update read: x itself, or
                        // (first two passes of a multi-pass solve) an FP32 workspace field
    const double *b;    // residual: right-hand side
    float *r;           // residual: FP32 output
    int rows;           // rows per z-plane
    int kind;
    int xk;             // XK_* (x operator)
    const void *xq;     // x transform matrix of this job (set by the x launchers)
    int zk;             // XK_* kind of the z operator
    const void *zq;     // z transform matrix of this job (set by the z launchers)
    int op;             // IBS_OP_* of the job (residual stencil)
    double c;
    void *info;
};
struct SplitSet {
    SplitJob j[4];
    int n;
};
// x transform: in (FP64 when in64, else FP32) -> out (FP32), or, for the
// inverse: mode 1: x = result; 2: x += result with norm partials; 3: xs =
// result in FP32; 4: x = xs (FP32) + result with norm partials.
// pass: refinement pass of an update (mode 2), selecting its partial-sum region.
// Kernels of pass >= 2 return at once for jobs whose stop flag is set.
hipError_t launch_split_xgemm(const SplitSet &ss, const Plan &p, const State &st, bool inverse, bool in64,
                              int mode, int pass, hipStream_t s);
// Doubles of update partials one refinement pass of ncomp jobs writes.
size_t update_region(const Plan &p, int ncomp);
hipError_t launch_split_zgemm(const SplitSet &ss, const Plan &p, const State &st, bool inverse, int pass,
                              hipStream_t s);
// pass: refinement pass (0 records the rhs mean; later passes steer the
// Poisson correction so that x + d has zero weighted mean)
hipError_t launch_tridiag_f32(const JobSet &js, const Plan &p, const State &st, bool poisson, int pass,
                              hipStream_t s);
// x32: the stored iterate xs is FP32 (else FP64)
hipError_t launch_residual_f32(const SplitSet &ss, const Plan &p, const State &st, int pass, bool x32,
                               hipStream_t s);
int residual_tiles(const Plan &p);   // residual blocks (x-sum partials) per job
// After pass >= 1: predict the error, write the report, set the stop flag.
// pass 0 (a one-pass solve): no estimate exists; the report says so.
hipError_t launch_refine_check(const SplitSet &ss, const Plan &p, const State &st, int pass, hipStream_t s);
hipError_t launch_residual_scale(const SplitSet &ss, const State &st, hipStream_t s);

inline const double *blob_ptr(const Plan &p, size_t off) {
    return reinterpret_cast<const double *>(static_cast<const unsigned char *>(p.dev_const) + off);
}
inline double *blob_mut(const Plan &p, size_t off) {
    return reinterpret_cast<double *>(static_cast<unsigned char *>(p.dev_const) + off);
}

}  // namespace ibs
