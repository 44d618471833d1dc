/*
 * ibsolve: direct solver for the linear systems of one fractional step of
 * an incompressible staggered-grid flow solver, on AMD Instinct MI355X
 * (gfx950).
 *
 * The systems are those of the Runge-Kutta sub-step (Section 2.1):
 *   - the Helmholtz problem for each intermediate velocity component,
 *     eq. (e), written here as (I - c L) x = r with c = beta_n dt / Re
 *     (or 0.5 nu dt for Crank-Nicolson);
 *   - the pseudo-pressure Poisson problem, eq. (f), L_p phi = b, with the
 *     null mode fixed (Section 2.3.3, items S2 and S2.1);
 *   - the projection u = u* - g grad(phi), eq. (g), and the pressure
 *     update p += phi - c_p lap(phi), eq. (h).
 * Second-order central differences on a staggered Cartesian grid
 * (Section 2.1): periodic in x and z, walls in y (homogeneous Dirichlet
 * velocity, homogeneous Neumann pressure, Appendix B), y faces optionally
 * stretched by tanh.
 *
 * Method: x and z are diagonalised by precomputed 1-D orthonormal
 * eigenvector matrices applied as dense contractions (the paper's 2-D FFT
 * of the two periodic directions, Section 2.3.3, items S1.1/S2.1, with the
 * modified wavenumbers of Appendix A as eigenvalues); every (x-mode,
 * z-mode) pencil is then a tridiagonal system along y (Appendix B), solved
 * directly.
 *
 * Conventions for every entry point:
 *   - Arrays are C-contiguous [z][y][x] (x fastest), FP64, in device memory
 *     owned by the caller.  Cell fields (p, phi, b) and the x- and z-face
 *     velocities (u, w) are [nz][ny][nx].  The y-face velocity v is
 *     [nz][ny+1][nx]; its wall faces j = 0 and j = ny are ignored on input
 *     and written as 0 on output.
 *   - u[k][j][i] sits on the x-face at x = i*hx (between cells i-1 and i),
 *     w[k][j][i] on the z-face at z = k*hz, v[k][j][i] on the y-face y_f[j].
 *   - The library never allocates device memory: constants and workspace are
 *     caller-owned buffers sized by solver_plan_bytes().
 *   - Every call is asynchronous on the given stream (a hipStream_t passed
 *     as void*; NULL = the default stream) and returns an ibs_status.
 *     Argument errors are detected on the host before anything is enqueued.
 *     Errors raised asynchronously by the device surface in info->status or
 *     at the next call.  No call throws across this interface.
 *   - ibs_last_error() returns a thread-local message for the last failure.
 */
#ifndef IBSOLVE_H
#define IBSOLVE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ibs_plan_s *ibs_plan;

typedef enum {
    IBS_OK = 0,
    IBS_ERR_INVALID_ARG = 1,         /* bad pointer, size, shape or value       */
    IBS_ERR_UNSUPPORTED = 2,         /* valid request this build does not serve */
    IBS_ERR_WORKSPACE_TOO_SMALL = 3, /* work_bytes below solver_plan_bytes()    */
    IBS_ERR_HIP = 4,                 /* a HIP runtime call failed               */
    IBS_ERR_NOT_CONVERGED = 5,       /* refined path missed tol within max_iter */
    IBS_ERR_INCOMPATIBLE_RHS = 6,    /* strict_compat and b has a weighted mean */
    IBS_ERR_NOT_UPLOADED = 7         /* solver_plan_upload() not called yet     */
} ibs_status;

typedef enum {
    IBS_FP64 = 0,           /* every stage in FP64                              */
    IBS_REFINED_FP16X2 = 1, /* reserved: split-FP16 transforms; not built, so
                               solver_plan() returns IBS_ERR_UNSUPPORTED        */
    IBS_REFINED_BF16X3 = 2, /* split-BF16 (3 terms) transforms, FP32
                               accumulation, FP32 work arrays, refined against
                               an FP64 residual stored scaled by a power of
                               two taken from the first pass (rhs magnitudes
                               of about 1e-30 to 1e35 converge; beyond, a
                               solve may report IBS_ERR_NOT_CONVERGED)          */
    IBS_REFINED_AUTO = 3    /* reserved: library-chosen split scheme; not
                               built, so IBS_ERR_UNSUPPORTED                    */
} ibs_precision;

typedef enum { IBS_PERIODIC = 0, IBS_DIRICHLET = 1, IBS_NEUMANN = 2 } ibs_bc;

/* Problem description.  Grid: nx*ny*nz cells on [0,lx]x[0,ly]x[0,lz];
 * hx = lx/nx, hz = lz/nz; y faces y_f[j] = (ly/2)(1 + tanh(beta(2j/ny-1))/
 * tanh(beta)), j = 0..ny (beta = 0: uniform), unless y_faces is given.
 * Supported: nx, nz multiples of 16 in [16, 1024] (refined path: multiples
 * of 32, at most 512); ny in [2, 768]; bc_x and bc_z each IBS_PERIODIC or
 * IBS_DIRICHLET (walls, below); and in y
 * either walls (bc_y_vel = IBS_DIRICHLET, bc_y_p = IBS_NEUMANN) or
 * periodic y (bc_y_vel = bc_y_p = IBS_PERIODIC: the triply periodic
 * branch of Section 2.3.3, items S1/S2; ny in {48, 64, 80, 96, 128, 160,
 * 192, 256, 320, 384, 512}; the y faces, stretched or not, wrap: the
 * centres of cells ny-1 and 0 are (Delta_0 + Delta_{ny-1})/2 apart).  With
 * periodic y there are no walls: v is [nz][ny][nx] (face j at y_f[j],
 * face ny being face 0), the y pencils are cyclic, and the pressure's null
 * mode is fixed by the same zero volume-weighted mean.
 * Walls in x (bc_x = IBS_DIRICHLET; the non-periodic direction of the
 * paper's inflow-outflow example, Section 3.2, closed by walls; uniform x):
 * homogeneous Dirichlet velocity and Neumann pressure at x = 0 and x = lx.
 * Every field keeps its [nz][rows][nx] layout.  u's slot i holds the face
 * x = i hx: slot 0 is the wall face x = 0 (ignored on input, written as
 * zero on output; residual() reports 0 there) and the wall face x = lx is
 * not stored; its unknowns are slots 1..nx-1.  v and w (cell centres in x)
 * take the mirror-ghost Dirichlet row at the walls, the pressure zero flux.
 * The x transforms are then the cosine (pressure), sine-on-centres (v, w)
 * and sine-on-faces (u) eigenbases of the wall-bounded x operators, as
 * plain (unfolded) matrix products; ibs_rk_stage() is not served.
 * Walls in z (bc_z = IBS_DIRICHLET) are the same along z, w being the
 * face-normal component: w's plane 0 is the wall face z = 0 (ignored on
 * input, zero on output), the face z = lz is not stored; u and v take the
 * mirror-ghost row.  Walls in x and z together make a duct.
 * A wall-bounded x or z may be stretched (x_faces / z_faces: this
 * library's extension of the uniform grid of Section 2.1, as y's): every
 * operator along it is then the flux form over the local cell widths
 * Delta_i = f[i+1] - f[i] and centre distances delta_i (as in y), the
 * pressure's volume weights take Delta_x Delta_y Delta_z, and the
 * transforms along it are the generalised eigenbases of S q = lambda W q
 * (S the symmetric flux form, W the control widths), computed when the
 * plan is built (implicit QL in long double; O(n^3) host time).
 * Conditioning: a grid with a cell narrower than 1e-7 of its axis's length
 * (tanh stretching beyond beta = 8 at 64 cells, say) is refused with
 * IBS_ERR_UNSUPPORTED: its operators' condition number is past what FP64
 * residuals resolve, so neither path could solve it to a known accuracy. */
typedef struct {
    int32_t nx, ny, nz;
    double lx, ly, lz;        /* <= 0 means 1                                */
    double beta;              /* tanh stretching of y; 0 = uniform           */
    const double *y_faces;    /* optional host array [ny+1], strictly
                                 increasing; overrides beta/ly; copied        */
    int32_t bc_x, bc_z;       /* ibs_bc                                      */
    int32_t bc_y_vel, bc_y_p; /* ibs_bc                                      */
    int32_t precision;        /* ibs_precision                               */
    double tol;               /* refined path: target predicted relative
                                 error of x (1e-10 if <= 0)                  */
    int32_t max_iter;         /* refined path: most solve passes, 0..8 (0:
                                 3 for Poisson, 2 for Helmholtz); passes stop
                                 early once the predicted error meets tol.
                                 A single pass (max_iter = 1) measures no
                                 correction, so its report is always
                                 IBS_ERR_NOT_CONVERGED with NaN estimates    */
    int32_t strict_compat;    /* 1: a Poisson rhs whose volume-weighted mean
                                 exceeds 1e-10 times its weighted rms
                                 (checked in FP64 on b itself) reports
                                 IBS_ERR_INCOMPATIBLE_RHS in info (the solve
                                 still runs, with the mean removed)          */
    const double *x_faces;    /* optional host array [nx+1], finite and
                                 strictly increasing, the x faces of a
                                 stretched x (bc_x = IBS_DIRICHLET only);
                                 overrides lx (= x_faces[nx] - x_faces[0]);
                                 copied.  NULL: uniform                      */
    const double *z_faces;    /* the same for z ([nz+1], bc_z walls)         */
} ibs_grid_desc;

/* Per-solve report, written by the device at the end of the solve.  Must
 * point to memory the device can write (device memory or pinned host
 * memory); may be NULL. */
typedef struct {
    int32_t iters;          /* solve passes (1 for FP64; refinement passes)    */
    int32_t status;         /* ibs_status of the device part of the solve      */
    double rel_residual;    /* refined: predicted relative error of x, i.e.
                               rel_correction times the last observed
                               contraction ratio; NOT_CONVERGED if > tol       */
    double rel_correction;  /* refined: ||delta|| / ||x|| of the last pass     */
    double removed_mean;    /* Poisson: volume-weighted mean removed from b    */
} ibs_solve_info;

/* Operation codes for solver_plan_bytes() and residual(). */
#define IBS_OP_POISSON 0
#define IBS_OP_HELMHOLTZ_U 1
#define IBS_OP_HELMHOLTZ_V 2
#define IBS_OP_HELMHOLTZ_W 3

/* Build a plan on the host: the y grid, the tridiagonal coefficients of the
 * y operators (Appendix B, generalised to stretched y), the x and z
 * eigenvector matrices and eigenvalues (Appendix A: lambda = -kappa'^2),
 * kernel tile choices.  *out owns host memory only; free it with
 * solver_plan_destroy().  Errors: IBS_ERR_INVALID_ARG, IBS_ERR_UNSUPPORTED. */
ibs_status solver_plan(const ibs_grid_desc *desc, ibs_plan *out);

/* Byte counts for the caller's buffers.  op: IBS_OP_POISSON, or
 * IBS_OP_HELMHOLTZ_U for a Helmholtz batch of ncomp (1..3) components (the
 * count covers any mix of u, v, w); ncomp is ignored for Poisson.
 * const_bytes: size of the device constant buffer for solver_plan_upload();
 * work_bytes: minimum workspace for one solve call: one FP64 field per
 * component on the FP64 path, three FP32 fields per component on the
 * refined path (cells of a field: nz * ny * nx, or nz * (ny+1) * nx for a
 * Helmholtz batch), followed by the call's mutable state (mean of the
 * rhs, refinement stop flags, reduction partials; under 2 MB at 512^3).
 * Either output pointer may be NULL. */
ibs_status solver_plan_bytes(ibs_plan plan, int32_t op, int32_t ncomp,
                             size_t *const_bytes, size_t *work_bytes);

/* Copy the plan's constants into dev_const (device memory, >= const_bytes,
 * 256-byte aligned) on stream.  The plan remembers dev_const; it must stay
 * allocated while the plan is used.  The copy reads host memory owned by
 * the plan, so the plan must outlive the copy.  After the upload the
 * device constants are only read: solves on one plan may run concurrently
 * (on different streams, from different host threads) as long as each call
 * has a workspace of its own; calls that share a workspace race. */
ibs_status solver_plan_upload(ibs_plan plan, void *dev_const, size_t bytes,
                              void *stream);

ibs_status solver_plan_destroy(ibs_plan plan);

/* Pressure Poisson problem, eq. (f): L_p phi = b with homogeneous Neumann
 * walls.  The volume-weighted mean of b is removed first (Neumann
 * compatibility; reported in info->removed_mean) and phi is returned with
 * zero volume-weighted mean (the null mode; internally the singular
 * (0,0) pencil is pinned at its first point as in Section 2.3.3, item
 * S2.1, then shifted).  b: [nz][ny][nx] device, read only; phi: same shape.
 * FP64 path: phi may alias b.  Refined path: phi must not alias b (later
 * passes re-read b; IBS_ERR_INVALID_ARG).  work: device buffer of >=
 * work_bytes (solver_plan_bytes with IBS_OP_POISSON), 32-byte aligned, not
 * shared with a concurrent call.  Errors: IBS_ERR_INVALID_ARG,
 * IBS_ERR_NOT_UPLOADED, IBS_ERR_WORKSPACE_TOO_SMALL, IBS_ERR_HIP. */
ibs_status solve_poisson(ibs_plan plan, const double *b, double *phi, void *work,
                         size_t work_bytes, ibs_solve_info *info, void *stream);

/* Helmholtz problems, eq. (e): (I - c[q] L) x[q] = r[q] for ncomp (1..3)
 * components solved together (one launch per stage).  comp[q] in {0 = u,
 * 1 = v, 2 = w} selects the grid of component q (u, w: Dirichlet wall by a
 * mirror ghost, Appendix B alpha = 2; v: wall-face values, alpha = 1).
 * comp, c, r, x are HOST arrays of ncomp entries; r[q], x[q] are device
 * fields of the component's shape; c[q] >= 0.  FP64 path: x[q] may alias
 * r[q].  Refined path: x[q] must not alias r[q] (IBS_ERR_INVALID_ARG).
 * info: NULL or ncomp records.  work as for solve_poisson, sized with
 * IBS_OP_HELMHOLTZ_U and ncomp.  Errors as solve_poisson. */
ibs_status solve_helmholtz_batch(ibs_plan plan, int32_t ncomp, const int32_t *comp,
                                 const double *c, const double *const *r,
                                 double *const *x, void *work, size_t work_bytes,
                                 ibs_solve_info *info, void *stream);

/* Pressure Poisson problem exactly as solve_poisson(), for callers that
 * cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): no workspace argument,
 * and no allocation.  The work fields and per-call state live in a fixed
 * array of IBS_NOALLOC_SCRATCH_BYTES inside this library, one per GPU,
 * held until the process ends; a grid whose Poisson workspace
 * (solver_plan_bytes) exceeds it is refused with
 * IBS_ERR_WORKSPACE_TOO_SMALL before anything is enqueued.  Every call on
 * one GPU shares that GPU's array: calls that overlap in time on one GPU
 * (other streams, other host threads) race and must be ordered by the
 * caller.  Results are bitwise those of solve_poisson().  Errors as
 * solve_poisson, and IBS_ERR_HIP if the array's address cannot be resolved
 * on the current device. */
#define IBS_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
ibs_status solve_poisson_noalloc(ibs_plan plan, const double *b, double *phi,
                                 ibs_solve_info *info, void *stream);

/* Residual r = b - A x in FP64 for op IBS_OP_POISSON (A = L_p) or
 * IBS_OP_HELMHOLTZ_{U,V,W} (A = I - c L), with the 7-point stencil.  x, b, r
 * device fields of the op's shape (r may not alias x).  norms2: NULL or a
 * device double[2] receiving ||r||_2^2 and ||b||_2^2 over the unknowns
 * (deterministic fixed-order reduction).  work: only read when norms2 is
 * not NULL (then the reduction partials go there): a 32-byte aligned device
 * buffer of >= the work_bytes solver_plan_bytes() gives for IBS_OP_POISSON
 * (op 0) or IBS_OP_HELMHOLTZ_U with ncomp 1 (ops 1..3), not shared with a
 * concurrent call; may be NULL otherwise.  Errors: IBS_ERR_INVALID_ARG,
 * IBS_ERR_NOT_UPLOADED, IBS_ERR_WORKSPACE_TOO_SMALL. */
ibs_status residual(ibs_plan plan, int32_t op, double c, const double *x,
                    const double *b, double *r, double *norms2, void *work,
                    size_t work_bytes, void *stream);

/* RHS of the Poisson problem (kernel E2 of Section 2.3.2):
 * b = scale * D(u, v, w), D the staggered divergence.  v's wall faces are
 * read (a nonzero wall flux makes b incompatible).  b: [nz][ny][nx]. */
ibs_status ibs_divergence(ibs_plan plan, const double *u, const double *v,
                          const double *w, double *b, double scale, void *stream);

/* Inhomogeneous wall data (Section 2.3.3, subroutine BC2.2; Appendix B's
 * boundary terms): adds to the right-hand side rhs of op (in place) the
 * contribution of prescribed data at the walls y = 0 (lo) and y = ly (hi),
 * so that the homogeneous solve of the modified rhs returns the solution
 * with that data.  lo, hi: device arrays [nz][nx] (one value per wall
 * column), either may be NULL (zero data).
 *   IBS_OP_POISSON: the wall flux dphi/dy (Neumann data);
 *     b[0] += lo/Delta_0, b[ny-1] -= hi/Delta_{ny-1} (c unused).
 *   IBS_OP_HELMHOLTZ_U / _W: the wall value of the velocity (mirror ghost
 *     2g - f_0, Appendix B alpha = 2); r[0] += 2c lo/Delta_0^2,
 *     r[ny-1] += 2c hi/Delta_{ny-1}^2, c the coefficient of the solve.
 *   IBS_OP_HELMHOLTZ_V: the value of the wall face itself (alpha = 1);
 *     r at face 1 += c lo/(Delta_0 delta_1), at face ny-1 += c hi/
 *     (Delta_{ny-1} delta_{ny-1}).  The solve writes 0 to the solution's
 *     wall faces; the caller stores lo/hi there.
 * A Poisson rhs with Neumann data is compatible when the weighted mean of
 * the modified rhs is zero (the solve removes what is not).  Call it once
 * per rhs, before the solve, on the solve's stream.  Errors:
 * IBS_ERR_INVALID_ARG, IBS_ERR_NOT_UPLOADED, IBS_ERR_HIP. */
ibs_status ibs_wall_data(ibs_plan plan, int32_t op, double c, const double *lo,
                         const double *hi, double *rhs, void *stream);

/* ---- One Runge-Kutta sub-step of the fractional-step method ------------
 * (Section 2.1, eqs. a-h; kernels E1, L1, E2, E3 and the solves of Section
 * 2.3): with stage coefficients alpha, beta, gamma, zeta (user supplied,
 * e.g. a low-storage RK3), time step dt and Reynolds number Re,
 *   (a) u^e = u + dt[(alpha+beta)/Re L u - (alpha+beta) G p - gamma N(u)
 *               - zeta N(u of the stage before)]
 *   (b-d) immersed boundary: U^e(X) interpolated with the Roma three-point
 *       kernel, F = (U^d - U^e)/dt, f spread back with dV_eta
 *   (e) (I - c L) u_s = u^e - c L u + dt f,   c = beta dt / Re
 *   (f) L_p phi = D u_s / ((alpha+beta) dt)
 *   (g) u = u_s - (alpha+beta) dt G phi;  (h) p += phi - c D u_s / ((alpha+beta) dt)
 * (u_s: the intermediate velocity).
 * N(u) is the convective term div(u u) in divergence form on the staggered
 * grid (second-order central differences; products on the faces/edges
 * where their derivatives need them, from arithmetic means). */
typedef struct {
    double alpha, beta, gamma, zeta;   /* stage coefficients of eq. (a)         */
    double dt, re;                     /* time step (> 0), Reynolds number (> 0) */
} ibs_rk_coef;

typedef struct {
    double *u, *v, *w, *p;   /* device; in: u^{n-1}, p^{n-1}; out: u^n, p^n (in place) */
    double *nu, *nv, *nw;    /* device, shaped like u, v, w; in: N of the stage before
                                (read only when zeta != 0); out: N(u^{n-1}) for the next
                                stage (may be the same arrays) */
    const double *markers;   /* device [nmarkers][3] marker positions (x, y, z), or NULL */
    const double *ud;        /* device [nmarkers][3] prescribed velocity U^d            */
    const double *dvol;      /* device [nmarkers] volume dV_eta of each marker          */
    double *force;           /* device [nmarkers][3] out: F, or NULL                    */
    int32_t nmarkers;        /* 0: no immersed body                                     */
} ibs_stage_fields;

/* Workspace bytes for ibs_rk_stage() on this plan (u^e and the Helmholtz
 * right-hand sides, the Poisson fields, and one solve's workspace). */
ibs_status ibs_stage_bytes(ibs_plan plan, size_t *work_bytes);

/* One sub-step, asynchronous on stream.  The Helmholtz and Poisson solves
 * run in the plan's precision; info: NULL or 4 device records (Helmholtz
 * u, v, w, then Poisson).  With markers the grid must be uniform in y (the
 * kernel's spacing; IBS_ERR_UNSUPPORTED otherwise); the spreading adds by
 * atomics, so results with markers are reproducible to rounding, not
 * bitwise.  Errors: IBS_ERR_INVALID_ARG, IBS_ERR_UNSUPPORTED,
 * IBS_ERR_NOT_UPLOADED, IBS_ERR_WORKSPACE_TOO_SMALL, IBS_ERR_HIP. */
ibs_status ibs_rk_stage(ibs_plan plan, const ibs_rk_coef *coef, const ibs_stage_fields *fields,
                        void *work, size_t work_bytes, ibs_solve_info *info, void *stream);

/* Projection, eq. (g), and pressure update, eq. (h) (kernel E3):
 * u -= g dphi/dx, v -= g dphi/dy (interior faces; walls set to 0),
 * w -= g dphi/dz; if p != NULL: p += phi - cp * lap_phi, where lap_phi is the
 * already-known Laplacian of phi (the Poisson right-hand side b; may be
 * NULL when cp == 0).  In place on u, v, w, p. */
ibs_status ibs_correct(ibs_plan plan, const double *phi, double *u, double *v,
                       double *w, double g, double *p, const double *lap_phi,
                       double cp, void *stream);

/* ---- Batched execution (many independent grids, one graph launch) ----- */

typedef struct ibs_batch_s *ibs_batch;

/* One solve of a batch.  op: IBS_OP_POISSON (rhs[0] -> x[0]) or
 * IBS_OP_HELMHOLTZ_U for a Helmholtz batch of ncomp components (comp, c,
 * rhs, x as in solve_helmholtz_batch).  Every pointer is captured as is:
 * the buffers must stay allocated, and at the same addresses, for the
 * lifetime of the batch.  Jobs that share a workspace are ordered one after
 * the other (same graph branch); jobs with distinct workspaces may overlap,
 * whether or not they share a plan. */
typedef struct {
    ibs_plan plan;
    int32_t op;
    int32_t ncomp;
    int32_t comp[3];
    double c[3];
    const double *rhs[3];
    double *x[3];
    void *work;
    size_t work_bytes;
    ibs_solve_info *info;   /* NULL or ncomp (Poisson: 1) device records */
} ibs_batch_job;

/* Schedule policies of a batch: how the jobs' workspaces are dealt to the
 * graph's lanes (jobs sharing a workspace always share a lane). */
#define IBS_SCHED_BALANCED 0   /* largest work first, each to the least loaded lane */
#define IBS_SCHED_IN_ORDER 1   /* workspaces in submission order, round-robin */

/* Record njobs solves (the batching of the multi-grid configuration) into
 * one HIP graph by stream capture.  Jobs are spread over up to nlanes
 * independent graph branches by IBS_SCHED_BALANCED so that small grids
 * overlap on the device.  Nothing is executed.  The schedule never changes
 * a result: each job's launches run in the same order on its own
 * workspace.  Errors: IBS_ERR_INVALID_ARG (bad job; ibs_last_error() names
 * it), IBS_ERR_HIP, and any error a job's solve call would return. */
ibs_status ibs_batch_build(const ibs_batch_job *jobs, int32_t njobs, int32_t nlanes,
                           ibs_batch *out);
/* As ibs_batch_build() with the schedule policy given (IBS_SCHED_*). */
ibs_status ibs_batch_build_sched(const ibs_batch_job *jobs, int32_t njobs, int32_t nlanes, int32_t policy,
                                 ibs_batch *out);
/* Schedule autotuner: builds the batch for each candidate (lane counts 1,
 * 2, 4, ... up to the number of distinct workspaces, both policies),
 * replays each once untimed and then `reps` times in each of three
 * interleaved rounds on stream (synchronising), keeps each candidate's
 * fastest round and returns the fastest candidate's lane count, policy
 * and ms per replay (ms may be NULL).  The jobs run; their outputs are
 * those of any schedule.  Errors as ibs_batch_build(), IBS_ERR_HIP. */
ibs_status ibs_batch_autotune(const ibs_batch_job *jobs, int32_t njobs, int32_t reps, int32_t *nlanes,
                              int32_t *policy, float *ms, void *stream);
/* Multi-grid batch (the many-grid configuration through persistent
 * work-queue kernels): every field of every job is listed in one device job
 * table, and each stage of the separable solve (x transform, z transform,
 * y tridiagonal, inverse z, inverse x; Section 2.3.3, items S2.1-S2.2) is
 * ONE persistent launch whose waves walk a device work list of tiles drawn
 * from all grids, so a batch of G grids of any sizes replays as 5 kernel
 * launches in one graph.  FP64 arithmetic throughout (plain FP64
 * matrix-core transforms against each grid's eigenbases, Thomas pencils):
 * results agree with solve_poisson / solve_helmholtz_batch to rounding, not
 * bitwise.  Jobs: plans uploaded, precision IBS_FP64, walls in y (not
 * periodic y), strict_compat 0, any x / z conditions (uniform or
 * stretched); workspaces as for the single solves (solver_plan_bytes),
 * one of its own per job (jobs run side by side); rhs, x and work 32-byte
 * aligned, as for the single solves; rhs may alias x.  info
 * reports as the FP64 solves do.  The builder allocates one device buffer
 * (job table, work lists, transform tables, and the tridiagonal pencils'
 * forward factors, which depend on the systems only: one field's size per
 * field, about as much device memory again as the fields themselves; freed
 * by ibs_batch_destroy()) and computes those factors once on the device
 * before capturing the graph (synchronously).  Errors: IBS_ERR_INVALID_ARG (bad job, shared
 * workspace), IBS_ERR_UNSUPPORTED (refined or periodic-y plan, strict
 * compatibility), IBS_ERR_NOT_UPLOADED, IBS_ERR_WORKSPACE_TOO_SMALL,
 * IBS_ERR_HIP. */
ibs_status ibs_batch_build_multigrid(const ibs_batch_job *jobs, int32_t njobs, ibs_batch *out);
/* Replay the whole batch on stream with one graph launch (asynchronous). */
ibs_status ibs_batch_launch(ibs_batch batch, void *stream);
ibs_status ibs_batch_destroy(ibs_batch batch);

/* Host copies of the plan's tables, for inspection and host-side checks.
 * table: 0 y faces [ny+1]; 1 Q_x [nx*nx] (row-major, Q[i*nx+a] = mode a at
 * grid index i); 2 Q_z [nz*nz]; 3 lambda_x [nx]; 4 lambda_z [nz];
 * 5+3*kind+{0,1,2}: lower, diagonal, upper coefficients [ny+1] of the y
 * operator of kind 0 (pressure), 1 (u, w), 2 (v, rows = faces 0..ny), 3 (v
 * of a periodic-y plan, rows = faces 0..ny-1).  With periodic y, kinds 0
 * and 1 hold the cyclic cell operator; lower[0] and upper[ny-1] are then
 * the corner couplings (row 0 to row ny-1 and back).  Tables 1 and 3 are
 * the pressure's x basis; with walls in x, 17 and 18 are Q_x of v/w and of
 * u, 19 and 20 their lambda_x (periodic x: the same as 1 and 3); with walls
 * in z, 21 and 22 are Q_z of u/v and of w, 23 and 24 their lambda_z
 * (periodic z: the same as 2 and 4).  The Q tables are the forward
 * transforms, xhat_a = sum_i Q[i*n+a] x_i; 25 + k (x) and 28 + k (z) are
 * the inverse transforms G of kind k (0 pressure, 1 mirror-ghost velocity
 * components, 2 the face-normal one), x_i = sum_a G[i*n+a] xhat_a, equal
 * to Q except on a stretched axis; 31 and 32 the x and z faces [n+1].
 * out: host array of n doubles; n must equal the table length (queried by
 * passing out = NULL, which returns the length through *n). */
ibs_status ibs_plan_export(ibs_plan plan, int32_t table, double *out, size_t *n);

/* Live per-kernel profile of one plan's launches, for benchmarking.
 * ibs_profile(plan, 1) clears the record and brackets every later launch of
 * the plan with HIP events on the launch stream; ibs_profile(plan, 0) stops.
 * ibs_profile_read() synchronises on the recorded events and returns, for
 * kernel class `kernel`, the summed device time (ms), the launch count and
 * the summed algorithmic flops and HBM bytes of those launches (the work
 * the method needs, not counter readings).  Kernel classes: 0 x transform
 * (FP64 matrix cores), 1 z transform (FP64), 2 y tridiagonal (FP64),
 * 3 divergence, 4 correction, 5 residual, 6 x transform (split),
 * 7 z transform (split), 8 y tridiagonal (FP32 data), 9 refinement update,
 * 10 explicit estimate of a Runge-Kutta stage, 11 immersed-boundary forcing.
 * Any output pointer may be NULL. */
ibs_status ibs_profile(ibs_plan plan, int32_t enable);
ibs_status ibs_profile_read(ibs_plan plan, int32_t kernel, double *ms, int64_t *launches,
                            double *flops, double *bytes);

/* Measured choice of launch shapes.  Some kernels come in several tile
 * shapes that compute every output element with the same operations in the
 * same order (so results are bitwise identical whichever is used) but run
 * at different speeds on a given grid.  ibs_autotune() times each candidate
 * of each such knob on the plan's own grid, using `scratch` (device memory
 * of at least ibs_autotune_bytes() bytes, contents overwritten), keeps the
 * fastest in the plan, and writes the chosen indices to `choices`
 * (IBS_NUM_TUNE entries; may be NULL; -1 for a knob that does not apply to
 * this grid).  It synchronises `stream`, so it belongs to set-up, not to a
 * captured or timed sequence.  The plan must have been uploaded.
 * ibs_plan_set_tiles() restores choices saved earlier for the same grid
 * (entries < 0 keep the default; out-of-range entries are rejected). */
#define IBS_NUM_TUNE 2   /* 0: folded FP64 x transform, 1: folded FP64 z transform */
ibs_status ibs_autotune_bytes(ibs_plan plan, size_t *bytes);
ibs_status ibs_autotune(ibs_plan plan, void *scratch, size_t scratch_bytes, int32_t *choices,
                        void *stream);
ibs_status ibs_plan_set_tiles(ibs_plan plan, const int32_t *choices, int32_t n);

/* Thread-local text of the last error (never NULL). */
const char *ibs_last_error(void);

/* Library version string. */
const char *ibs_version(void);

#ifdef __cplusplus
}
#endif
#endif /* IBSOLVE_H */
