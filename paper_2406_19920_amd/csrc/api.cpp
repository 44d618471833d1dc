// C ABI of the solver library: validation, error layer, stage sequencing.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>

#include "ibs_internal.h"

namespace ibs {

static thread_local std::string g_err;

void set_error(const std::string &msg) { g_err = msg; }

ibs_status build_plan(const ibs_grid_desc &d, Plan *&out);

static size_t field_doubles(const Plan &p, int rows) { return (size_t)p.nz * rows * p.nx; }

static ibs_status hip_fail(hipError_t e, const char *where)
{
    set_error(std::string(where) + ": " + hipGetErrorString(e));
    return IBS_ERR_HIP;
}

static bool aligned32(const void *ptr) { return (reinterpret_cast<uintptr_t>(ptr) & 31u) == 0; }

static ibs_status check_plan(ibs_plan plan)
{
    if (!plan) { set_error("plan is NULL"); return IBS_ERR_INVALID_ARG; }
    Plan *p = reinterpret_cast<Plan *>(plan);
    if (!p->dev_const) { set_error("solver_plan_upload() has not been called"); return IBS_ERR_NOT_UPLOADED; }
    return IBS_OK;
}

// ---- optional live profile ------------------------------------------------
static hipEvent_t pool_get(Profile &pr)
{
    if (!pr.pool.empty()) {
        hipEvent_t e = pr.pool.back();
        pr.pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

static void prof_collect(Profile &pr)
{
    for (auto &r : pr.recs) {
        float ms = 0.f;
        if (hipEventSynchronize(r.stop) == hipSuccess &&
            hipEventElapsedTime(&ms, r.start, r.stop) == hipSuccess) {
            pr.ms[r.kid] += ms;
            pr.flops[r.kid] += r.flops;
            pr.bytes[r.kid] += r.bytes;
            pr.launches[r.kid] += 1;
        }
        pr.pool.push_back(r.start);
        pr.pool.push_back(r.stop);
    }
    pr.recs.clear();
}

// Launch through f(); when profiling, bracket it with events on stream s and
// book the algorithmic flops and bytes of the launch to kernel class kid.
template <typename F>
static hipError_t timed(Plan &p, int kid, double flops, double bytes, hipStream_t s, F f)
{
    if (!p.prof.on) return f();
    if (p.prof.recs.size() > 4096) prof_collect(p.prof);
    ProfRec r{kid, pool_get(p.prof), pool_get(p.prof), flops, bytes};
    if (!r.start || !r.stop) return f();
    hipEventRecord(r.start, s);
    hipError_t e = f();
    hipEventRecord(r.stop, s);
    p.prof.recs.push_back(r);
    return e;
}

// Profiling records events around launches, which must not happen while a
// batch is being captured into a graph.
ibs_status profile_suspend(ibs_plan plan, bool *was_on)
{
    Plan *p = reinterpret_cast<Plan *>(plan);
    *was_on = p->prof.on;
    p->prof.on = false;
    return IBS_OK;
}
void profile_resume(ibs_plan plan, bool was_on) { reinterpret_cast<Plan *>(plan)->prof.on = was_on; }

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Upper bound on the passes; the device stops earlier once the predicted
// error meets tol.  The Helmholtz systems are well conditioned (two passes
// reach ~1e-13); the pressure problem on large stretched grids may need a
// third.
static int default_passes(const Plan &p, bool poisson)
{
    if (p.desc.max_iter > 0) return p.desc.max_iter;
    return poisson ? 3 : 2;
}

// FP64 path: one FP64 scratch field per component.  Refined path: three
// FP32 fields per component (two transform buffers and the stored first
// iterate).
size_t field_bytes_for(const Plan &p, int op, int ncomp)
{
    const size_t per = p.desc.precision == IBS_FP64 ? sizeof(double) : 3 * sizeof(float);
    if (op == IBS_OP_POISSON) return field_doubles(p, p.ny) * per;
    return (size_t)ncomp * field_doubles(p, p.ny + 1) * per;
}

// Doubles of the state's reduction region: the update partials of every
// refinement pass (refined path), at least the residual() partials.
static size_t red_doubles(const Plan &p, int op, int ncomp)
{
    size_t n = 2 * (size_t)RESID_SLOTS;
    if (p.desc.precision != IBS_FP64) {
        const int nc = op == IBS_OP_POISSON ? 1 : ncomp;
        const size_t upd = (size_t)default_passes(p, op == IBS_OP_POISSON) * update_region(p, nc);
        n = upd > n ? upd : n;
    }
    return n;
}

// State layout (after the fields, 256-byte aligned): bmean[4], done[4],
// incompat[4], xsum[4][XSUM_SLOTS], compat[2 COMPAT_SLOTS], red[...],
// bmax[4][BMAX_SLOTS], scale[4].
size_t state_bytes_for(const Plan &p, int op, int ncomp)
{
    size_t o = align256(STATE_JOBS * sizeof(double));
    o += align256(2 * STATE_JOBS * sizeof(int));
    o += align256((size_t)STATE_JOBS * XSUM_SLOTS * sizeof(double));
    o += align256(2 * (size_t)COMPAT_SLOTS * sizeof(double));
    o += align256(red_doubles(p, op, ncomp) * sizeof(double));
    o += align256((size_t)STATE_JOBS * BMAX_SLOTS * sizeof(double));
    o += align256(STATE_JOBS * sizeof(double));
    return o;
}

State state_in(const Plan &p, void *work, int op, int ncomp)
{
    unsigned char *b = static_cast<unsigned char *>(work) + align256(field_bytes_for(p, op, ncomp));
    State st;
    st.bmean = reinterpret_cast<double *>(b);
    b += align256(STATE_JOBS * sizeof(double));
    st.done = reinterpret_cast<int *>(b);
    st.incompat = st.done + STATE_JOBS;
    b += align256(2 * STATE_JOBS * sizeof(int));
    st.xsum = reinterpret_cast<double *>(b);
    b += align256((size_t)STATE_JOBS * XSUM_SLOTS * sizeof(double));
    st.compat = reinterpret_cast<double *>(b);
    b += align256(2 * (size_t)COMPAT_SLOTS * sizeof(double));
    st.red = reinterpret_cast<double *>(b);
    st.red_count = red_doubles(p, op, ncomp);
    b += align256(st.red_count * sizeof(double));
    st.bmax = reinterpret_cast<double *>(b);
    b += align256((size_t)STATE_JOBS * BMAX_SLOTS * sizeof(double));
    st.scale = reinterpret_cast<double *>(b);
    return st;
}

size_t work_bytes_for(const Plan &p, int op, int ncomp)
{
    return align256(field_bytes_for(p, op, ncomp)) + state_bytes_for(p, op, ncomp);
}

static double total_cells(const JobSet &js, const Plan &p)
{
    double n = 0;
    for (int q = 0; q < js.n; ++q) n += (double)p.nz * js.j[q].rows * p.nx;
    return n;
}

// The five FP64 stages.  js.j[q].in holds the right-hand side; W[q] is the
// job's scratch field and X[q] its output.
static ibs_status run_fp64_pipeline_multi(Plan &p, JobSet js, double *const *W, double *const *X,
                                          const State &st, bool poisson, hipStream_t s)
{
    hipError_t e;
    const double cells = total_cells(js, p);
    // matrix-core flops per cell: 2n for the plain transform, n folded
    const bool fx = x_folds(p), fz = z_folds(p);
    const double xflop = (fx ? 1.0 : 2.0) * p.nx * cells, zflop = (fz ? 1.0 : 2.0) * p.nz * cells;
    const double rw = 16.0 * cells;
    const double *xb_f[NUM_XK], *xb_i[NUM_XK];
    for (int k = 0; k < NUM_XK; ++k) {
        xb_f[k] = blob_ptr(p, p.lay.bx_fwd[k]);
        xb_i[k] = blob_ptr(p, p.lay.bx_inv[k]);
    }
    const double *za_f[NUM_XK], *za_i[NUM_XK];
    for (int k = 0; k < NUM_XK; ++k) {
        za_f[k] = blob_ptr(p, p.lay.az_fwd[k]);
        za_i[k] = blob_ptr(p, p.lay.az_inv[k]);
    }
    auto xform = [&](bool inverse) {
        return fx ? launch_xfold_f64(js, p, inverse, s)
                  : launch_xgemm_f64(js, p.nz, p.nx, p.nx, inverse ? xb_i : xb_f, s);
    };
    auto zform = [&](bool inverse) {
        return fz ? launch_zfold_f64(js, p, inverse, s)
                  : launch_zgemm_f64(js, p.nz, p.nz, p.nx, inverse ? za_i : za_f, s);
    };
    for (int q = 0; q < js.n; ++q) js.j[q].out = W[q];
    e = timed(p, PK_XGEMM, xflop, rw, s, [&] { return xform(false); });
    if (e != hipSuccess) return hip_fail(e, "x forward");
    for (int q = 0; q < js.n; ++q) { js.j[q].in = W[q]; js.j[q].out = X[q]; }
    e = timed(p, PK_ZGEMM, zflop, rw, s, [&] { return zform(false); });
    if (e != hipSuccess) return hip_fail(e, "z forward");
    for (int q = 0; q < js.n; ++q) js.j[q].in = X[q];
    e = timed(p, PK_TRIDIAG, 20.0 * cells, rw, s, [&] { return launch_tridiag_f64(js, p, st, poisson, s); });
    if (e != hipSuccess) return hip_fail(e, "tridiagonal");
    for (int q = 0; q < js.n; ++q) { js.j[q].in = X[q]; js.j[q].out = W[q]; }
    e = timed(p, PK_ZGEMM, zflop, rw, s, [&] { return zform(true); });
    if (e != hipSuccess) return hip_fail(e, "z inverse");
    for (int q = 0; q < js.n; ++q) { js.j[q].in = W[q]; js.j[q].out = X[q]; }
    e = timed(p, PK_XGEMM, xflop, rw, s, [&] { return xform(true); });
    if (e != hipSuccess) return hip_fail(e, "x inverse");
    return IBS_OK;
}

static ibs_status run_fp64_pipeline(Plan &p, JobSet js, double *W, double *X, const State &st,
                                    bool poisson, hipStream_t s)
{
    return run_fp64_pipeline_multi(p, js, &W, &X, st, poisson, s);
}

// Refined path: pass 0 solves A x = b with the split-precision transforms;
// every later pass forms r = b - A x in FP64 (stored FP32), solves A d = r
// the same way and updates x += d in FP64.  The job records carry the
// right-hand side (b), the FP64 iterate (x) and three FP32 work fields each:
// two transform buffers and W3, which holds the first iterate in FP32 when a
// second pass follows (that pass then writes x = W3 + d).
// Every condition a refined launcher would refuse, checked on the host
// before anything of the call is enqueued.
static ibs_status check_refined(const Plan &p, int ncomp, int passes, const State &st)
{
    if (passes < 1 || passes > MAX_PASSES) {
        set_error("refinement passes out of range");
        return IBS_ERR_INVALID_ARG;
    }
    if ((size_t)(passes > 1 ? passes - 1 : 0) * update_region(p, ncomp) > st.red_count) {
        set_error("workspace state too small for the refinement passes");
        return IBS_ERR_WORKSPACE_TOO_SMALL;
    }
    return IBS_OK;
}

static ibs_status run_refined(Plan &p, SplitSet ss, float *const *W1, float *const *W2,
                              float *const *W3, const State &st, bool poisson, int passes, hipStream_t s)
{
    hipError_t e;
    double cells = 0;
    for (int q = 0; q < ss.n; ++q) cells += (double)p.nz * ss.j[q].rows * p.nx;
    // algorithmic flops per cell: 2n for the plain transform, n folded
    const double xfl = (x_folds_split(p) ? 1.0 : 2.0) * p.nx * cells;
    const double zfl = (z_folds_split(p) ? 1.0 : 2.0) * p.nz * cells;
    JobSet js{};
    js.n = ss.n;
    void *info[4];
    for (int q = 0; q < ss.n; ++q) {
        info[q] = ss.j[q].info;
        js.j[q].out = reinterpret_cast<double *>(W2[q]);
        js.j[q].in = js.j[q].out;
        js.j[q].rows = ss.j[q].rows;
        js.j[q].kind = ss.j[q].kind;
        js.j[q].xk = ss.j[q].xk;
        js.j[q].zk = ss.j[q].zk;
        js.j[q].c = ss.j[q].c;
    }
    // With a second pass to come, the first iterate is only FP32-accurate
    // and the second pass rewrites x: keep it in FP32 in W3 until then.
    const bool x32 = passes >= 2;
    for (int pass = 0; pass < passes; ++pass) {
        const bool xs32 = x32 && pass <= 1;
        for (int q = 0; q < ss.n; ++q)
            ss.j[q].xs = xs32 ? static_cast<void *>(W3[q]) : static_cast<void *>(ss.j[q].x);
        if (pass > 0) {
            if (pass == 1) {
                e = launch_residual_scale(ss, st, s);
                if (e != hipSuccess) return hip_fail(e, "residual scale");
            }
            for (int q = 0; q < ss.n; ++q) ss.j[q].r = W2[q];
            e = timed(p, PK_RESIDUAL, 10.0 * cells, (xs32 ? 16.0 : 20.0) * cells, s,
                      [&] { return launch_residual_f32(ss, p, st, pass, xs32, s); });
            if (e != hipSuccess) return hip_fail(e, "residual (refined)");
        }
        for (int q = 0; q < ss.n; ++q) {
            ss.j[q].in = pass == 0 ? static_cast<const void *>(ss.j[q].b) : static_cast<const void *>(W2[q]);
            ss.j[q].out = W1[q];
        }
        e = timed(p, PK_XGEMM_SPLIT, xfl, (pass == 0 ? 12.0 : 8.0) * cells, s,
                  [&] { return launch_split_xgemm(ss, p, st, false, pass == 0, 0, pass, s); });
        if (e != hipSuccess) return hip_fail(e, "x forward (split)");
        for (int q = 0; q < ss.n; ++q) { ss.j[q].in = W1[q]; ss.j[q].out = W2[q]; }
        e = timed(p, PK_ZGEMM_SPLIT, zfl, 8.0 * cells, s, [&] { return launch_split_zgemm(ss, p, st, false, pass, s); });
        if (e != hipSuccess) return hip_fail(e, "z forward (split)");
        for (int q = 0; q < ss.n; ++q) js.j[q].info = pass == 0 ? info[q] : nullptr;
        e = timed(p, PK_TRIDIAG_F32, 20.0 * cells, 8.0 * cells, s, [&] { return launch_tridiag_f32(js, p, st, poisson, pass, s); });
        if (e != hipSuccess) return hip_fail(e, "tridiagonal (refined)");
        for (int q = 0; q < ss.n; ++q) { ss.j[q].in = W2[q]; ss.j[q].out = W1[q]; }
        e = timed(p, PK_ZGEMM_SPLIT, zfl, 8.0 * cells, s, [&] { return launch_split_zgemm(ss, p, st, true, pass, s); });
        if (e != hipSuccess) return hip_fail(e, "z inverse (split)");
        for (int q = 0; q < ss.n; ++q) ss.j[q].in = W1[q];
        const int mode = pass == 0 ? (xs32 ? 3 : 1) : (xs32 ? 4 : 2);
        const double ub = mode == 3 ? 8.0 : (mode == 1 ? 12.0 : (mode == 4 ? 16.0 : 20.0));
        e = timed(p, PK_UPDATE, xfl, ub * cells, s,
                  [&] { return launch_split_xgemm(ss, p, st, true, false, mode, pass, s); });
        if (e != hipSuccess) return hip_fail(e, "x inverse + update (split)");
        // a one-pass solve has no error estimate: pass 0's check says so
        if (pass >= 1 || passes == 1) {
            e = launch_refine_check(ss, p, st, pass, s);
            if (e != hipSuccess) return hip_fail(e, "refinement check");
        }
    }
    return IBS_OK;
}

// Strict compatibility (Poisson): the weighted mean of b against its
// weighted rms, in FP64 on b itself; partials before the solve, the
// verdict after it (so that it overrides the status the solve wrote).
static ibs_status compat_begin(Plan &p, const double *b, const State &st, hipStream_t s)
{
    if (!p.desc.strict_compat) return IBS_OK;
    hipError_t e = launch_compat_partials(p, &b, 1, st, s);
    return e == hipSuccess ? IBS_OK : hip_fail(e, "compatibility partials");
}
static ibs_status compat_end(Plan &p, ibs_solve_info *info, const State &st, hipStream_t s)
{
    if (!p.desc.strict_compat) return IBS_OK;
    void *inf = info;
    hipError_t e = launch_compat_final(p, &inf, 1, st, s);
    return e == hipSuccess ? IBS_OK : hip_fail(e, "compatibility check");
}

}  // namespace ibs

using namespace ibs;

extern "C" {

const char *ibs_last_error(void) { return g_err.c_str(); }

const char *ibs_version(void) { return "ibsolve 0.1 (gfx950)"; }

ibs_status solver_plan(const ibs_grid_desc *desc, ibs_plan *out)
{
    try {
        if (!desc || !out) { set_error("desc and out must be non-NULL"); return IBS_ERR_INVALID_ARG; }
        *out = nullptr;
        if (desc->ny > 768) { set_error("ny must be <= 768"); return IBS_ERR_UNSUPPORTED; }
        Plan *p = nullptr;
        ibs_status st = build_plan(*desc, p);
        if (st != IBS_OK) return st;
        *out = reinterpret_cast<ibs_plan>(p);
        return IBS_OK;
    } catch (...) {
        set_error("host exception while building the plan");
        return IBS_ERR_INVALID_ARG;
    }
}

ibs_status solver_plan_bytes(ibs_plan plan, int32_t op, int32_t ncomp, size_t *const_bytes,
                             size_t *work_bytes)
{
    if (!plan) { set_error("plan is NULL"); return IBS_ERR_INVALID_ARG; }
    Plan *p = reinterpret_cast<Plan *>(plan);
    if (op < IBS_OP_POISSON || op > IBS_OP_HELMHOLTZ_W) { set_error("bad op"); return IBS_ERR_INVALID_ARG; }
    if (op != IBS_OP_POISSON && (ncomp < 1 || ncomp > 3)) { set_error("ncomp must be 1..3"); return IBS_ERR_INVALID_ARG; }
    if (const_bytes) *const_bytes = p->lay.total;
    if (work_bytes) *work_bytes = work_bytes_for(*p, op, ncomp);
    return IBS_OK;
}

ibs_status solver_plan_upload(ibs_plan plan, void *dev_const, size_t bytes, void *stream)
{
    if (!plan || !dev_const) { set_error("plan and dev_const must be non-NULL"); return IBS_ERR_INVALID_ARG; }
    Plan *p = reinterpret_cast<Plan *>(plan);
    if (bytes < p->lay.total) { set_error("constant buffer smaller than const_bytes"); return IBS_ERR_WORKSPACE_TOO_SMALL; }
    if ((reinterpret_cast<uintptr_t>(dev_const) & 255u) != 0) { set_error("dev_const must be 256-byte aligned"); return IBS_ERR_INVALID_ARG; }
    hipError_t e = hipMemcpyAsync(dev_const, p->blob.data(), p->lay.total, hipMemcpyHostToDevice,
                                  static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "solver_plan_upload");
    p->dev_const = dev_const;
    return IBS_OK;
}

ibs_status solver_plan_destroy(ibs_plan plan)
{
    Plan *p = reinterpret_cast<Plan *>(plan);
    if (p) {
        prof_collect(p->prof);
        for (hipEvent_t e : p->prof.pool) hipEventDestroy(e);
    }
    delete p;
    return IBS_OK;
}

ibs_status solve_poisson(ibs_plan plan, const double *b, double *phi, void *work, size_t work_bytes,
                         ibs_solve_info *info, void *stream)
{
    ibs_status chk = check_plan(plan);
    if (chk != IBS_OK) return chk;
    Plan &p = *reinterpret_cast<Plan *>(plan);
    if (!b || !phi || !work) { set_error("b, phi and work must be non-NULL"); return IBS_ERR_INVALID_ARG; }
    if (!aligned32(b) || !aligned32(phi) || !aligned32(work)) { set_error("device arrays must be 32-byte aligned"); return IBS_ERR_INVALID_ARG; }
    if (work_bytes < work_bytes_for(p, IBS_OP_POISSON, 1)) { set_error("workspace too small"); return IBS_ERR_WORKSPACE_TOO_SMALL; }
    hipStream_t s = static_cast<hipStream_t>(stream);
    const State st = state_in(p, work, IBS_OP_POISSON, 1);
    if (p.desc.precision != IBS_FP64) {
        if (phi == b) { set_error("the refined path needs phi distinct from b"); return IBS_ERR_INVALID_ARG; }
        ibs_status v = check_refined(p, 1, default_passes(p, true), st);
        if (v != IBS_OK) return v;
    }
    ibs_status r = compat_begin(p, b, st, s);
    if (r != IBS_OK) return r;
    if (p.desc.precision != IBS_FP64) {
        SplitSet ss{};
        ss.n = 1;
        ss.j[0].b = b;
        ss.j[0].x = phi;
        ss.j[0].rows = p.ny;
        ss.j[0].kind = KIND_P;
        ss.j[0].xk = XK_P;
        ss.j[0].zk = XK_P;
        ss.j[0].op = IBS_OP_POISSON;
        ss.j[0].c = 0.0;
        ss.j[0].info = info;
        float *W1 = static_cast<float *>(work);
        float *W2 = W1 + field_doubles(p, p.ny);
        float *W3 = W2 + field_doubles(p, p.ny);
        r = run_refined(p, ss, &W1, &W2, &W3, st, true, default_passes(p, true), s);
        return r != IBS_OK ? r : compat_end(p, info, st, s);
    }
    double *W = static_cast<double *>(work);
    JobSet js{};
    js.n = 1;
    js.j[0].rows = p.ny;
    js.j[0].kind = KIND_P;
    js.j[0].c = 0.0;
    js.j[0].info = info;
    // x forward: b -> W; z forward: W -> phi; pencils in place on phi;
    // z inverse: phi -> W; x inverse: W -> phi
    js.j[0].in = b; js.j[0].out = W;
    r = run_fp64_pipeline(p, js, W, phi, st, true, s);
    return r != IBS_OK ? r : compat_end(p, info, st, s);
}

ibs_status solve_helmholtz_batch(ibs_plan plan, int32_t ncomp, const int32_t *comp, const double *c,
                                 const double *const *r, double *const *x, void *work,
                                 size_t work_bytes, ibs_solve_info *info, void *stream)
{
    ibs_status chk = check_plan(plan);
    if (chk != IBS_OK) return chk;
    Plan &p = *reinterpret_cast<Plan *>(plan);
    if (ncomp < 1 || ncomp > 3) { set_error("ncomp must be 1..3"); return IBS_ERR_INVALID_ARG; }
    if (!comp || !c || !r || !x || !work) { set_error("comp, c, r, x and work must be non-NULL"); return IBS_ERR_INVALID_ARG; }
    if (work_bytes < work_bytes_for(p, IBS_OP_HELMHOLTZ_U, ncomp)) { set_error("workspace too small"); return IBS_ERR_WORKSPACE_TOO_SMALL; }
    if (!aligned32(work)) { set_error("work must be 32-byte aligned"); return IBS_ERR_INVALID_ARG; }
    JobSet js{};
    js.n = ncomp;
    const size_t stride = field_doubles(p, p.ny + 1);
    double *W = static_cast<double *>(work);
    for (int q = 0; q < ncomp; ++q) {
        if (comp[q] < 0 || comp[q] > 2) { set_error("comp must be 0 (u), 1 (v) or 2 (w)"); return IBS_ERR_INVALID_ARG; }
        if (!(c[q] >= 0.0) || !std::isfinite(c[q])) { set_error("c must be finite and >= 0"); return IBS_ERR_INVALID_ARG; }
        if (!r[q] || !x[q] || !aligned32(r[q]) || !aligned32(x[q])) { set_error("r[q], x[q] must be non-NULL and 32-byte aligned"); return IBS_ERR_INVALID_ARG; }
        js.j[q].rows = comp_rows(p, comp[q]);
        js.j[q].kind = comp_kind(p, comp[q]);
        js.j[q].xk = comp_xkind(p, comp[q]);
        js.j[q].zk = comp_zkind(p, comp[q]);
        js.j[q].c = c[q];
        js.j[q].info = info ? info + q : nullptr;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    const State st = state_in(p, work, IBS_OP_HELMHOLTZ_U, ncomp);
    if (p.desc.precision != IBS_FP64) {
        SplitSet ss{};
        ss.n = ncomp;
        float *W1[4], *W2[4], *W3[4];
        for (int q = 0; q < ncomp; ++q) {
            if (x[q] == r[q]) { set_error("the refined path needs x[q] distinct from r[q]"); return IBS_ERR_INVALID_ARG; }
            ss.j[q].b = r[q];
            ss.j[q].x = x[q];
            ss.j[q].rows = js.j[q].rows;
            ss.j[q].kind = js.j[q].kind;
            ss.j[q].xk = js.j[q].xk;
            ss.j[q].zk = js.j[q].zk;
            ss.j[q].op = comp[q] + 1;
            ss.j[q].c = c[q];
            ss.j[q].info = js.j[q].info;
            W1[q] = static_cast<float *>(work) + 3 * q * stride;
            W2[q] = W1[q] + stride;
            W3[q] = W2[q] + stride;
        }
        ibs_status v = check_refined(p, ncomp, default_passes(p, false), st);
        if (v != IBS_OK) return v;
        return run_refined(p, ss, W1, W2, W3, st, false, default_passes(p, false), s);
    }
    for (int q = 0; q < ncomp; ++q) { js.j[q].in = r[q]; js.j[q].out = W + q * stride; }
    double *Ws[4], *Xs[4];
    for (int q = 0; q < ncomp; ++q) { Ws[q] = W + q * stride; Xs[q] = x[q]; }
    return run_fp64_pipeline_multi(p, js, Ws, Xs, st, false, s);
}

ibs_status residual(ibs_plan plan, int32_t op, double c, const double *x, const double *b, double *r,
                    double *norms2, void *work, size_t work_bytes, void *stream)
{
    ibs_status chk = check_plan(plan);
    if (chk != IBS_OK) return chk;
    Plan &p = *reinterpret_cast<Plan *>(plan);
    if (op < IBS_OP_POISSON || op > IBS_OP_HELMHOLTZ_W) { set_error("bad op"); return IBS_ERR_INVALID_ARG; }
    if (!x || !b || !r) { set_error("x, b, r must be non-NULL"); return IBS_ERR_INVALID_ARG; }
    if (r == x) { set_error("r may not alias x"); return IBS_ERR_INVALID_ARG; }
    if (!std::isfinite(c)) { set_error("c must be finite"); return IBS_ERR_INVALID_ARG; }
    double *red = nullptr;
    if (norms2) {
        const int wop = op == IBS_OP_POISSON ? IBS_OP_POISSON : IBS_OP_HELMHOLTZ_U;
        if (!work || !aligned32(work)) { set_error("norms2 needs a 32-byte aligned workspace"); return IBS_ERR_INVALID_ARG; }
        if (work_bytes < work_bytes_for(p, wop, 1)) { set_error("workspace too small"); return IBS_ERR_WORKSPACE_TOO_SMALL; }
        red = state_in(p, work, wop, 1).red;
    }
    const double cells = (double)p.nz * comp_rows(p, op - 1) * p.nx;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = timed(p, PK_RESIDUAL, 10.0 * cells, 24.0 * cells, s,
                         [&] { return launch_residual(p, op, c, x, b, r, norms2, red, s); });
    if (e != hipSuccess) return hip_fail(e, "residual");
    return IBS_OK;
}

ibs_status ibs_divergence(ibs_plan plan, const double *u, const double *v, const double *w, double *b,
                          double scale, void *stream)
{
    ibs_status chk = check_plan(plan);
    if (chk != IBS_OK) return chk;
    Plan &p = *reinterpret_cast<Plan *>(plan);
    if (!u || !v || !w || !b) { set_error("u, v, w, b must be non-NULL"); return IBS_ERR_INVALID_ARG; }
    const double cells = (double)p.nz * p.ny * p.nx;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = timed(p, PK_DIVERGENCE, 7.0 * cells, 8.0 * (4.0 * cells + (double)p.nz * p.nx), s,
                         [&] { return launch_divergence(p, u, v, w, b, scale, s); });
    if (e != hipSuccess) return hip_fail(e, "divergence");
    return IBS_OK;
}

ibs_status ibs_correct(ibs_plan plan, const double *phi, double *u, double *v, double *w, double g,
                       double *pres, const double *lap_phi, double cp, void *stream)
{
    ibs_status chk = check_plan(plan);
    if (chk != IBS_OK) return chk;
    Plan &p = *reinterpret_cast<Plan *>(plan);
    if (!phi || !u || !v || !w) { set_error("phi, u, v, w must be non-NULL"); return IBS_ERR_INVALID_ARG; }
    if (pres && cp != 0.0 && !lap_phi) { set_error("lap_phi is required when p != NULL and cp != 0"); return IBS_ERR_INVALID_ARG; }
    const double cells = (double)p.nz * p.ny * p.nx;
    const double extra = pres ? (lap_phi && cp != 0.0 ? 24.0 : 16.0) * cells : 0.0;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = timed(p, PK_CORRECT, 9.0 * cells, 56.0 * cells + 16.0 * p.nz * p.nx + extra, s,
                         [&] { return launch_correct(p, phi, u, v, w, g, pres, lap_phi, cp, s); });
    if (e != hipSuccess) return hip_fail(e, "correct");
    return IBS_OK;
}

ibs_status ibs_wall_data(ibs_plan plan, int32_t op, double c, const double *lo, const double *hi,
                         double *rhs, void *stream)
{
    ibs_status chk = check_plan(plan);
    if (chk != IBS_OK) return chk;
    Plan &p = *reinterpret_cast<Plan *>(plan);
    if (op < IBS_OP_POISSON || op > IBS_OP_HELMHOLTZ_W) { set_error("bad op"); return IBS_ERR_INVALID_ARG; }
    if (!rhs) { set_error("rhs must be non-NULL"); return IBS_ERR_INVALID_ARG; }
    if (!std::isfinite(c) || (op != IBS_OP_POISSON && c < 0.0)) { set_error("c must be finite and >= 0"); return IBS_ERR_INVALID_ARG; }
    if (p.py) { set_error("wall data need walls; this plan is periodic in y"); return IBS_ERR_UNSUPPORTED; }
    if (!lo && !hi) return IBS_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = launch_wall_data(p, op, c, lo, hi, rhs, s);
    if (e != hipSuccess) return hip_fail(e, "wall data");
    return IBS_OK;
}

// Workspace of a sub-step: u^e and r (three fields each, v-shaped
// stride), b and phi (cell fields), then one solve's workspace (the larger
// of the Helmholtz batch of three and the Poisson solve; they run one
// after the other).
static size_t stage_field_doubles(const Plan &p) { return field_doubles(p, p.ny + 1); }
static size_t stage_solver_offset(const Plan &p)
{
    return align256((6 * stage_field_doubles(p) + 2 * field_doubles(p, p.ny)) * sizeof(double));
}
static size_t stage_solver_bytes(const Plan &p)
{
    const size_t h = work_bytes_for(p, IBS_OP_HELMHOLTZ_U, 3), q = work_bytes_for(p, IBS_OP_POISSON, 1);
    return h > q ? h : q;
}

ibs_status ibs_stage_bytes(ibs_plan plan, size_t *work_bytes)
{
    if (!plan || !work_bytes) { set_error("plan and work_bytes must be non-NULL"); return IBS_ERR_INVALID_ARG; }
    const Plan &p = *reinterpret_cast<Plan *>(plan);
    *work_bytes = stage_solver_offset(p) + stage_solver_bytes(p);
    return IBS_OK;
}

ibs_status ibs_rk_stage(ibs_plan plan, const ibs_rk_coef *coef, const ibs_stage_fields *f, void *work,
                        size_t work_bytes, ibs_solve_info *info, void *stream)
{
    ibs_status chk = check_plan(plan);
    if (chk != IBS_OK) return chk;
    Plan &p = *reinterpret_cast<Plan *>(plan);
    if (!coef || !f || !work) { set_error("coef, fields and work must be non-NULL"); return IBS_ERR_INVALID_ARG; }
    const ibs_rk_coef &k = *coef;
    const bool finite = std::isfinite(k.alpha) && std::isfinite(k.beta) && std::isfinite(k.gamma) &&
                        std::isfinite(k.zeta) && std::isfinite(k.dt) && std::isfinite(k.re);
    if (!finite || !(k.dt > 0.0) || !(k.re > 0.0) || !(k.beta >= 0.0) || !(k.alpha + k.beta > 0.0)) {
        set_error("coefficients must be finite with dt > 0, re > 0, beta >= 0 and alpha + beta > 0");
        return IBS_ERR_INVALID_ARG;
    }
    if (p.wx || p.wz) {
        set_error("the Runge-Kutta stage is built for periodic x and z (walls there are served by the solves)");
        return IBS_ERR_UNSUPPORTED;
    }
    const void *ptrs[] = {f->u, f->v, f->w, f->p, f->nu, f->nv, f->nw};
    for (const void *q : ptrs)
        if (!q || !aligned32(q)) { set_error("u, v, w, p, nu, nv, nw must be non-NULL and 32-byte aligned"); return IBS_ERR_INVALID_ARG; }
    if (f->nmarkers < 0 || (f->nmarkers > 0 && (!f->markers || !f->ud || !f->dvol))) {
        set_error("nmarkers must be >= 0, with markers, ud and dvol when it is positive");
        return IBS_ERR_INVALID_ARG;
    }
    if (f->nmarkers > 0) {
        const double h = p.desc.ly / p.ny;
        for (double d : p.dyc)
            if (std::fabs(d - h) > 1e-12 * h) {
                set_error("the immersed boundary needs a uniform spacing in y");
                return IBS_ERR_UNSUPPORTED;
            }
    }
    size_t need = 0;
    ibs_stage_bytes(plan, &need);
    if (work_bytes < need) { set_error("workspace smaller than ibs_stage_bytes()"); return IBS_ERR_WORKSPACE_TOO_SMALL; }
    if (!aligned32(work)) { set_error("work must be 32-byte aligned"); return IBS_ERR_INVALID_ARG; }

    double *W = static_cast<double *>(work);
    const size_t fs = stage_field_doubles(p);
    FsStage s{};
    s.alpha = k.alpha; s.beta = k.beta; s.gamma = k.gamma; s.zeta = k.zeta; s.dt = k.dt; s.re = k.re;
    s.u = f->u; s.v = f->v; s.w = f->w; s.p = f->p;
    s.nu = f->nu; s.nv = f->nv; s.nw = f->nw;
    s.ue = W; s.ve = W + fs; s.we = W + 2 * fs;
    s.ru = W + 3 * fs; s.rv = W + 4 * fs; s.rw = W + 5 * fs;
    s.markers = f->markers; s.ud = f->ud; s.dvol = f->dvol; s.force = f->force; s.nmarkers = f->nmarkers;
    double *b = W + 6 * fs, *phi = b + field_doubles(p, p.ny);
    void *sw = static_cast<unsigned char *>(work) + stage_solver_offset(p);
    const size_t swb = stage_solver_bytes(p);
    hipStream_t st = static_cast<hipStream_t>(stream);
    const double c = k.beta * k.dt / k.re, g = (k.alpha + k.beta) * k.dt;

    // algorithmic traffic of the explicit estimate: u, v, w, p (+ the previous
    // N when zeta != 0) read, r and N (+ u^e when markers interpolate it)
    // written, 8 bytes each per cell
    const double cells = (double)p.nx * p.ny * p.nz;
    const double ebytes = 8.0 * cells * (10.0 + (k.zeta != 0.0 ? 3.0 : 0.0) + (f->nmarkers > 0 ? 3.0 : 0.0));
    hipError_t e = timed(p, PK_EXPLICIT, 150.0 * cells, ebytes, st,
                         [&] { return launch_explicit(p, s, st); });   // (a) and the rhs of (e)
    if (e != hipSuccess) return hip_fail(e, "explicit estimate");
    // per marker and component: 27 reads and 27 atomic updates
    const double ibytes = (double)f->nmarkers * 3 * 27 * 24.0;
    e = timed(p, PK_IBM, (double)f->nmarkers * 3 * 27 * 8.0, ibytes, st,
              [&] { return launch_ibm(p, s, st); });                  // (b)-(d), into the rhs
    if (e != hipSuccess) return hip_fail(e, "immersed boundary");
    const int32_t comps[3] = {0, 1, 2};
    const double cs[3] = {c, c, c};
    const double *rs[3] = {s.ru, s.rv, s.rw};
    double *xs[3] = {f->u, f->v, f->w};
    ibs_status r = solve_helmholtz_batch(plan, 3, comps, cs, rs, xs, sw, swb, info, stream);   // (e)
    if (r != IBS_OK) return r;
    r = ibs_divergence(plan, f->u, f->v, f->w, b, 1.0 / g, stream);                          // rhs of (f)
    if (r != IBS_OK) return r;
    r = solve_poisson(plan, b, phi, sw, swb, info ? info + 3 : nullptr, stream);              // (f)
    if (r != IBS_OK) return r;
    return ibs_correct(plan, phi, f->u, f->v, f->w, g, f->p, b, c, stream);                  // (g), (h)
}

ibs_status ibs_profile(ibs_plan plan, int32_t enable)
{
    if (!plan) { set_error("plan is NULL"); return IBS_ERR_INVALID_ARG; }
    Plan &p = *reinterpret_cast<Plan *>(plan);
    prof_collect(p.prof);
    for (int k = 0; k < NUM_PK; ++k) {
        p.prof.ms[k] = 0; p.prof.flops[k] = 0; p.prof.bytes[k] = 0; p.prof.launches[k] = 0;
    }
    p.prof.on = enable != 0;
    return IBS_OK;
}

ibs_status ibs_profile_read(ibs_plan plan, int32_t kernel, double *ms, int64_t *launches,
                            double *flops, double *bytes)
{
    if (!plan || kernel < 0 || kernel >= NUM_PK) { set_error("bad plan or kernel class"); return IBS_ERR_INVALID_ARG; }
    Plan &p = *reinterpret_cast<Plan *>(plan);
    prof_collect(p.prof);
    if (ms) *ms = p.prof.ms[kernel];
    if (launches) *launches = p.prof.launches[kernel];
    if (flops) *flops = p.prof.flops[kernel];
    if (bytes) *bytes = p.prof.bytes[kernel];
    return IBS_OK;
}

static size_t autotune_doubles(const Plan &p) { return 2 * (size_t)p.nz * (p.ny + 1) * p.nx; }

ibs_status ibs_autotune_bytes(ibs_plan plan, size_t *bytes)
{
    if (!plan || !bytes) { set_error("plan and bytes must be non-NULL"); return IBS_ERR_INVALID_ARG; }
    *bytes = autotune_doubles(*reinterpret_cast<Plan *>(plan)) * sizeof(double);
    return IBS_OK;
}

ibs_status ibs_autotune(ibs_plan plan, void *scratch, size_t scratch_bytes, int32_t *choices,
                        void *stream_ptr)
{
    hipStream_t stream = static_cast<hipStream_t>(stream_ptr);
    if (!plan || !scratch) { set_error("plan and scratch must be non-NULL"); return IBS_ERR_INVALID_ARG; }
    Plan &p = *reinterpret_cast<Plan *>(plan);
    if (!p.dev_const) { set_error("solver_plan_upload() has not been called"); return IBS_ERR_NOT_UPLOADED; }
    const size_t nd = autotune_doubles(p);
    if (scratch_bytes < nd * sizeof(double)) {
        set_error("scratch smaller than ibs_autotune_bytes()");
        return IBS_ERR_WORKSPACE_TOO_SMALL;
    }
    double *A = static_cast<double *>(scratch), *B = A + nd / 2;
    hipError_t e = hipMemsetAsync(scratch, 0, nd * sizeof(double), stream);
    if (e != hipSuccess) return hip_fail(e, "autotune scratch clear");
    // one pressure-sized field, forward then inverse transform per trial
    JobSet js{};
    js.n = 1;
    js.j[0].rows = p.ny;
    js.j[0].kind = KIND_P;
    hipEvent_t ev[2];
    if ((e = hipEventCreate(&ev[0])) != hipSuccess) return hip_fail(e, "autotune event");
    if ((e = hipEventCreate(&ev[1])) != hipSuccess) {
        hipEventDestroy(ev[0]);
        return hip_fail(e, "autotune event");
    }
    struct Knob { int id; bool applies; hipError_t (*launch)(const JobSet &, const Plan &, bool, hipStream_t); };
    const Knob knobs[NUM_TUNE] = {{TUNE_XFOLD, x_folds(p), launch_xfold_f64},
                                  {TUNE_ZFOLD, z_folds(p), launch_zfold_f64}};
    ibs_status st = IBS_OK;
    // candidates timed in interleaved rounds, each keeping its fastest
    // round, so that a transient slowdown of one measurement (clock ramp,
    // another process) does not decide between candidates a few per cent
    // apart
    constexpr int ROUNDS = 3;
    for (const Knob &k : knobs) {
        if (!k.applies) { p.tune[k.id] = -1; continue; }
        std::vector<float> cand_ms(fold_candidates(), 0.f);
        for (int trial_no = 0; trial_no < ROUNDS * fold_candidates() && st == IBS_OK; ++trial_no) {
            const int round = trial_no / fold_candidates(), cand = trial_no % fold_candidates();
            p.tune[k.id] = cand;
            auto trial = [&](int reps) {
                hipError_t r = hipSuccess;
                for (int i = 0; i < reps && r == hipSuccess; ++i) {
                    js.j[0].in = A; js.j[0].out = B;
                    r = k.launch(js, p, false, stream);
                    if (r != hipSuccess) break;
                    js.j[0].in = B; js.j[0].out = A;
                    r = k.launch(js, p, true, stream);
                }
                return r;
            };
            float ms = 0.f;
            if ((e = trial(1)) != hipSuccess || (e = hipEventRecord(ev[0], stream)) != hipSuccess ||
                (e = trial(3)) != hipSuccess || (e = hipEventRecord(ev[1], stream)) != hipSuccess ||
                (e = hipEventSynchronize(ev[1])) != hipSuccess ||
                (e = hipEventElapsedTime(&ms, ev[0], ev[1])) != hipSuccess) {
                st = hip_fail(e, "autotune trial");
                break;
            }
            if (round == 0 || ms < cand_ms[cand]) cand_ms[cand] = ms;
        }
        int best = 0;
        for (int cand = 1; cand < fold_candidates(); ++cand)
            if (cand_ms[cand] < cand_ms[best]) best = cand;
        p.tune[k.id] = best;
    }
    hipEventDestroy(ev[0]);
    hipEventDestroy(ev[1]);
    if (st != IBS_OK) return st;
    if (choices)
        for (int i = 0; i < NUM_TUNE; ++i) choices[i] = p.tune[i];
    return IBS_OK;
}

ibs_status ibs_plan_set_tiles(ibs_plan plan, const int32_t *choices, int32_t n)
{
    if (!plan || !choices || n < 0 || n > NUM_TUNE) { set_error("bad plan, choices or count"); return IBS_ERR_INVALID_ARG; }
    Plan &p = *reinterpret_cast<Plan *>(plan);
    for (int i = 0; i < n; ++i)
        if (choices[i] >= fold_candidates()) { set_error("tile choice out of range"); return IBS_ERR_INVALID_ARG; }
    for (int i = 0; i < n; ++i) p.tune[i] = choices[i] < 0 ? -1 : choices[i];
    return IBS_OK;
}

ibs_status ibs_plan_export(ibs_plan plan, int32_t table, double *out, size_t *n)
{
    if (!plan || !n) { set_error("plan and n must be non-NULL"); return IBS_ERR_INVALID_ARG; }
    Plan &p = *reinterpret_cast<Plan *>(plan);
    const std::vector<double> *v = nullptr;
    switch (table) {
    case 0: v = &p.yf; break;
    case 1: v = &p.qx[XK_P]; break;
    case 2: v = &p.qz[XK_P]; break;
    case 3: v = &p.lam_x[XK_P]; break;
    case 4: v = &p.lam_z[XK_P]; break;
    default:
        if (table >= 5 && table < 5 + 3 * NUM_KINDS) {
            const int kd = (table - 5) / 3, which = (table - 5) % 3;
            v = which == 0 ? &p.lo[kd] : (which == 1 ? &p.di[kd] : &p.up[kd]);
        } else if (table >= 5 + 3 * NUM_KINDS && table < 5 + 3 * NUM_KINDS + 8) {
            // the x bases and eigenvalues of v/w (XK_C) and u (XK_F), then
            // the z ones of u/v (XK_C) and w (XK_F)
            const int t = (table - 5 - 3 * NUM_KINDS) % 4;
            const bool zax = table - 5 - 3 * NUM_KINDS >= 4;
            const int k = (t % 2 == 0) ? XK_C : XK_F;
            v = t < 2 ? (zax ? &p.qz[k] : &p.qx[k]) : (zax ? &p.lam_z[k] : &p.lam_x[k]);
        } else if (table >= 25 && table < 25 + 2 * NUM_XK) {
            // the inverse bases of kind XK_P, XK_C, XK_F: x, then z
            const int k = (table - 25) % NUM_XK;
            v = table - 25 < NUM_XK ? &p.gx[k] : &p.gz[k];
        } else if (table == 31) {
            v = &p.xf;
        } else if (table == 32) {
            v = &p.zf;
        }
    }
    if (!v) { set_error("unknown table"); return IBS_ERR_INVALID_ARG; }
    if (!out) { *n = v->size(); return IBS_OK; }
    if (*n != v->size()) { set_error("n does not match the table length"); return IBS_ERR_INVALID_ARG; }
    std::memcpy(out, v->data(), v->size() * sizeof(double));
    return IBS_OK;
}

}  // extern "C"
