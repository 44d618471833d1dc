// Batched execution of many independent solves as one HIP graph.
//
// ibs_batch_build() records every job's launches once (stream capture) into
// a graph whose independent branches ("lanes") the GPU may run side by
// side; ibs_batch_launch() replays the whole batch with one hipGraphLaunch.
// All solves that use the same workspace are placed on the same lane (the
// workspace holds a call's fields and mutable state, so calls sharing it
// must not overlap); the workspaces are dealt to the lanes by a schedule
// policy (balanced by work, or in submission order), and ibs_batch_autotune()
// times the candidate lane counts and policies on the device and returns
// the fastest.  The plans' device constants are only read, so jobs of one
// plan with distinct workspaces may run side by side.  Every schedule runs
// each job's launches in the same order on its own workspace, so the
// results do not depend on the schedule.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "ibs_internal.h"
#include "multigrid.h"

namespace ibs {
ibs_status profile_suspend(ibs_plan plan, bool *was_on);
void profile_resume(ibs_plan plan, bool was_on);
}  // namespace ibs

using namespace ibs;

struct ibs_batch_s {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int njobs = 0;
    int nlanes = 0;
    void *dev = nullptr;   // multi-grid batches: job table, work lists, tables
};

static ibs_status fail_hip(hipError_t e, const char *where)
{
    set_error(std::string(where) + ": " + hipGetErrorString(e));
    return IBS_ERR_HIP;
}

// Lane of every workspace under a schedule policy (IBS_SCHED_*).
static std::map<void *, int> assign_lanes(const ibs_batch_job *jobs, int njobs, int nlanes, int policy,
                                          int &L)
{
    std::map<void *, double> cost;
    std::vector<void *> first_seen;
    for (int q = 0; q < njobs; ++q) {
        Plan *p = reinterpret_cast<Plan *>(jobs[q].plan);
        const double cells = (double)p->nx * p->ny * p->nz;
        if (!cost.count(jobs[q].work)) first_seen.push_back(jobs[q].work);
        cost[jobs[q].work] += cells * (jobs[q].op == IBS_OP_POISSON ? 1 : jobs[q].ncomp);
    }
    L = std::min<int>(nlanes, (int)first_seen.size());
    std::map<void *, int> lane_of;
    if (policy == IBS_SCHED_IN_ORDER) {
        for (size_t w = 0; w < first_seen.size(); ++w) lane_of[first_seen[w]] = (int)(w % L);
        return lane_of;
    }
    // balanced: largest workspace first, each to the least loaded lane
    std::vector<std::pair<double, void *>> order;
    for (void *w : first_seen) order.push_back({cost[w], w});
    std::stable_sort(order.begin(), order.end(), [](auto &a, auto &b) { return a.first > b.first; });
    std::vector<double> load(L, 0.0);
    for (auto &o : order) {
        int best = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        lane_of[o.second] = best;
        load[best] += o.first;
    }
    return lane_of;
}

static ibs_status check_jobs(const ibs_batch_job *jobs, int32_t njobs)
{
    for (int q = 0; q < njobs; ++q) {
        const ibs_batch_job &j = jobs[q];
        if (!j.plan) { set_error("job without a plan"); return IBS_ERR_INVALID_ARG; }
        if (j.op != IBS_OP_POISSON && j.op != IBS_OP_HELMHOLTZ_U) { set_error("job op must be IBS_OP_POISSON or IBS_OP_HELMHOLTZ_U"); return IBS_ERR_INVALID_ARG; }
        if (j.op == IBS_OP_HELMHOLTZ_U && (j.ncomp < 1 || j.ncomp > 3)) { set_error("Helmholtz job ncomp must be 1..3"); return IBS_ERR_INVALID_ARG; }
    }
    return IBS_OK;
}

extern "C" {

ibs_status ibs_batch_build(const ibs_batch_job *jobs, int32_t njobs, int32_t nlanes, ibs_batch *out)
{
    return ibs_batch_build_sched(jobs, njobs, nlanes, IBS_SCHED_BALANCED, out);
}

ibs_status ibs_batch_build_sched(const ibs_batch_job *jobs, int32_t njobs, int32_t nlanes, int32_t policy,
                                 ibs_batch *out)
{
    if (!jobs || njobs < 1 || !out || nlanes < 1 || nlanes > 64) {
        set_error("jobs, out must be non-NULL, njobs >= 1, nlanes in [1, 64]");
        return IBS_ERR_INVALID_ARG;
    }
    if (policy != IBS_SCHED_BALANCED && policy != IBS_SCHED_IN_ORDER) {
        set_error("unknown schedule policy");
        return IBS_ERR_INVALID_ARG;
    }
    *out = nullptr;
    ibs_status chk = check_jobs(jobs, njobs);
    if (chk != IBS_OK) return chk;
    std::map<ibs_plan, int> plans;
    for (int q = 0; q < njobs; ++q) plans[jobs[q].plan] = 1;
    int L = 0;
    std::map<void *, int> lane_of = assign_lanes(jobs, njobs, nlanes, policy, L);

    hipStream_t cap = nullptr;
    std::vector<hipStream_t> lanes(L, nullptr);
    std::vector<hipEvent_t> evs(L + 1, nullptr);
    hipError_t e;
    ibs_status st = IBS_OK;
    ibs_batch_s *b = new ibs_batch_s();
    std::vector<std::pair<ibs_plan, bool>> suspended;
    for (auto &kv : plans) {
        bool was = false;
        profile_suspend(kv.first, &was);
        suspended.push_back({kv.first, was});
    }
    auto cleanup = [&]() {
        for (auto &s : lanes) if (s) hipStreamDestroy(s);
        if (cap) hipStreamDestroy(cap);
        for (auto &ev : evs) if (ev) hipEventDestroy(ev);
        for (auto &sp : suspended) profile_resume(sp.first, sp.second);
    };
    if ((e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking)) != hipSuccess) { st = fail_hip(e, "capture stream"); goto done; }
    for (int l = 0; l < L; ++l)
        if ((e = hipStreamCreateWithFlags(&lanes[l], hipStreamNonBlocking)) != hipSuccess) { st = fail_hip(e, "lane stream"); goto done; }
    for (auto &ev : evs)
        if ((e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess) { st = fail_hip(e, "event"); goto done; }
    if ((e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal)) != hipSuccess) { st = fail_hip(e, "begin capture"); goto done; }
    hipEventRecord(evs[L], cap);
    for (int l = 0; l < L; ++l) hipStreamWaitEvent(lanes[l], evs[L], 0);
    for (int q = 0; q < njobs && st == IBS_OK; ++q) {
        const ibs_batch_job &j = jobs[q];
        hipStream_t s = lanes[lane_of[j.work]];
        if (j.op == IBS_OP_POISSON) {
            st = solve_poisson(j.plan, j.rhs[0], j.x[0], j.work, j.work_bytes, j.info, s);
        } else {
            st = solve_helmholtz_batch(j.plan, j.ncomp, j.comp, j.c, j.rhs, j.x, j.work, j.work_bytes,
                                       j.info, s);
        }
        if (st != IBS_OK) set_error(std::string("batch job ") + std::to_string(q) + ": " + ibs_last_error());
    }
    for (int l = 0; l < L; ++l) {
        hipEventRecord(evs[l], lanes[l]);
        hipStreamWaitEvent(cap, evs[l], 0);
    }
    {
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(cap, &g);
        if (st == IBS_OK && e != hipSuccess) st = fail_hip(e, "end capture");
        if (st != IBS_OK) {
            if (g) hipGraphDestroy(g);
            goto done;
        }
        b->graph = g;
    }
    if ((e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0)) != hipSuccess) { st = fail_hip(e, "instantiate"); goto done; }
    b->njobs = njobs;
    b->nlanes = L;
done:
    cleanup();
    if (st != IBS_OK) {
        if (b->exec) hipGraphExecDestroy(b->exec);
        if (b->graph) hipGraphDestroy(b->graph);
        delete b;
        return st;
    }
    *out = b;
    return IBS_OK;
}

ibs_status ibs_batch_launch(ibs_batch batch, void *stream)
{
    if (!batch || !batch->exec) { set_error("batch is NULL"); return IBS_ERR_INVALID_ARG; }
    hipError_t e = hipGraphLaunch(batch->exec, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return fail_hip(e, "graph launch");
    return IBS_OK;
}

ibs_status ibs_batch_destroy(ibs_batch batch)
{
    if (!batch) return IBS_OK;
    if (batch->exec) hipGraphExecDestroy(batch->exec);
    if (batch->graph) hipGraphDestroy(batch->graph);
    if (batch->dev) hipFree(batch->dev);
    delete batch;
    return IBS_OK;
}

// Multi-grid batch: the fields of every job in one device job table, one
// work list per stage kind (x transforms: 64 x 64 tiles of rows x modes; z
// transforms: 64 x 64 tiles of modes x columns; pencils: 64-pencil runs of
// a plane), the plain transform tables of every (plan, axis, kind,
// direction) used, and a graph of the five stage launches.
ibs_status ibs_batch_build_multigrid(const ibs_batch_job *jobs, int32_t njobs, ibs_batch *out)
{
    if (!jobs || njobs < 1 || !out) {
        set_error("jobs, out must be non-NULL, njobs >= 1");
        return IBS_ERR_INVALID_ARG;
    }
    *out = nullptr;
    ibs_status chk = check_jobs(jobs, njobs);
    if (chk != IBS_OK) return chk;
    std::map<void *, int> works;
    for (int q = 0; q < njobs; ++q) {
        const ibs_batch_job &j = jobs[q];
        const Plan &p = *reinterpret_cast<const Plan *>(j.plan);
        const std::string who = "multi-grid job " + std::to_string(q) + ": ";
        if (!p.dev_const) { set_error(who + "plan not uploaded"); return IBS_ERR_NOT_UPLOADED; }
        if (p.desc.precision != IBS_FP64 || p.py || p.desc.strict_compat) {
            set_error(who + "multi-grid batches take FP64 plans with walls in y and strict_compat 0");
            return IBS_ERR_UNSUPPORTED;
        }
        const int nc = j.op == IBS_OP_POISSON ? 1 : j.ncomp;
        if (!j.work || j.work_bytes < work_bytes_for(p, j.op, nc)) {
            set_error(who + "workspace missing or too small");
            return IBS_ERR_WORKSPACE_TOO_SMALL;
        }
        if (works.count(j.work)) {
            set_error(who + "multi-grid jobs run side by side and need workspaces of their own");
            return IBS_ERR_INVALID_ARG;
        }
        works[j.work] = q;
        auto aligned = [](const void *ptr) { return (reinterpret_cast<uintptr_t>(ptr) & 31u) == 0; };
        if (!aligned(j.work)) { set_error(who + "work must be 32-byte aligned"); return IBS_ERR_INVALID_ARG; }
        for (int k = 0; k < nc; ++k) {
            if (!j.rhs[k] || !j.x[k]) { set_error(who + "rhs and x must be non-NULL"); return IBS_ERR_INVALID_ARG; }
            if (!aligned(j.rhs[k]) || !aligned(j.x[k])) {
                set_error(who + "rhs and x must be 32-byte aligned");
                return IBS_ERR_INVALID_ARG;
            }
            if (j.op != IBS_OP_POISSON &&
                (j.comp[k] < 0 || j.comp[k] > 2 || !(j.c[k] >= 0.0) || !std::isfinite(j.c[k]))) {
                set_error(who + "comp must be 0..2 and c finite and >= 0");
                return IBS_ERR_INVALID_ARG;
            }
        }
    }

    // host images: tables first (deduplicated), then fields and work lists
    std::vector<double> tables;
    std::map<std::tuple<const Plan *, int, int, int>, size_t> table_at;   // (plan, axis, kind, inv) -> doubles
    auto table = [&](const Plan &p, bool z, int kind, bool inv) {
        const auto key = std::make_tuple(&p, z ? 1 : 0, kind, inv ? 1 : 0);
        auto it = table_at.find(key);
        if (it != table_at.end()) return it->second;
        std::vector<double> t;
        plain_transform_table(p, z, kind, inv, t);
        const size_t at = tables.size();
        tables.insert(tables.end(), t.begin(), t.end());
        tables.resize((tables.size() + 31) & ~size_t(31));   // 256-byte aligned tables
        table_at[key] = at;
        return at;
    };
    struct Pending { MgField f; size_t xf, xi, zf, zi; };
    std::vector<Pending> fields;
    for (int q = 0; q < njobs; ++q) {
        const ibs_batch_job &j = jobs[q];
        const Plan &p = *reinterpret_cast<const Plan *>(j.plan);
        const bool pois = j.op == IBS_OP_POISSON;
        const int nc = pois ? 1 : j.ncomp;
        for (int k = 0; k < nc; ++k) {
            const int comp = pois ? -1 : j.comp[k];
            const int kind = pois ? KIND_P : comp_kind(p, comp);
            const int xk = pois ? XK_P : comp_xkind(p, comp);
            const int zk = pois ? XK_P : comp_zkind(p, comp);
            Pending e{};
            MgField &f = e.f;
            f.in = j.rhs[k];
            f.out = j.x[k];
            f.work = static_cast<double *>(j.work) + (size_t)k * p.nz * (p.ny + 1) * p.nx;
            f.lam_x = blob_ptr(p, p.lay.lam_x[xk]);
            f.lam_z = blob_ptr(p, p.lay.lam_z[zk]);
            f.lo = blob_ptr(p, p.lay.lo[kind]);
            f.di = blob_ptr(p, p.lay.di[kind]);
            f.up = blob_ptr(p, p.lay.up[kind]);
            f.wy = blob_ptr(p, p.lay.wy);
            f.info = j.info ? j.info + k : nullptr;
            f.c = pois ? 0.0 : j.c[k];
            f.inv_sqrt_nxnz = 1.0 / std::sqrt((double)p.nx * (double)p.nz);
            f.nx = p.nx; f.ny = p.ny; f.nz = p.nz;
            f.rows = p.rows[kind];
            f.kind = kind;
            f.poisson = pois ? 1 : 0;
            e.xf = table(p, false, xk, false);
            e.xi = table(p, false, xk, true);
            e.zf = table(p, true, zk, false);
            e.zi = table(p, true, zk, true);
            fields.push_back(e);
        }
    }
    std::vector<int4> xitems, zitems, titems;
    std::vector<size_t> cpt_at;   // doubles from the start of the factor region
    size_t cpt_doubles = 0;
    for (size_t fi = 0; fi < fields.size(); ++fi) {
        const MgField &f = fields[fi].f;
        cpt_at.push_back(cpt_doubles);
        cpt_doubles += ((size_t)f.nz * f.rows * f.nx + 31) & ~size_t(31);
    }
    for (size_t fi = 0; fi < fields.size(); ++fi) {
        const MgField &f = fields[fi].f;
        const int trows = f.rows - skip_first_row(f.kind);
        for (int r = 0; r < f.nz * trows; r += 16 * MG_WM)
            for (int c = 0; c < f.nx; c += 64) xitems.push_back(make_int4((int)fi, r, c, 0));
        for (int r = 0; r < f.nz; r += 16 * MG_WM)
            for (int c = 0; c < trows * f.nx; c += 64) zitems.push_back(make_int4((int)fi, r, c, 0));
        for (int c = 0; c < f.nz; ++c)
            for (int a = 0; a < f.nx; a += 64) titems.push_back(make_int4((int)fi, c, a, 0));
    }
    auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
    const size_t o_tab = 0;
    const size_t o_fld = al(o_tab + tables.size() * sizeof(double));
    const size_t o_x = al(o_fld + fields.size() * sizeof(MgField));
    const size_t o_z = al(o_x + xitems.size() * sizeof(int4));
    const size_t o_t = al(o_z + zitems.size() * sizeof(int4));
    const size_t o_cp = al(o_t + titems.size() * sizeof(int4));
    const size_t total = al(o_cp + cpt_doubles * sizeof(double));
    const size_t upload = o_cp;   // the factor region is filled on the device

    ibs_batch_s *b = new ibs_batch_s();
    hipStream_t cap = nullptr;
    hipError_t e;
    ibs_status st = IBS_OK;
    std::vector<unsigned char> img(upload, 0);
    unsigned char *dev = nullptr;
    if ((e = hipMalloc(&b->dev, total)) != hipSuccess) { st = fail_hip(e, "multi-grid buffer"); goto fail; }
    dev = static_cast<unsigned char *>(b->dev);
    std::memcpy(img.data() + o_tab, tables.data(), tables.size() * sizeof(double));
    for (size_t fi = 0; fi < fields.size(); ++fi) {
        MgField f = fields[fi].f;
        f.xfwd = reinterpret_cast<const double *>(dev + o_tab) + fields[fi].xf;
        f.xinv = reinterpret_cast<const double *>(dev + o_tab) + fields[fi].xi;
        f.zfwd = reinterpret_cast<const double *>(dev + o_tab) + fields[fi].zf;
        f.zinv = reinterpret_cast<const double *>(dev + o_tab) + fields[fi].zi;
        f.cpt = reinterpret_cast<double *>(dev + o_cp) + cpt_at[fi];
        std::memcpy(img.data() + o_fld + fi * sizeof(MgField), &f, sizeof(MgField));
    }
    std::memcpy(img.data() + o_x, xitems.data(), xitems.size() * sizeof(int4));
    std::memcpy(img.data() + o_z, zitems.data(), zitems.size() * sizeof(int4));
    std::memcpy(img.data() + o_t, titems.data(), titems.size() * sizeof(int4));
    if ((e = hipMemcpy(b->dev, img.data(), upload, hipMemcpyHostToDevice)) != hipSuccess) { st = fail_hip(e, "multi-grid upload"); goto fail; }
    if ((e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking)) != hipSuccess) { st = fail_hip(e, "capture stream"); goto fail; }
    // the pencils' factors, once (they depend on the systems, not the data)
    if ((e = launch_multigrid_stage(MG_FACTOR, reinterpret_cast<const MgField *>(dev + o_fld),
                                    reinterpret_cast<const int4 *>(dev + o_t), (int)titems.size(), cap)) != hipSuccess ||
        (e = hipStreamSynchronize(cap)) != hipSuccess) {
        st = fail_hip(e, "multi-grid factors");
        goto fail;
    }
    if ((e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal)) != hipSuccess) { st = fail_hip(e, "begin capture"); goto fail; }
    {
        const MgField *fl = reinterpret_cast<const MgField *>(dev + o_fld);
        const int4 *xi = reinterpret_cast<const int4 *>(dev + o_x);
        const int4 *zi = reinterpret_cast<const int4 *>(dev + o_z);
        const int4 *ti = reinterpret_cast<const int4 *>(dev + o_t);
        const int nx_ = (int)xitems.size(), nz_ = (int)zitems.size(), nt_ = (int)titems.size();
        hipError_t le = launch_multigrid_stage(MG_X_FWD, fl, xi, nx_, cap);
        if (le == hipSuccess) le = launch_multigrid_stage(MG_Z_FWD, fl, zi, nz_, cap);
        if (le == hipSuccess) le = launch_multigrid_stage(MG_TRI, fl, ti, nt_, cap);
        if (le == hipSuccess) le = launch_multigrid_stage(MG_Z_INV, fl, zi, nz_, cap);
        if (le == hipSuccess) le = launch_multigrid_stage(MG_X_INV, fl, xi, nx_, cap);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(cap, &g);
        if (le != hipSuccess) { if (g) hipGraphDestroy(g); st = fail_hip(le, "multi-grid stage launch"); goto fail; }
        if (e != hipSuccess) { st = fail_hip(e, "end capture"); goto fail; }
        b->graph = g;
    }
    if ((e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0)) != hipSuccess) { st = fail_hip(e, "instantiate"); goto fail; }
    hipStreamDestroy(cap);
    b->njobs = njobs;
    b->nlanes = 1;
    *out = b;
    return IBS_OK;
fail:
    if (cap) hipStreamDestroy(cap);
    ibs_batch_destroy(b);
    return st;
}

ibs_status ibs_batch_autotune(const ibs_batch_job *jobs, int32_t njobs, int32_t reps, int32_t *nlanes,
                              int32_t *policy, float *ms, void *stream)
{
    if (!jobs || njobs < 1 || reps < 1 || reps > 100 || !nlanes || !policy) {
        set_error("jobs, nlanes, policy must be non-NULL, njobs >= 1, reps in [1, 100]");
        return IBS_ERR_INVALID_ARG;
    }
    ibs_status chk = check_jobs(jobs, njobs);
    if (chk != IBS_OK) return chk;
    hipStream_t s = static_cast<hipStream_t>(stream);
    // candidates: lane counts up to the number of workspaces, both policies
    int nws = 0;
    assign_lanes(jobs, njobs, 64, IBS_SCHED_BALANCED, nws);
    struct Cand { int lanes, policy; float best; };
    std::vector<int> counts;
    for (int l : {1, 2, 4, 8, 12, 16, 24, 32, 48, 64}) {
        const int ll = std::min(l, nws);
        if (counts.empty() || counts.back() != ll) counts.push_back(ll);
    }
    std::vector<Cand> cands;
    for (int ll : counts) {
        cands.push_back({ll, IBS_SCHED_BALANCED, 1e30f});
        if (ll > 1) cands.push_back({ll, IBS_SCHED_IN_ORDER, 1e30f});
    }
    hipEvent_t ev[2] = {nullptr, nullptr};
    hipError_t e;
    if ((e = hipEventCreate(&ev[0])) != hipSuccess) return fail_hip(e, "autotune event");
    if ((e = hipEventCreate(&ev[1])) != hipSuccess) { hipEventDestroy(ev[0]); return fail_hip(e, "autotune event"); }
    ibs_status st = IBS_OK;
    std::vector<ibs_batch> built(cands.size(), nullptr);
    for (size_t c = 0; c < cands.size() && st == IBS_OK; ++c)
        st = ibs_batch_build_sched(jobs, njobs, cands[c].lanes, cands[c].policy, &built[c]);
    // one warm replay each, then three interleaved timed rounds; each
    // candidate keeps its fastest round
    constexpr int ROUNDS = 3;
    for (int round = -1; round < ROUNDS && st == IBS_OK; ++round)
        for (size_t c = 0; c < cands.size() && st == IBS_OK; ++c) {
            const int n = round < 0 ? 1 : reps;
            hipEventRecord(ev[0], s);
            for (int r = 0; r < n && st == IBS_OK; ++r) st = ibs_batch_launch(built[c], s);
            hipEventRecord(ev[1], s);
            if (st != IBS_OK) break;
            if ((e = hipEventSynchronize(ev[1])) != hipSuccess) { st = fail_hip(e, "autotune sync"); break; }
            float t = 0.f;
            hipEventElapsedTime(&t, ev[0], ev[1]);
            if (round >= 0) cands[c].best = std::min(cands[c].best, t / n);
        }
    for (ibs_batch b : built) ibs_batch_destroy(b);
    hipEventDestroy(ev[0]);
    hipEventDestroy(ev[1]);
    if (st != IBS_OK) return st;
    size_t pick = 0;
    for (size_t c = 1; c < cands.size(); ++c)
        if (cands[c].best < cands[pick].best) pick = c;
    *nlanes = cands[pick].lanes;
    *policy = cands[pick].policy;
    if (ms) *ms = cands[pick].best;
    return IBS_OK;
}

}  // extern "C"
