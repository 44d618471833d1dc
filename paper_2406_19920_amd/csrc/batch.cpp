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
#include <map>
#include <string>
#include <vector>

#include "ibs_internal.h"

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
    delete batch;
    return IBS_OK;
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
