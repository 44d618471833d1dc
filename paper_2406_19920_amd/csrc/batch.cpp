// Batched execution of many independent solves as one HIP graph.
//
// ibs_batch_build() records every job's launches once (stream capture) into
// a graph whose independent branches ("lanes") the GPU may run side by
// side; ibs_batch_launch() replays the whole batch with one hipGraphLaunch.
// All solves that use the same workspace are placed on the same lane (the
// workspace holds a call's fields and mutable state, so calls sharing it
// must not overlap), and lanes are balanced greedily by the work of their
// jobs.  The plans' device constants are only read, so jobs of one plan
// with distinct workspaces may run side by side.
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

extern "C" {

ibs_status ibs_batch_build(const ibs_batch_job *jobs, int32_t njobs, int32_t nlanes, ibs_batch *out)
{
    if (!jobs || njobs < 1 || !out || nlanes < 1 || nlanes > 64) {
        set_error("jobs, out must be non-NULL, njobs >= 1, nlanes in [1, 64]");
        return IBS_ERR_INVALID_ARG;
    }
    *out = nullptr;
    for (int q = 0; q < njobs; ++q) {
        const ibs_batch_job &j = jobs[q];
        if (!j.plan) { set_error("job without a plan"); return IBS_ERR_INVALID_ARG; }
        if (j.op != IBS_OP_POISSON && j.op != IBS_OP_HELMHOLTZ_U) { set_error("job op must be IBS_OP_POISSON or IBS_OP_HELMHOLTZ_U"); return IBS_ERR_INVALID_ARG; }
        if (j.op == IBS_OP_HELMHOLTZ_U && (j.ncomp < 1 || j.ncomp > 3)) { set_error("Helmholtz job ncomp must be 1..3"); return IBS_ERR_INVALID_ARG; }
    }
    // lane per workspace, greedy by work (cells x solve count)
    std::map<void *, double> cost;
    std::map<ibs_plan, int> plans;
    for (int q = 0; q < njobs; ++q) {
        Plan *p = reinterpret_cast<Plan *>(jobs[q].plan);
        const double cells = (double)p->nx * p->ny * p->nz;
        cost[jobs[q].work] += cells * (jobs[q].op == IBS_OP_POISSON ? 1 : jobs[q].ncomp);
        plans[jobs[q].plan] = 1;
    }
    std::vector<std::pair<double, void *>> order;
    for (auto &kv : cost) order.push_back({kv.second, kv.first});
    std::stable_sort(order.begin(), order.end(), [](auto &a, auto &b) { return a.first > b.first; });
    const int L = std::min<int>(nlanes, (int)order.size());
    std::vector<double> load(L, 0.0);
    std::map<void *, int> lane_of;
    for (auto &o : order) {
        int best = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        lane_of[o.second] = best;
        load[best] += o.first;
    }

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

}  // extern "C"
