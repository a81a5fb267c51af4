// Graph-captured job steps (encore_plan_*): the hot path of encore_npcf over one
// grid -- gather -> coupling -> in-order FP64 reduction -> contraction -> zeta to
// pinned host memory -- recorded once into a HIP graph and replayed.
//
// Creation prepares everything that needs the host (primary list, slice tables,
// workspaces, tables, normalisation) on the plan's own stream, runs the steps
// once eagerly (which also sets kernel attributes on first use), then captures
// only kernel launches and the final device-to-host copy: replay allocates
// nothing and records no memset (zeroing is done by fill kernels).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "engine.h"

using namespace encore;

struct encore_plan {
    encore_ctx* ctx = nullptr;
    encore_grid* grid = nullptr;
    NpcfPlan pl;
    DevTables* tb = nullptr;
    Exec x;
    std::vector<Buf> segs, splits, redp;
    std::vector<SliceLaunch> slices;
    bool normalize = false;
    size_t need = 0;
    int64_t outs = 0;
    double* zeta_host = nullptr;   // pinned
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
};

namespace {

// The recorded sequence (eager or under capture).
int plan_steps(encore_plan* P)
{
    const hipStream_t s = P->x.s;
    int rc;
    HIPTRY((hipError_t)launch_fill((double*)P->x.Tjob.p, P->outs, 0.0, s));
    for (const SliceLaunch& L : P->slices) {
        if ((rc = launch_slice_gather(L, P->pl, s))) return rc;
        if ((rc = launch_slice_couple(L, P->pl, P->tb, s))) return rc;
    }
    if ((rc = contract_job(P->x, P->pl, P->tb, (const double*)P->x.Tjob.p,
                           P->normalize ? (const double*)P->x.bscale.p : nullptr, (double*)P->x.zeta.p)))
        return rc;
    HIPTRY(hipMemcpyAsync(P->zeta_host, P->x.zeta.p, sizeof(double) * std::max<size_t>(P->need, 1),
                          hipMemcpyDeviceToHost, s));
    return ENCORE_OK;
}

void plan_release(encore_plan* P)
{
    if (P->x.s) (void)hipStreamSynchronize(P->x.s);
    if (P->gexec) (void)hipGraphExecDestroy(P->gexec);
    if (P->graph) (void)hipGraphDestroy(P->graph);
    for (auto* v : {&P->segs, &P->splits, &P->redp})
        for (Buf& b : *v)
            if (b.p) (void)hipFree(b.p);
    if (P->zeta_host) (void)hipHostFree(P->zeta_host);
    exec_release(P->x);
    if (P->grid) P->grid->plans--;
    delete P;
}

int plan_build(encore_plan* P, const double* edges, uint32_t flags, double volume)
{
    encore_ctx* ctx = P->ctx;
    const NpcfPlan& pl = P->pl;
    int rc;
    if ((rc = exec_init(P->x))) return rc;
    const hipStream_t s = P->x.s;
    if ((rc = get_tables_for(ctx, pl, &P->tb))) return rc;
    P->outs = acc_len(pl, P->tb);
    P->need = (size_t)(pl.nlam * pl.nB);
    const DevGrid& g = P->grid->g;
    const int64_t n = g.n;
    Exec& x = P->x;
    if ((rc = ensure(x.prim, sizeof(int32_t) * std::max<int64_t>(n, 1)))) return rc;
    HIPTRY((hipError_t)launch_iota((int32_t*)x.prim.p, n, s));
    if ((rc = ensure(x.Tjob, sizeof(double) * (size_t)std::max<int64_t>(P->outs, 1)))) return rc;
    if ((rc = ensure(x.zeta, sizeof(double) * std::max<size_t>(P->need, 1)))) return rc;
    const int64_t cap = cap_rows(pl);
    const int64_t sr = job_split_rows(pl, P->tb, n, cap);
    const int64_t per_slice = std::max<int64_t>(sr, cap / sr * sr);
    for (int64_t r0 = 0; r0 < n; r0 += per_slice) {
        const int64_t r1 = std::min<int64_t>(n, r0 + per_slice);
        std::vector<Chunk> chunks{Chunk{&g, (const int32_t*)x.prim.p, r0, r1, sr, (double*)x.Tjob.p}};
        P->segs.emplace_back();
        P->splits.emplace_back();
        P->redp.emplace_back();
        P->slices.emplace_back();
        if ((rc = prepare_slice(x, P->segs.back(), P->splits.back(), P->redp.back(), pl, P->tb, edges,
                                chunks, P->slices.back())))
            return rc;
        P->slices.back().ga.npairs = nullptr;   // no pair count in the replayed steps
        HIPTRY(hipStreamSynchronize(s));         // the host tables of this slice are copied
    }
    P->normalize = flags & ENCORE_NORMALIZE;
    if (P->normalize) {
        const double V = volume > 0.0 ? volume : g.Lx * g.Ly * g.Lz;
        const std::vector<double> sc = bin_scale(pl, edges, V);
        if ((rc = ensure(x.bscale, sizeof(double) * std::max<size_t>(sc.size(), 1)))) return rc;
        HIPTRY(hipMemcpyAsync(x.bscale.p, sc.data(), sizeof(double) * sc.size(), hipMemcpyHostToDevice, s));
    }
    HIPTRY(hipHostMalloc((void**)&P->zeta_host, sizeof(double) * std::max<size_t>(P->need, 1)));
    // one eager pass, then the capture
    if ((rc = plan_steps(P))) return rc;
    HIPTRY(hipStreamSynchronize(s));
    HIPTRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    rc = plan_steps(P);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(s, &graph);
    if (rc) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    P->graph = graph;
    HIPTRY(hipGraphInstantiate(&P->gexec, P->graph, nullptr, nullptr, 0));
    return ENCORE_OK;
}

}  // namespace

extern "C" {

int encore_plan_create(encore_ctx* ctx, encore_grid* grid, int npcf, int lmax, int nbins,
                       const double* edges, uint32_t flags, double volume, encore_plan** out)
{
    if (!ctx || !grid || !out) return fail(ENCORE_EINVAL, "NULL ctx, grid or out");
    if (grid->ctx != ctx) return fail(ENCORE_EINVAL, "grid belongs to another context");
    auto* P = new encore_plan();
    P->ctx = ctx;
    int rc = plan_call(npcf, lmax, nbins, edges, flags, &P->pl);
    if (!rc) P->pl.nbg = ctx_nbg(ctx, P->pl);
    if (!rc) rc = check_grid_edges(grid->g, edges, nbins);
    if (!rc && (flags & ENCORE_NORMALIZE) && !(volume > 0.0) && !grid->g.periodic)
        rc = fail(ENCORE_EINVAL, "ENCORE_NORMALIZE needs volume > 0 without a periodic box");
    if (rc) {
        delete P;
        return rc;
    }
    if (hipSetDevice(ctx->device) != hipSuccess) {
        delete P;
        return fail(ENCORE_EDEVICE, "hipSetDevice");
    }
    P->grid = grid;
    grid->plans++;
    if ((rc = plan_build(P, edges, flags, volume))) {
        plan_release(P);
        return rc;
    }
    *out = P;
    return ENCORE_OK;
}

int encore_plan_execute(encore_plan* plan, double* zeta, size_t zeta_len)
{
    if (!plan) return fail(ENCORE_EINVAL, "plan is NULL");
    if (!zeta && plan->need > 0) return fail(ENCORE_EINVAL, "zeta is NULL");
    if (zeta_len < plan->need)
        return fail(ENCORE_ESIZE, "zeta_len too small: need " + std::to_string(plan->need));
    HIPTRY(hipSetDevice(plan->ctx->device));
    HIPTRY(hipGraphLaunch(plan->gexec, plan->x.s));
    HIPTRY(hipStreamSynchronize(plan->x.s));
    if (plan->need) std::memcpy(zeta, plan->zeta_host, sizeof(double) * plan->need);
    return ENCORE_OK;
}

int encore_plan_destroy(encore_plan* plan)
{
    if (!plan) return ENCORE_OK;
    (void)hipSetDevice(plan->ctx->device);
    plan_release(plan);
    return ENCORE_OK;
}

}  // extern "C"
