// Serving loop (encore_server_*): catalog jobs are submitted from any thread,
// admitted by device-memory footprint, and run by lane threads, each with its
// own HIP stream and workspaces.  Every iteration a lane takes one slice of
// primary rows from the admitted jobs of one class (continuous batching: jobs
// that arrive while slices run join at the next iteration), runs gather ->
// coupling -> reduction into each job's resident T, and finishes the jobs whose
// rows are all done (contraction, zeta to the host, device memory released).
// Lanes run concurrently, so one lane's coupling overlaps another's gather.
//
// Nothing on a lane's path synchronises the whole device: a job's device memory
// (catalog staging, grid, primary list, T) and the lanes' workspaces come from a
// stream-ordered pool owned by the server and are returned to it with
// hipFreeAsync on the lane's stream (hipFree would wait for every lane's work),
// and catalogs reach the device through pinned, double-buffered staging of the
// lane (a pageable copy would go through the runtime's own staging).
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <map>
#include <memory>
#include <thread>

#include "engine.h"
#include "sched.h"

using namespace encore;

namespace {

using Clock = std::chrono::steady_clock;

struct SrvJob {
    SchedJob sj;
    // request
    int64_t n = 0, n_data = 0;
    uint32_t flags = 0;
    bool periodic = false;
    double box[3] = {0, 0, 0};
    std::vector<double> edges;
    std::vector<double> pos, w;   // host copies until the grid is built
    NpcfPlan pl;
    // device state
    DevTables* tb = nullptr;
    DevGrid g;
    bool has_grid = false;
    int32_t* prim = nullptr;
    double* T = nullptr;
    double* bscale = nullptr;
    // result
    std::vector<double> zeta;
    int rc = ENCORE_OK;
    std::string err;
    bool started = false;
    double t_submit = 0, t_admit = 0, t_start = 0, t_done = 0;
};

}  // namespace

namespace {
// Pinned host staging of one lane: two halves used alternately, each free again
// once the copy recorded by its event has finished.
constexpr size_t kStageHalf = (size_t)8 << 20;
struct Stage {
    unsigned char* host = nullptr;   // [2 * kStageHalf], hipHostMalloc
    hipEvent_t ev[2] = {nullptr, nullptr};
};
}  // namespace

struct encore_server {
    encore_ctx* ctx = nullptr;
    hipMemPool_t pool = nullptr;
    std::vector<Stage> stage;   // one per lane
    Scheduler sch;
    int64_t slice_rows = 0;
    std::mutex mu;
    std::condition_variable cv;
    std::map<int64_t, std::unique_ptr<SrvJob>> jobs;
    std::map<std::vector<double>, uint64_t> classes;   // class key -> id
    int64_t next_id = 1;
    std::vector<Exec> lanes;
    std::vector<std::thread> threads;
    bool stop = false;
    Clock::time_point t0;
    // statistics
    int64_t n_submitted = 0, n_done = 0, n_failed = 0, rows_done = 0, slices = 0;
    double ms_gather = 0, ms_couple = 0;

    encore_server(size_t budget, int max_active) : sch(budget, max_active) {}
    double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
};

namespace {

// Device memory of a job back to the pool, ordered on stream s (after the job's
// last use, which every caller has already waited for).
void release_job(encore_server* S, SrvJob* j, hipStream_t s)
{
    if (j->has_grid) grid_free(j->g, s);
    j->has_grid = false;
    for (void* p : {(void*)j->prim, (void*)j->T, (void*)j->bscale}) dev_free(p, S->pool, s);
    j->prim = nullptr;
    j->T = nullptr;
    j->bscale = nullptr;
    std::vector<double>().swap(j->pos);
    std::vector<double>().swap(j->w);
}

// bytes host -> device through the lane's pinned staging, on stream s
int stage_upload(Stage& st, hipStream_t s, void* dst, const void* src, size_t bytes)
{
    size_t off = 0;
    int h = 0;
    while (off < bytes) {
        const size_t c = std::min(kStageHalf, bytes - off);
        HIPTRY(hipEventSynchronize(st.ev[h]));   // the half's previous copy is done
        unsigned char* buf = st.host + (size_t)h * kStageHalf;
        std::memcpy(buf, (const unsigned char*)src + off, c);
        HIPTRY(hipMemcpyAsync((unsigned char*)dst + off, buf, c, hipMemcpyHostToDevice, s));
        HIPTRY(hipEventRecord(st.ev[h], s));
        off += c;
        h ^= 1;
    }
    return ENCORE_OK;
}

// Grid, primary list, T and tables of an admitted job, on lane li.
int setup_job(encore_server* S, SrvJob* j, int li)
{
    Exec& x = S->lanes[li];
    const hipStream_t s = x.s;
    int rc;
    if ((rc = get_tables_for(S->ctx, j->pl, &j->tb))) return rc;
    double* d_pos = nullptr;
    double* d_w = nullptr;
    hipError_t e = dev_alloc((void**)&d_pos, sizeof(double) * 3 * j->n, S->pool, s);
    if (e == hipSuccess) e = dev_alloc((void**)&d_w, sizeof(double) * j->n, S->pool, s);
    if (e != hipSuccess) {
        dev_free(d_pos, S->pool, s);
        return hip_fail(e, "server: catalog staging");
    }
    rc = stage_upload(S->stage[li], s, d_pos, j->pos.data(), sizeof(double) * 3 * j->n);
    if (rc == ENCORE_OK) rc = stage_upload(S->stage[li], s, d_w, j->w.data(), sizeof(double) * j->n);
    if (rc == ENCORE_OK) {
        double div = 0.0, xsub = 0.0;
        ctx_cells(S->ctx, &div, &xsub);
        rc = build_grid_dev(S->ctx->device, d_pos, d_w, j->n, j->n_data, (j->flags & ENCORE_DMR) != 0,
                            j->periodic ? j->box : nullptr, j->edges[j->pl.nbins], div, xsub, s, j->g,
                            S->pool);
        j->has_grid = rc == ENCORE_OK;
    }
    dev_free(d_pos, S->pool, s);   // stream-ordered: after the grid build has read them
    dev_free(d_w, S->pool, s);
    if (rc) return rc;
    std::vector<double>().swap(j->pos);
    std::vector<double>().swap(j->w);
    const int64_t outs = acc_len(j->pl, j->tb);
    HIPTRY(dev_alloc((void**)&j->prim, sizeof(int32_t) * j->n, S->pool, s));
    HIPTRY(dev_alloc((void**)&j->T, sizeof(double) * std::max<int64_t>(outs, 1), S->pool, s));
    HIPTRY((hipError_t)launch_iota(j->prim, j->n, s));
    HIPTRY((hipError_t)launch_fill(j->T, outs, 0.0, s));
    if (j->flags & ENCORE_NORMALIZE) {
        const std::vector<double> sc = bin_scale(j->pl, j->edges.data(), j->box[0] * j->box[1] * j->box[2]);
        HIPTRY(dev_alloc((void**)&j->bscale, sizeof(double) * std::max<size_t>(sc.size(), 1), S->pool, s));
        HIPTRY(hipMemcpyAsync(j->bscale, sc.data(), sizeof(double) * sc.size(), hipMemcpyHostToDevice, s));
        HIPTRY(hipStreamSynchronize(s));   // sc is a local
    }
    HIPTRY(hipStreamSynchronize(s));
    j->sj.split_rows = job_split_rows(j->pl, j->tb, j->n, cap_rows(j->pl));
    return ENCORE_OK;
}

// Contraction of a job whose rows are all reduced; zeta to the host.
int finish_job(SrvJob* j, Exec& x)
{
    const size_t need = (size_t)(j->pl.nlam * j->pl.nB);
    int rc;
    if ((rc = ensure(x.zeta, sizeof(double) * std::max<size_t>(need, 1)))) return rc;
    if ((rc = contract_job(x, j->pl, j->tb, j->T, j->bscale, (double*)x.zeta.p))) return rc;
    j->zeta.resize(need);
    HIPTRY(hipMemcpyAsync(j->zeta.data(), x.zeta.p, sizeof(double) * need, hipMemcpyDeviceToHost, x.s));
    HIPTRY(hipStreamSynchronize(x.s));
    return ENCORE_OK;
}

void lane_main(encore_server* S, int li)
{
    (void)hipSetDevice(S->ctx->device);
    Exec& x = S->lanes[li];
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        std::vector<SchedJob*> adm = S->sch.admit();
        if (!adm.empty()) {
            const double t = S->now();
            for (SchedJob* sj : adm) static_cast<SrvJob*>(sj->user)->t_admit = t;
            lk.unlock();
            std::vector<int> rcs;
            std::vector<std::string> errs;
            for (SchedJob* sj : adm) {
                SrvJob* j = static_cast<SrvJob*>(sj->user);
                const int rc = setup_job(S, j, li);
                rcs.push_back(rc);
                errs.push_back(rc ? get_error() : "");
                if (rc) {
                    (void)hipStreamSynchronize(x.s);
                    release_job(S, j, x.s);
                }
            }
            lk.lock();
            for (size_t k = 0; k < adm.size(); ++k) {
                SrvJob* j = static_cast<SrvJob*>(adm[k]->user);
                if (rcs[k] == ENCORE_OK) {
                    S->sch.ready(adm[k]);
                } else {
                    j->rc = rcs[k];
                    j->err = errs[k];
                    j->t_done = S->now();
                    S->sch.finish(adm[k], false);
                    S->n_failed++;
                }
            }
            S->cv.notify_all();
            continue;
        }
        std::vector<SchedChunk> picked = S->sch.pick(S->slice_rows);
        if (picked.empty()) {
            if (S->stop && S->sch.queued() == 0 && S->sch.active() == 0) break;
            S->cv.wait(lk);
            continue;
        }
        const double t = S->now();
        for (const SchedChunk& c : picked) {
            SrvJob* j = static_cast<SrvJob*>(c.job->user);
            if (!j->started) { j->started = true; j->t_start = t; }
        }
        lk.unlock();
        SrvJob* j0 = static_cast<SrvJob*>(picked[0].job->user);
        std::vector<Chunk> chunks;
        int64_t rows = 0;
        for (const SchedChunk& c : picked) {
            SrvJob* j = static_cast<SrvJob*>(c.job->user);
            chunks.push_back(Chunk{&j->g, j->prim, c.r0, c.r1, j->sj.split_rows, j->T});
            rows += c.r1 - c.r0;
        }
        double mg = 0, mc = 0;
        int rc = run_slice(x, j0->pl, j0->tb, j0->edges.data(), chunks, &mg, &mc);
        std::string err = rc ? get_error() : "";
        lk.lock();
        S->slices++;
        S->rows_done += rows;
        S->ms_gather += mg;
        S->ms_couple += mc;
        std::vector<SchedJob*> complete = S->sch.slice_done(picked);
        if (rc) {
            // a failed slice fails every job in it; the others are not touched
            for (const SchedChunk& c : picked) {
                SrvJob* j = static_cast<SrvJob*>(c.job->user);
                if (j->sj.state == SchedJob::READY) {
                    j->rc = rc;
                    j->err = err;
                    j->sj.busy = true;
                }
            }
            complete.clear();
            for (const SchedChunk& c : picked) complete.push_back(c.job);
        }
        lk.unlock();
        std::vector<int> rcs;
        std::vector<std::string> errs;
        for (SchedJob* sj : complete) {
            SrvJob* j = static_cast<SrvJob*>(sj->user);
            int r = j->rc;
            if (r == ENCORE_OK) r = finish_job(j, x);
            rcs.push_back(r);
            errs.push_back(r ? (j->rc ? j->err : std::string(get_error())) : "");
            (void)hipStreamSynchronize(x.s);   // a failed slice may not have synchronised
            release_job(S, j, x.s);
        }
        lk.lock();
        for (size_t k = 0; k < complete.size(); ++k) {
            SrvJob* j = static_cast<SrvJob*>(complete[k]->user);
            if (j->sj.state != SchedJob::READY) continue;   // already finished
            j->rc = rcs[k];
            j->err = errs[k];
            j->t_done = S->now();
            S->sch.finish(complete[k], rcs[k] == ENCORE_OK);
            if (rcs[k] == ENCORE_OK) S->n_done++;
            else S->n_failed++;
        }
        S->cv.notify_all();
    }
    S->cv.notify_all();
}

// Device bytes a job holds from admission to completion: catalog staging,
// D-R weights, cell keys, the grid (sorted points, permutations, cell starts),
// its primary list, T and the normalisation table.
size_t footprint(int64_t n, int64_t ncell, int64_t outs, int64_t nB)
{
    return (size_t)n * (24 + 8 + 8 + 4 + 32 + 4 + 4 + 4) + (size_t)kSentinels * 32 + (size_t)ncell * 8 +
           (size_t)outs * 8 + (size_t)nB * 8 + ((size_t)1 << 16);
}

}  // namespace

extern "C" {

int encore_server_create(encore_ctx* ctx, size_t hbm_budget, int n_lanes, int max_active,
                         int64_t slice_rows, encore_server** out)
{
    if (!ctx || !out) return fail(ENCORE_EINVAL, "NULL ctx or out");
    if (hbm_budget == 0) return fail(ENCORE_EINVAL, "hbm_budget must be > 0");
    if (n_lanes < 1 || n_lanes > 8) return fail(ENCORE_EINVAL, "n_lanes must be 1..8");
    if (max_active < 1) return fail(ENCORE_EINVAL, "max_active must be >= 1");
    if (slice_rows < 1) return fail(ENCORE_EINVAL, "slice_rows must be >= 1");
    HIPTRY(hipSetDevice(ctx->device));
    auto* S = new encore_server(hbm_budget, max_active);
    S->ctx = ctx;
    S->slice_rows = slice_rows;
    S->t0 = Clock::now();
    S->lanes.resize(n_lanes);
    S->stage.resize(n_lanes);
    auto undo = [&](int rc) {
        for (Exec& x : S->lanes) exec_release(x);
        for (Stage& st : S->stage) {
            for (hipEvent_t& e : st.ev)
                if (e) (void)hipEventDestroy(e);
            if (st.host) (void)hipHostFree(st.host);
        }
        if (S->pool) (void)hipMemPoolDestroy(S->pool);
        delete S;
        return rc;
    };
    // the pool keeps what it has taken from the device until the server ends
    hipMemPoolProps props;
    std::memset(&props, 0, sizeof(props));
    props.allocType = hipMemAllocationTypePinned;
    props.location.type = hipMemLocationTypeDevice;
    props.location.id = ctx->device;
    hipError_t e = hipMemPoolCreate(&S->pool, &props);
    if (e != hipSuccess) {
        S->pool = nullptr;
        return undo(hip_fail(e, "hipMemPoolCreate"));
    }
    uint64_t keep = UINT64_MAX;
    e = hipMemPoolSetAttribute(S->pool, hipMemPoolAttrReleaseThreshold, &keep);
    if (e != hipSuccess) return undo(hip_fail(e, "hipMemPoolSetAttribute"));
    for (int i = 0; i < n_lanes; ++i) {
        const int rc = exec_init(S->lanes[i], S->pool);
        if (rc) return undo(rc);
        Stage& st = S->stage[i];
        e = hipHostMalloc((void**)&st.host, 2 * kStageHalf, hipHostMallocDefault);
        if (e != hipSuccess) {
            st.host = nullptr;
            return undo(hip_fail(e, "hipHostMalloc(staging)"));
        }
        for (hipEvent_t& ev : st.ev) {
            if ((e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess)
                return undo(hip_fail(e, "hipEventCreate"));
            if ((e = hipEventRecord(ev, S->lanes[i].s)) != hipSuccess) return undo(hip_fail(e, "hipEventRecord"));
        }
    }
    for (int i = 0; i < n_lanes; ++i) S->threads.emplace_back(lane_main, S, i);
    *out = S;
    return ENCORE_OK;
}

int encore_server_submit(encore_server* S, const double* pos, const double* w, int64_t n, int64_t n_data,
                         const double* box, int npcf, int lmax, int nbins, const double* edges,
                         uint32_t flags, int64_t* job_id)
{
    if (!S || !job_id) return fail(ENCORE_EINVAL, "NULL server or job_id");
    if (!pos || !w) return fail(ENCORE_EINVAL, "NULL pos or w");
    if (n < 1) return fail(ENCORE_EINVAL, "n must be >= 1");
    if (n > kMaxGridPoints) return fail(ENCORE_EINVAL, "catalog exceeds the point limit of one grid (2^26 - 64)");
    auto j = std::make_unique<SrvJob>();
    int rc;
    if ((rc = plan_call(npcf, lmax, nbins, edges, flags, &j->pl))) return rc;
    j->pl.nbg = ctx_nbg(S->ctx, j->pl);
    const double r_max = edges[nbins];
    j->periodic = flags & ENCORE_PERIODIC;
    if (j->periodic) {
        if (!box) return fail(ENCORE_EINVAL, "ENCORE_PERIODIC needs box");
        for (int a = 0; a < 3; ++a) {
            if (!(box[a] > 0.0) || !std::isfinite(box[a])) return fail(ENCORE_EINVAL, "box must be > 0");
            if (2.0 * r_max > box[a]) return fail(ENCORE_EINVAL, "periodic box: edges[nbins] must be <= box/2");
            j->box[a] = box[a];
        }
    } else if (flags & ENCORE_NORMALIZE) {
        return fail(ENCORE_EINVAL, "ENCORE_NORMALIZE in a served job needs a periodic box");
    }
    if ((flags & ENCORE_DMR) && (n_data < 1 || n_data >= n)) return fail(ENCORE_EINVAL, "ENCORE_DMR needs 1 <= n_data < n");
    // cells of the grid the job will build (an upper bound for open boxes)
    double div = 0.0, xsub = 0.0;
    ctx_cells(S->ctx, &div, &xsub);
    const double cs_yz = r_max / div;
    const double cs_axis[3] = {cs_yz / xsub, cs_yz, cs_yz};
    int64_t ncell = 1;
    if (j->periodic) {
        for (int a = 0; a < 3; ++a) ncell *= std::max<int64_t>(1, (int64_t)std::floor(box[a] / cs_axis[a]));
    } else {
        double lo[3] = {pos[0], pos[1], pos[2]}, hi[3] = {pos[0], pos[1], pos[2]};
        for (int64_t i = 0; i < n; ++i)
            for (int a = 0; a < 3; ++a) {
                const double v = pos[3 * i + a];
                if (v < lo[a]) lo[a] = v;
                if (v > hi[a]) hi[a] = v;
            }
        for (int a = 0; a < 3; ++a) {
            const double ext = hi[a] - lo[a];
            ncell *= std::isfinite(ext) ? (int64_t)std::floor(ext / cs_axis[a]) + 1 : 1;
        }
    }
    int64_t outs = 0;
    if ((rc = acc_len_host(j->pl, &outs))) return rc;
    j->n = n;
    j->n_data = n_data;
    j->flags = flags;
    j->edges.assign(edges, edges + nbins + 1);
    j->pos.assign(pos, pos + 3 * n);
    j->w.assign(w, w + n);
    j->sj.footprint = footprint(n, ncell, outs, j->pl.nB);
    j->sj.nrows = n;
    j->sj.user = j.get();
    std::lock_guard<std::mutex> lock(S->mu);
    if (S->stop) return fail(ENCORE_EINVAL, "server is shutting down");
    // class: jobs with the same kernels, tables and bins can share a slice
    std::vector<double> key{(double)npcf, (double)lmax, (double)nbins,
                            (double)(flags & (ENCORE_PREC_MASK | ENCORE_ALLPARITY))};
    key.insert(key.end(), edges, edges + nbins + 1);
    auto it = S->classes.find(key);
    if (it == S->classes.end()) it = S->classes.emplace(key, (uint64_t)S->classes.size()).first;
    j->sj.cls = it->second;
    j->sj.id = S->next_id++;
    j->t_submit = S->now();
    if (!S->sch.submit(&j->sj))
        return fail(ENCORE_ESIZE, "job needs " + std::to_string(j->sj.footprint) +
                                      " device bytes, more than the server budget");
    *job_id = j->sj.id;
    S->jobs.emplace(j->sj.id, std::move(j));
    S->n_submitted++;
    S->cv.notify_all();
    return ENCORE_OK;
}

int encore_server_wait(encore_server* S, int64_t job_id, double timeout_s, double* zeta, size_t zeta_len,
                       double* times)
{
    if (!S) return fail(ENCORE_EINVAL, "NULL server");
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->jobs.find(job_id);
    if (it == S->jobs.end()) return fail(ENCORE_EINVAL, "unknown job id (or already collected)");
    SrvJob* j = it->second.get();
    auto finished = [&]() { return j->sj.state == SchedJob::DONE || j->sj.state == SchedJob::FAILED; };
    if (timeout_s < 0) S->cv.wait(lk, finished);
    else if (!S->cv.wait_for(lk, std::chrono::duration<double>(timeout_s), finished))
        return fail(ENCORE_EAGAIN, "job not finished");
    if (times) {
        times[0] = j->t_submit; times[1] = j->t_admit; times[2] = j->t_start; times[3] = j->t_done;
    }
    if (j->sj.state == SchedJob::FAILED) {
        const int rc = j->rc ? j->rc : ENCORE_EDEVICE;
        const std::string msg = "job " + std::to_string(job_id) + " failed: " + j->err;
        S->jobs.erase(it);
        return fail(rc, msg);
    }
    if (zeta_len < j->zeta.size() || (!zeta && !j->zeta.empty()))
        return fail(ENCORE_ESIZE, "zeta needs " + std::to_string(j->zeta.size()) + " elements");
    std::copy(j->zeta.begin(), j->zeta.end(), zeta);
    S->jobs.erase(it);
    return ENCORE_OK;
}

int encore_server_stats(encore_server* S, double* out, size_t out_len)
{
    if (!S || !out) return fail(ENCORE_EINVAL, "NULL server or out");
    if (out_len < 12) return fail(ENCORE_ESIZE, "stats need 12 entries");
    std::lock_guard<std::mutex> lock(S->mu);
    size_t ws = 0;
    for (const Exec& x : S->lanes) ws += exec_bytes(x);
    const double v[12] = {(double)S->n_submitted, (double)S->n_done, (double)S->n_failed,
                          (double)S->sch.queued(), (double)S->sch.active(), (double)S->sch.used(),
                          (double)S->sch.peak(), (double)S->rows_done, (double)S->slices,
                          S->ms_gather, S->ms_couple, (double)ws};
    std::copy(v, v + 12, out);
    return ENCORE_OK;
}

int encore_server_destroy(encore_server* S)
{
    if (!S) return ENCORE_OK;
    {
        std::lock_guard<std::mutex> lock(S->mu);
        S->stop = true;
        S->cv.notify_all();
    }
    for (std::thread& t : S->threads) t.join();
    (void)hipSetDevice(S->ctx->device);
    for (auto& kv : S->jobs) release_job(S, kv.second.get(), S->lanes[0].s);
    for (Exec& x : S->lanes) exec_release(x);   // synchronises each lane's stream
    for (Stage& st : S->stage) {
        for (hipEvent_t& e : st.ev)
            if (e) (void)hipEventDestroy(e);
        if (st.host) (void)hipHostFree(st.host);
    }
    (void)hipMemPoolDestroy(S->pool);
    delete S;
    return ENCORE_OK;
}

}  // extern "C"
