// C ABI of libencore (declared in include/encore.h): contexts, grids and the
// synchronous entry points.  One encore_npcf call runs on one HIP stream:
//   primary list -> [gather a~ for a slice of primaries -> couple -> reduce into T] x slices
//   -> contract T with the coupling terms -> zeta (FP64) -> host.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "engine.h"

using namespace encore;

namespace encore {

// Primaries of one job as cell-sorted indices at dst (device, room for the count):
// every point (subset NULL) or the subset given in input order.  *np: the count.
int fill_primaries(Exec& x, const encore_grid* grid, const int64_t* subset, int64_t k, int32_t* dst,
                   int64_t* np)
{
    const hipStream_t s = x.s;
    const int64_t n = grid->g.n;
    if (!subset) {
        HIPTRY((hipError_t)launch_iota(dst, n, s));
        *np = n;
        return ENCORE_OK;
    }
    if (k < 0) return fail(ENCORE_EINVAL, "n_subset < 0");
    int rc;
    if ((rc = ensure(x.misc, sizeof(int64_t) * std::max<int64_t>(k, 1) + 16))) return rc;
    int* d_bad = (int*)x.misc.p;
    int64_t* d_idx = (int64_t*)((char*)x.misc.p + 16);
    int bad = 0;
    HIPTRY(hipMemcpyAsync(d_bad, &bad, sizeof(int), hipMemcpyHostToDevice, s));
    if (k > 0) {
        HIPTRY(hipMemcpyAsync(d_idx, subset, sizeof(int64_t) * k, hipMemcpyHostToDevice, s));
        HIPTRY((hipError_t)launch_map_subset(d_idx, k, grid->g.inv, n, dst, d_bad, s));
    }
    HIPTRY(hipMemcpyAsync(&bad, d_bad, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPTRY(hipStreamSynchronize(s));
    if (bad) return fail(ENCORE_EINVAL, "primary_subset holds an index outside [0, n)");
    *np = k;
    return ENCORE_OK;
}

}  // namespace encore

namespace {

// Primary list of one job into x.prim; returns count in *np.
int make_primaries(Exec& x, const encore_grid* grid, const int64_t* subset, int64_t k, int64_t* np)
{
    const int64_t cnt = subset ? k : grid->g.n;
    int rc = ensure(x.prim, sizeof(int32_t) * (size_t)std::max<int64_t>(cnt, 1));
    if (rc) return rc;
    return fill_primaries(x, grid, subset, k, (int32_t*)x.prim.p, np);
}

int build_grid_impl(encore_ctx* ctx, const double* pos, const double* w, int64_t n, int64_t n_data,
                    const double* box, double r_max, uint32_t flags, void* stream, encore_grid** out,
                    bool device_ptrs)
{
    if (!ctx || !out) return fail(ENCORE_EINVAL, "NULL ctx or out");
    if (!pos || !w) return fail(ENCORE_EINVAL, "NULL pos or w");
    if (n < 1) return fail(ENCORE_EINVAL, "n must be >= 1");
    if (!(r_max > 0.0) || !std::isfinite(r_max)) return fail(ENCORE_EINVAL, "r_max must be finite and > 0");
    const bool periodic = flags & ENCORE_PERIODIC;
    if (periodic) {
        if (!box) return fail(ENCORE_EINVAL, "ENCORE_PERIODIC needs box");
        for (int a = 0; a < 3; ++a)
            if (!(box[a] > 0.0) || !std::isfinite(box[a])) return fail(ENCORE_EINVAL, "box must be > 0");
    }
    HIPTRY(hipSetDevice(ctx->device));
    const hipStream_t s = stream ? (hipStream_t)stream : ctx->main.s;
    const double* d_pos = pos;
    const double* d_w = w;
    double* tmp_pos = nullptr;
    double* tmp_w = nullptr;
    if (!device_ptrs) {
        HIPTRY(hipMalloc(&tmp_pos, sizeof(double) * 3 * n));
        hipError_t e = hipMalloc(&tmp_w, sizeof(double) * n);
        if (e != hipSuccess) { (void)hipFree(tmp_pos); return hip_fail(e, "hipMalloc"); }
        e = hipMemcpyAsync(tmp_pos, pos, sizeof(double) * 3 * n, hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipMemcpyAsync(tmp_w, w, sizeof(double) * n, hipMemcpyHostToDevice, s);
        if (e != hipSuccess) {
            (void)hipFree(tmp_pos); (void)hipFree(tmp_w);
            return hip_fail(e, "hipMemcpyAsync(catalog)");
        }
        d_pos = tmp_pos; d_w = tmp_w;
    }
    auto* gr = new encore_grid();
    gr->ctx = ctx;
    double div = 0.0, xsub = 0.0;
    ctx_cells(ctx, &div, &xsub);
    const int rc = build_grid_dev(ctx->device, d_pos, d_w, n, n_data, (flags & ENCORE_DMR) != 0,
                                  periodic ? box : nullptr, r_max, div, xsub, s, gr->g);
    if (tmp_pos) (void)hipFree(tmp_pos);
    if (tmp_w) (void)hipFree(tmp_w);
    if (rc != 0) {
        delete gr;
        return rc;
    }
    ctx->live_grids++;
    *out = gr;
    return ENCORE_OK;
}

// Grids of the call: checks and the volume used by ENCORE_NORMALIZE.
int check_grids(const encore_grid* const* grids, int njobs, const encore_ctx* ctx, const double* edges,
                int nbins, uint32_t flags, double volume)
{
    int rc;
    for (int j = 0; j < njobs; ++j) {
        if (!grids[j]) return fail(ENCORE_EINVAL, "NULL grid");
        if (grids[j]->ctx != ctx) return fail(ENCORE_EINVAL, "grid belongs to another context");
        if ((rc = check_grid_edges(grids[j]->g, edges, nbins))) return rc;
        if ((flags & ENCORE_NORMALIZE) && !(volume > 0.0) && !grids[j]->g.periodic)
            return fail(ENCORE_EINVAL, "ENCORE_NORMALIZE needs volume > 0 without a periodic box");
    }
    return ENCORE_OK;
}

// points per r_max^3 (averaged over the parts) from which encore_npcf_splits keeps
// the data part of a~: measured break-even between 2,000 (0.95x) and 16,000 (1.09x)
constexpr double kSplitCacheDensity = 6000.0;

}  // namespace

namespace encore {

int run_jobs(encore_ctx* ctx, Exec& x, const DevTables* tb, int64_t cap, const std::vector<JobRows>& jobs,
             const NpcfPlan& pl, uint32_t flags, const double* edges, double volume, double* zeta)
{
    const hipStream_t s = x.s;
    const int njobs = (int)jobs.size();
    const size_t need = (size_t)(pl.nlam * pl.nB);
    int rc;
    const int64_t outs = acc_len(pl, tb);
    if ((rc = ensure(x.Tjob, sizeof(double) * (size_t)(njobs * outs)))) return rc;
    if ((rc = ensure(x.zeta, sizeof(double) * (size_t)njobs * std::max<size_t>(need, 1)))) return rc;
    if ((rc = ensure(x.misc, 64))) return rc;
    unsigned long long* d_pairs = (unsigned long long*)x.misc.p;
    HIPTRY((hipError_t)launch_fill((double*)x.Tjob.p, njobs * outs, 0.0, s));
    HIPTRY((hipError_t)launch_fill((double*)d_pairs, 1, 0.0, s));   // zero bits = 0ull

    std::vector<int64_t> srows(jobs.size());
    for (size_t j = 0; j < jobs.size(); ++j) srows[j] = job_split_rows(pl, tb, jobs[j].nprim, cap);

    double t_gather = 0.0, t_couple = 0.0;
    int nslice = 0;
    size_t jcur = 0;
    int64_t jpos = 0;   // rows of jobs[jcur] already done
    std::vector<Chunk> chunks;
    while (jcur < jobs.size()) {
        chunks.clear();
        int64_t rows = 0;
        while (jcur < jobs.size() && rows < cap && chunks.size() < 4096) {
            const JobRows& J = jobs[jcur];
            const int64_t sr = srows[jcur];
            int64_t take = J.nprim - jpos;
            if (take > cap - rows) take = (cap - rows) / sr * sr;   // whole splits only
            if (take == 0 && J.nprim > jpos) break;                  // next slice
            if (take > 0) {
                chunks.push_back(Chunk{&J.grid->g, J.prim, jpos, jpos + take, sr,
                                       (double*)x.Tjob.p + (size_t)jcur * outs, J.Pq, J.cache});
                rows += take;
                jpos += take;
            }
            if (jpos >= J.nprim) { ++jcur; jpos = 0; }
        }
        if (rows == 0) {
            if (jcur < jobs.size())   // cannot happen while cap_rows >= every split length
                return fail(ENCORE_EINVAL, "slice row cap below the coupling split length");
            break;
        }
        if ((rc = run_slice(x, pl, tb, edges, chunks, &t_gather, &t_couple))) return rc;
        ++nslice;
    }
    std::vector<double> sc;
    if (flags & ENCORE_NORMALIZE) {
        if ((rc = ensure(x.bscale, sizeof(double) * (size_t)(njobs * std::max<int64_t>(pl.nB, 1))))) return rc;
        for (int j = 0; j < njobs; ++j) {
            const DevGrid& g = jobs[j].grid->g;
            const double V = volume > 0.0 ? volume : g.Lx * g.Ly * g.Lz;
            std::vector<double> one = bin_scale(pl, edges, V);
            sc.insert(sc.end(), one.begin(), one.end());
        }
        HIPTRY(hipMemcpyAsync(x.bscale.p, sc.data(), sizeof(double) * sc.size(), hipMemcpyHostToDevice, s));
    }
    HIPTRY(hipEventRecord(x.ev[1], s));
    for (int j = 0; j < njobs; ++j) {
        const double* bs = (flags & ENCORE_NORMALIZE) ? (const double*)x.bscale.p + (size_t)j * pl.nB : nullptr;
        if ((rc = contract_job(x, pl, tb, (const double*)x.Tjob.p + (size_t)j * outs, bs,
                               (double*)x.zeta.p + (size_t)j * need)))
            return rc;
    }
    HIPTRY(hipEventRecord(x.ev[2], s));
    HIPTRY(hipMemcpyAsync(zeta, x.zeta.p, sizeof(double) * need * njobs, hipMemcpyDeviceToHost, s));
    HIPTRY(hipEventRecord(x.ev[3], s));
    HIPTRY(hipEventSynchronize(x.ev[3]));
    float ms_c = 0.f, ms_tot = 0.f;
    HIPTRY(hipEventElapsedTime(&ms_c, x.ev[1], x.ev[2]));
    HIPTRY(hipEventElapsedTime(&ms_tot, x.ev[0], x.ev[3]));
    unsigned long long pairs = 0;
    HIPTRY(hipMemcpy(&pairs, d_pairs, sizeof(pairs), hipMemcpyDeviceToHost));
    ctx->timings[0] = ms_tot;
    ctx->timings[1] = t_gather;
    ctx->timings[2] = t_couple;
    ctx->timings[3] = ms_c;
    ctx->timings[4] = nslice;
    ctx->timings[5] = (double)pairs;
    return ENCORE_OK;
}

}  // namespace encore

namespace {

// The hot path on the context's main exec, its cached tables and the default
// slice size (ctx->mu held).
int run_jobs(encore_ctx* ctx, const std::vector<JobRows>& jobs, const NpcfPlan& pl, uint32_t flags,
             const double* edges, double volume, double* zeta)
{
    DevTables* tb = nullptr;
    const int rc = get_tables_for(ctx, pl, &tb);
    if (rc) return rc;
    return run_jobs(ctx, ctx->main, tb, cap_rows(pl), jobs, pl, flags, edges, volume, zeta);
}

// Runs f with the main exec on the caller's stream (if any); ctx->mu is held.
template <typename F>
int on_stream(encore_ctx* ctx, void* stream, F&& f)
{
    hipStream_t own = ctx->main.s;
    if (stream) ctx->main.s = (hipStream_t)stream;
    const int rc = f();
    ctx->main.s = own;
    return rc;
}

}  // namespace

extern "C" {

const char* encore_last_error(void) { return get_error(); }

const char* encore_version(void) { return "encore-mi355x 0.2 (gfx950)"; }

int encore_create(int hip_device, encore_ctx** out)
{
    if (!out) return fail(ENCORE_EINVAL, "out is NULL");
    int ndev = 0;
    HIPTRY(hipGetDeviceCount(&ndev));
    if (hip_device < 0 || hip_device >= ndev)
        return fail(ENCORE_EINVAL, "hip_device out of range (" + std::to_string(ndev) + " devices)");
    HIPTRY(hipSetDevice(hip_device));
    int rc = noalloc_init(hip_device);   // the scratch address of encore_npcf_noalloc on this device
    if (rc) return rc;
    auto* c = new encore_ctx();
    c->device = hip_device;
    rc = exec_init(c->main);
    if (rc) {
        exec_release(c->main);
        delete c;
        return rc;
    }
    *out = c;
    return ENCORE_OK;
}

int encore_destroy(encore_ctx* ctx)
{
    if (!ctx) return ENCORE_OK;
    if (ctx->live_grids > 0) return fail(ENCORE_EINVAL, "free every grid before destroying the context");
    (void)hipSetDevice(ctx->device);
    mesh_release(ctx);
    exec_release(ctx->main);
    for (auto& kv : ctx->tables) {
        DevTables& d = kv.second;
        for (void* p : {(void*)d.tuple_off, (void*)d.tuple_flags, (void*)d.btab, (void*)d.term_start,
                        (void*)d.term_tuple, (void*)d.term_coef, (void*)d.kappa,
                        (void*)d.mf_rows, (void*)d.mf_cols, (void*)d.mf_tmap, (void*)d.mf_jobs[0],
                        (void*)d.mf_jobs[1], (void*)d.mf_jobs[2], (void*)d.mf_jobs[3]})
            if (p) (void)hipFree(p);
    }
    delete ctx;
    return ENCORE_OK;
}

int encore_build_grid(encore_ctx* ctx, const double* pos, const double* w, int64_t n, int64_t n_data,
                      const double* box, double r_max, uint32_t flags, void* stream, encore_grid** out)
{
    return build_grid_impl(ctx, pos, w, n, n_data, box, r_max, flags, stream, out, false);
}

int encore_build_grid_device(encore_ctx* ctx, const double* pos, const double* w, int64_t n,
                             int64_t n_data, const double* box, double r_max, uint32_t flags,
                             void* stream, encore_grid** out)
{
    return build_grid_impl(ctx, pos, w, n, n_data, box, r_max, flags, stream, out, true);
}

int encore_free_grid(encore_grid* grid)
{
    if (!grid) return ENCORE_OK;
    if (grid->plans > 0) return fail(ENCORE_EINVAL, "destroy the plans built on this grid first");
    (void)hipSetDevice(grid->ctx->device);
    (void)hipDeviceSynchronize();
    grid_free(grid->g);
    if (grid->rand_only) {
        grid_free(grid->rand_only->g);
        delete grid->rand_only;
    }
    grid->ctx->live_grids--;
    delete grid;
    return ENCORE_OK;
}

int64_t encore_grid_size(const encore_grid* grid)
{
    if (!grid) return fail(ENCORE_EINVAL, "grid is NULL");
    return grid->g.n;
}

int64_t encore_num_multiplets(int npcf, int lmax, uint32_t flags)
{
    if (npcf < 3 || npcf > 6) return fail(ENCORE_EINVAL, "npcf must be 3..6");
    if (!valid_lmax(npcf, lmax)) return fail(ENCORE_EINVAL, "lmax out of range for this N");
    return (int64_t)enumerate_multiplets(npcf, lmax, flags & ENCORE_ALLPARITY).size() /
           multiplet_width(npcf);
}

int64_t encore_num_bin_tuples(int npcf, int nbins)
{
    if (npcf < 3 || npcf > 6) return fail(ENCORE_EINVAL, "npcf must be 3..6");
    if (nbins < 0) return fail(ENCORE_EINVAL, "nbins < 0");
    return binomial(nbins, npcf - 1);
}

int encore_multiplet_table(int npcf, int lmax, uint32_t flags, int32_t* out, size_t out_len)
{
    if (npcf < 3 || npcf > 6) return fail(ENCORE_EINVAL, "npcf must be 3..6");
    if (!valid_lmax(npcf, lmax)) return fail(ENCORE_EINVAL, "lmax out of range for this N");
    std::vector<int32_t> t = enumerate_multiplets(npcf, lmax, flags & ENCORE_ALLPARITY);
    if (!out || out_len < t.size())
        return fail(ENCORE_ESIZE, "multiplet table needs " + std::to_string(t.size()) + " entries");
    std::copy(t.begin(), t.end(), out);
    return ENCORE_OK;
}

int encore_coupling_terms(int npcf, int lmax, uint32_t flags, int64_t* n_terms, int64_t cap,
                          int32_t* lam, int32_t* l, int32_t* m, double* coef)
{
    if (npcf < 3 || npcf > 6) return fail(ENCORE_EINVAL, "npcf must be 3..6");
    if (!valid_lmax(npcf, lmax)) return fail(ENCORE_EINVAL, "lmax out of range for this N");
    if (!n_terms) return fail(ENCORE_EINVAL, "n_terms is NULL");
    const TermTable& tt = term_table(npcf, lmax, flags & ENCORE_ALLPARITY);
    const int64_t nt = (int64_t)tt.coef.size();
    *n_terms = nt;
    if (!lam && !l && !m && !coef) return ENCORE_OK;
    if (!lam || !l || !m || !coef) return fail(ENCORE_EINVAL, "pass all four output arrays or none");
    if (cap < nt) return fail(ENCORE_ESIZE, "coupling terms need capacity " + std::to_string(nt));
    const int K = npcf - 1;
    std::copy(tt.lam.begin(), tt.lam.end(), lam);
    std::copy(tt.l.begin(), tt.l.begin() + nt * K, l);
    std::copy(tt.m.begin(), tt.m.begin() + nt * K, m);
    std::copy(tt.coef.begin(), tt.coef.end(), coef);
    return ENCORE_OK;
}

double encore_wigner3j(int j1, int j2, int j3, int m1, int m2, int m3)
{
    return wigner3j(j1, j2, j3, m1, m2, m3);
}

int encore_npcf(encore_ctx* ctx, const encore_grid* grid, int npcf, int lmax, int nbins,
                const double* edges, uint32_t flags, double volume, double* zeta, size_t zeta_len,
                const int64_t* primary_subset, int64_t n_subset, void* stream)
{
    if (!ctx || !grid) return fail(ENCORE_EINVAL, "NULL ctx or grid");
    NpcfPlan pl;
    int rc;
    if ((rc = plan_call(npcf, lmax, nbins, edges, flags, &pl))) return rc;
    pl.nbg = ctx_nbg(ctx, pl);
    if ((rc = check_grids(&grid, 1, ctx, edges, nbins, flags, volume))) return rc;
    const size_t need = (size_t)(pl.nlam * pl.nB);
    if (!zeta && need > 0) return fail(ENCORE_EINVAL, "zeta is NULL");
    if (zeta_len < need) return fail(ENCORE_ESIZE, "zeta needs " + std::to_string(need) + " elements");
    std::lock_guard<std::mutex> lock(ctx->mu);
    for (double& t : ctx->timings) t = 0.0;
    if (need == 0) return ENCORE_OK;
    HIPTRY(hipSetDevice(ctx->device));
    return on_stream(ctx, stream, [&]() {
        Exec& x = ctx->main;
        HIPTRY(hipEventRecord(x.ev[0], x.s));
        int64_t nprim = 0;
        int rc2;
        if ((rc2 = make_primaries(x, grid, primary_subset, n_subset, &nprim))) return rc2;
        std::vector<JobRows> jobs{JobRows{grid, (const int32_t*)x.prim.p, nprim}};
        return run_jobs(ctx, jobs, pl, flags, edges, volume, zeta);
    });
}

int encore_npcf_batch(encore_ctx* ctx, const encore_grid* const* grids, int njobs, int npcf, int lmax,
                      int nbins, const double* edges, uint32_t flags, double* zeta, size_t zeta_len,
                      const int64_t* const* primary_subsets, const int64_t* n_subsets, void* stream)
{
    if (!ctx || !grids) return fail(ENCORE_EINVAL, "NULL ctx or grids");
    if (njobs < 1) return fail(ENCORE_EINVAL, "njobs must be >= 1");
    if (primary_subsets && !n_subsets) return fail(ENCORE_EINVAL, "primary_subsets without n_subsets");
    auto subset_of = [&](int j) -> const int64_t* { return primary_subsets ? primary_subsets[j] : nullptr; };
    for (int j = 0; j < njobs; ++j)
        if (subset_of(j) && n_subsets[j] < 0) return fail(ENCORE_EINVAL, "n_subsets[j] < 0");
    NpcfPlan pl;
    int rc;
    if ((rc = plan_call(npcf, lmax, nbins, edges, flags, &pl))) return rc;
    pl.nbg = ctx_nbg(ctx, pl);
    if ((rc = check_grids(grids, njobs, ctx, edges, nbins, flags, 0.0))) return rc;
    const size_t need = (size_t)(pl.nlam * pl.nB);
    if (!zeta && need > 0) return fail(ENCORE_EINVAL, "zeta is NULL");
    if (zeta_len < need * (size_t)njobs)
        return fail(ENCORE_ESIZE, "zeta needs " + std::to_string(need * njobs) + " elements");
    std::lock_guard<std::mutex> lock(ctx->mu);
    for (double& t : ctx->timings) t = 0.0;
    if (need == 0) return ENCORE_OK;
    HIPTRY(hipSetDevice(ctx->device));
    return on_stream(ctx, stream, [&]() {
        Exec& x = ctx->main;
        HIPTRY(hipEventRecord(x.ev[0], x.s));
        // primaries: every point of a catalog in its grid's cell order, or the subset
        int64_t tot = 0;
        for (int j = 0; j < njobs; ++j) tot += subset_of(j) ? n_subsets[j] : grids[j]->g.n;
        int rc2;
        if ((rc2 = ensure(x.prim, sizeof(int32_t) * (size_t)std::max<int64_t>(tot, 1)))) return rc2;
        std::vector<JobRows> jobs(njobs);
        int64_t off = 0;
        for (int j = 0; j < njobs; ++j) {
            int64_t np = 0;
            int32_t* dst = (int32_t*)x.prim.p + off;
            if ((rc2 = fill_primaries(x, grids[j], subset_of(j), subset_of(j) ? n_subsets[j] : 0, dst, &np)))
                return rc2;
            jobs[j] = JobRows{grids[j], dst, np};
            off += np;
        }
        return run_jobs(ctx, jobs, pl, flags, edges, 0.0, zeta);
    });
}

int encore_npcf_splits(encore_ctx* ctx, const encore_grid* data_grid, const encore_grid* const* split_grids,
                       int nsplit, int npcf, int lmax, int nbins, const double* edges, uint32_t flags,
                       double volume, double* zeta, size_t zeta_len, double* zeta_splits,
                       size_t zeta_splits_len, void* stream)
{
    if (!ctx || !data_grid || !split_grids) return fail(ENCORE_EINVAL, "NULL ctx, data_grid or split_grids");
    if (nsplit < 1) return fail(ENCORE_EINVAL, "nsplit must be >= 1");
    NpcfPlan pl;
    int rc;
    if ((rc = plan_call(npcf, lmax, nbins, edges, flags, &pl))) return rc;
    pl.nbg = ctx_nbg(ctx, pl);
    if ((rc = check_grids(split_grids, nsplit, ctx, edges, nbins, flags, volume))) return rc;
    if ((rc = check_grids(&data_grid, 1, ctx, edges, nbins, 0u, 0.0))) return rc;
    const DevGrid& gD = data_grid->g;
    if (gD.dmr) return fail(ENCORE_EINVAL, "data_grid must be built without ENCORE_DMR");
    for (int k = 0; k < nsplit; ++k) {
        const DevGrid& g = split_grids[k]->g;
        const std::string which = "split grid " + std::to_string(k);
        if (!g.dmr || g.n_data != gD.n)
            return fail(ENCORE_EINVAL, which + ": needs ENCORE_DMR with n_data = the data grid's size");
        if (g.periodic != gD.periodic ||
            (g.periodic && (g.Lx != gD.Lx || g.Ly != gD.Ly || g.Lz != gD.Lz)))
            return fail(ENCORE_EINVAL, which + ": periodic box differs from the data grid's");
    }
    const size_t need = (size_t)(pl.nlam * pl.nB);
    if (!zeta && need > 0) return fail(ENCORE_EINVAL, "zeta is NULL");
    if (zeta_len < need) return fail(ENCORE_ESIZE, "zeta needs " + std::to_string(need) + " elements");
    if (zeta_splits && zeta_splits_len < need * (size_t)nsplit)
        return fail(ENCORE_ESIZE, "zeta_splits needs " + std::to_string(need * nsplit) + " elements");
    std::lock_guard<std::mutex> lock(ctx->mu);
    for (double& t : ctx->timings) t = 0.0;
    if (need == 0) return ENCORE_OK;
    HIPTRY(hipSetDevice(ctx->device));
    return on_stream(ctx, stream, [&]() {
        Exec& x = ctx->main;
        const hipStream_t s = x.s;
        int rc2;
        // every part's data are the data grid's
        if ((rc2 = ensure(x.misc, 64))) return rc2;
        int* d_bad = (int*)((char*)x.misc.p + 16);
        HIPTRY((hipError_t)launch_fill_u32((unsigned*)d_bad, 1, 0u, s));
        for (int k = 0; k < nsplit; ++k) HIPTRY((hipError_t)launch_split_check(split_grids[k]->g, gD, d_bad, s));
        int bad = 0;
        HIPTRY(hipMemcpyAsync(&bad, d_bad, sizeof(int), hipMemcpyDeviceToHost, s));
        HIPTRY(hipStreamSynchronize(s));
        if (bad)
            return fail(ENCORE_EINVAL, "a split grid's first n_data points differ from the data grid's "
                                       "(positions and weights, in input order)");
        // Keeping the data part pays where pairs dominate a work item's cost (dense
        // catalogs); at a few thousand points per r_max^3 the item's geometry work
        // dominates, and visiting the data-data pairs in every part costs less than
        // the extra data-only gather.  It is only taken with FP64 coefficients: the
        // data and random shares of a D-R coefficient are each far larger than their
        // sum, so adding two FP32 sums loses what one interleaved FP32 sum keeps
        // (measured: 1.6e-3 against 1e-6 of max|Z| on a dense catalog).
        // ENCORE_SPLIT_CACHE=0 / 1 forces the choice.
        double dens = 0.0;
        for (int k = 0; k < nsplit; ++k) {
            const DevGrid& S = split_grids[k]->g;
            const double V = (S.ncx * S.csx) * (S.ncy * S.csy) * (S.ncz * S.csz);
            dens += (double)S.n / V / nsplit;
        }
        const double rmax = edges[nbins];
        bool use_cache = pl.prec == 0 && dens * rmax * rmax * rmax >= kSplitCacheDensity;
        if (const char* e = getenv("ENCORE_SPLIT_CACHE")) use_cache = atoi(e) != 0;
        if (!use_cache) {
            // each part as one catalog; the mean in part order
            int64_t nmax = 0;
            for (int k = 0; k < nsplit; ++k) nmax = std::max<int64_t>(nmax, split_grids[k]->g.n);
            if ((rc2 = ensure(x.prim, sizeof(int32_t) * (size_t)nmax))) return rc2;
            HIPTRY((hipError_t)launch_iota((int32_t*)x.prim.p, nmax, s));
            HIPTRY(hipEventRecord(x.ev[0], s));
            std::vector<JobRows> jobs(nsplit);
            for (int k = 0; k < nsplit; ++k)
                jobs[k] = JobRows{split_grids[k], (const int32_t*)x.prim.p, split_grids[k]->g.n};
            std::vector<double> zk(need * (size_t)nsplit);
            if ((rc2 = run_jobs(ctx, jobs, pl, flags, edges, volume, zk.data()))) return rc2;
            for (size_t i = 0; i < need; ++i) {
                double acc = 0.0;
                for (int k = 0; k < nsplit; ++k) acc += zk[(size_t)k * need + i];
                zeta[i] = acc / nsplit;
            }
            if (zeta_splits) std::copy(zk.begin(), zk.end(), zeta_splits);
            return ENCORE_OK;
        }
        // each part's randoms alone (their D-R weights), built once per split grid
        for (int k = 0; k < nsplit; ++k) {
            const encore_grid* sg = split_grids[k];
            if (sg->rand_only) continue;
            const DevGrid& S = sg->g;
            const int64_t nr = S.n - S.n_data;
            double* d_pos = nullptr;
            double* d_w = nullptr;
            HIPTRY(hipMalloc(&d_pos, sizeof(double) * 3 * nr));
            hipError_t e = hipMalloc(&d_w, sizeof(double) * nr);
            if (e == hipSuccess) e = (hipError_t)launch_split_randoms(S, d_pos, d_w, s);
            auto* rg = new encore_grid();
            rg->ctx = ctx;
            int rcb = e == hipSuccess ? ENCORE_OK : hip_fail(e, "split randoms");
            if (rcb == ENCORE_OK) {
                const double box[3] = {S.Lx, S.Ly, S.Lz};
                double div = 0.0, xsub = 0.0;
                ctx_cells(ctx, &div, &xsub);
                rcb = build_grid_dev(ctx->device, d_pos, d_w, nr, 0, false, S.periodic ? box : nullptr, S.r_max,
                                     div, xsub, s, rg->g);
            }
            (void)hipStreamSynchronize(s);
            if (d_pos) (void)hipFree(d_pos);
            if (d_w) (void)hipFree(d_w);
            if (rcb) {
                delete rg;
                return rcb;
            }
            sg->rand_only = rg;
        }
        HIPTRY(hipEventRecord(x.ev[0], s));
        DevTables* tb = nullptr;
        if ((rc2 = get_tables_for(ctx, pl, &tb))) return rc2;
        int64_t nmax = gD.n;
        for (int k = 0; k < nsplit; ++k) nmax = std::max<int64_t>(nmax, split_grids[k]->rand_only->g.n);
        if ((rc2 = ensure(x.prim, sizeof(int32_t) * (size_t)nmax))) return rc2;
        int32_t* prim = (int32_t*)x.prim.p;   // 0, 1, 2, ...: every point of a grid in its cell order
        HIPTRY((hipError_t)launch_iota(prim, nmax, s));

        // the data part of a~ of every data primary, gathered once into x.cache
        // (row p: the data grid's point p)
        const size_t rb = alm_row_bytes(pl);
        if ((rc2 = ensure(x.cache, rb * (size_t)gD.n))) return rc2;
        const int64_t cap = cap_rows(pl);
        unsigned long long* d_pairs = (unsigned long long*)x.misc.p;
        HIPTRY((hipError_t)launch_fill((double*)d_pairs, 1, 0.0, s));
        HIPTRY(hipEventRecord(x.ev[1], s));
        for (int64_t r0 = 0; r0 < gD.n; r0 += cap) {
            const int64_t r1 = std::min<int64_t>(gD.n, r0 + cap);
            std::vector<Chunk> chunks{Chunk{&gD, prim, r0, r1, r1 - r0, nullptr}};
            SliceLaunch L;
            if ((rc2 = prepare_slice(x, x.segs, x.splits, x.redp, pl, tb, edges, chunks, L))) return rc2;
            L.ga.alm = (char*)x.cache.p + (size_t)r0 * rb;
            if ((rc2 = launch_slice_gather(L, pl, s))) return rc2;
            HIPTRY(hipStreamSynchronize(s));   // the slice tables are rewritten by the next slice
        }
        HIPTRY(hipEventRecord(x.ev[2], s));
        HIPTRY(hipEventSynchronize(x.ev[2]));
        float ms_cache = 0.f;
        HIPTRY(hipEventElapsedTime(&ms_cache, x.ev[1], x.ev[2]));
        unsigned long long pairs_cache = 0;
        HIPTRY(hipMemcpy(&pairs_cache, d_pairs, sizeof(pairs_cache), hipMemcpyDeviceToHost));

        // per part two jobs: the data primaries against the part's randoms (plus
        // their cached rows), and the part's random primaries against data + randoms
        std::vector<JobRows> jobs(2 * (size_t)nsplit);
        for (int k = 0; k < nsplit; ++k) {
            const encore_grid* R = split_grids[k]->rand_only;
            jobs[2 * k] = JobRows{R, prim, gD.n, gD.P, x.cache.p};
            jobs[2 * k + 1] = JobRows{split_grids[k], prim, R->g.n, R->g.P, nullptr};
        }
        std::vector<double> zs(need * 2 * (size_t)nsplit);
        if ((rc2 = run_jobs(ctx, jobs, pl, flags, edges, volume, zs.data()))) return rc2;
        ctx->timings[1] += ms_cache;
        ctx->timings[5] += (double)pairs_cache;
        // Z of a part = data primaries' + random primaries' sums; the mean over the
        // parts in part order
        std::vector<double> zk(need * (size_t)nsplit);
        for (int k = 0; k < nsplit; ++k)
            for (size_t i = 0; i < need; ++i)
                zk[(size_t)k * need + i] = zs[(size_t)(2 * k) * need + i] + zs[(size_t)(2 * k + 1) * need + i];
        for (size_t i = 0; i < need; ++i) {
            double acc = 0.0;
            for (int k = 0; k < nsplit; ++k) acc += zk[(size_t)k * need + i];
            zeta[i] = acc / nsplit;
        }
        if (zeta_splits) std::copy(zk.begin(), zk.end(), zeta_splits);
        return ENCORE_OK;
    });
}

int encore_mfma_plan_stats(int npcf, int lmax, int nbins, uint32_t flags, int64_t* out, size_t out_len)
{
    if (!out || out_len < 4) return fail(ENCORE_ESIZE, "out needs 4 elements");
    if (npcf < 3 || npcf > 6) return fail(ENCORE_EINVAL, "npcf must be 3..6");
    if (!valid_lmax(npcf, lmax)) return fail(ENCORE_EINVAL, "lmax out of range for this N");
    if (nbins < 1 || nbins > kMaxBins) return fail(ENCORE_EINVAL, "nbins out of range");
    if (nbins * (lmax + 1) * (lmax + 2) / 2 > kMfmaMaxAllEntries)
        return fail(ENCORE_EUNSUPPORTED, "too many coefficients per primary for the MFMA coupling");
    int rc;
    if (use_gemm_coupling(npcf)) {
        GemmPlan G;
        if ((rc = build_gemm_plan(npcf, lmax, flags & ENCORE_ALLPARITY, nbins, gemm_split(npcf), G))) return rc;
        int64_t ops = 0;
        for (size_t m = 0; m < G.macros.size() / kGemmMacroWidth; ++m)
            ops += G.macros[m * kGemmMacroWidth + 2] + G.macros[m * kGemmMacroWidth + 3];
        out[0] = G.ntiles;
        out[1] = ops;
        out[2] = (int64_t)G.tmap.size();
        out[3] = G.ntiles * 256;
        return ENCORE_OK;
    }
    MfmaPlan P;
    if ((rc = build_mfma_plan(npcf, lmax, flags & ENCORE_ALLPARITY, nbins, P))) return rc;
    int64_t tiles = 0, rts = 0;
    for (int sh = 0; sh < kNumMfmaShapes; ++sh)
        for (size_t j = 0; j < P.jobs[sh].size() / kMfmaJobWidth; ++j) {
            const int nrt = P.jobs[sh][j * kMfmaJobWidth + 3];
            rts += nrt;
            tiles += (int64_t)nrt * kMfmaShapes[sh].NC;
        }
    out[0] = tiles;
    out[1] = rts;
    out[2] = (int64_t)P.tmap.size();
    out[3] = P.ntiles * 256;
    return ENCORE_OK;
}

int encore_autotune(encore_ctx* ctx, const double* pos, const double* w, int64_t n, int64_t n_data,
                    const double* box, int npcf, int lmax, int nbins, const double* edges, uint32_t flags,
                    int64_t n_sample, double* report, size_t report_len)
{
    if (!ctx || !pos || !w) return fail(ENCORE_EINVAL, "NULL ctx, pos or w");
    if (n < 1) return fail(ENCORE_EINVAL, "n must be >= 1");
    if (report && report_len < 5) return fail(ENCORE_ESIZE, "report needs 5 elements");
    NpcfPlan pl;
    int rc;
    if ((rc = plan_call(npcf, lmax, nbins, edges, flags, &pl))) return rc;
    const bool periodic = flags & ENCORE_PERIODIC;
    if (periodic && !box) return fail(ENCORE_EINVAL, "ENCORE_PERIODIC needs box");
    const double r_max = edges[nbins];
    if (periodic)
        for (int a = 0; a < 3; ++a) {
            if (!(box[a] > 0.0) || !std::isfinite(box[a])) return fail(ENCORE_EINVAL, "box must be finite and > 0");
            if (2.0 * r_max > box[a])
                return fail(ENCORE_EINVAL, "periodic box: edges[nbins] must be <= box/2 on every axis");
        }
    const int gprec = gather_precision(pl.prec);
    const std::vector<int> nbgs = gather_nbg_options(lmax, gprec);
    // cell shapes tried: (y/z divisor of r_max, extra x subdivision); the default first
    constexpr double kTuneMargin = 0.98;
    static const double kCells[][2] = {{5, 16}, {5, 8}, {6, 16}, {6, 8}, {8, 8}, {8, 4}, {5, 24}, {4, 16}};
    // The sample: 16 runs of consecutive cell-sorted primaries spread over the grid,
    // so that neighbouring work items share cells as in a full pass (a scattered
    // sample would time cache misses that a full pass does not have).
    const int64_t k = std::min<int64_t>(n, std::max<int64_t>(1, n_sample));
    const int64_t runs = std::min<int64_t>(16, k);
    std::vector<int32_t> sample;
    sample.reserve(k);
    for (int64_t q = 0; q < runs; ++q) {
        const int64_t len = k / runs + (q < k % runs ? 1 : 0);
        const int64_t start = runs > 1 ? (n - len) * q / (runs - 1) : 0;
        for (int64_t j = 0; j < len; ++j) sample.push_back((int32_t)(start + j));
    }
    const size_t need = (size_t)std::max<int64_t>(pl.nlam * pl.nB, 1);
    std::vector<double> ztmp(need);
    std::lock_guard<std::mutex> lock(ctx->mu);
    HIPTRY(hipSetDevice(ctx->device));
    Exec& x = ctx->main;
    const hipStream_t s = x.s;
    double* d_pos = nullptr;
    double* d_w = nullptr;
    HIPTRY(hipMalloc(&d_pos, sizeof(double) * 3 * n));
    hipError_t e = hipMalloc(&d_w, sizeof(double) * n);
    if (e == hipSuccess) e = hipMemcpyAsync(d_pos, pos, sizeof(double) * 3 * n, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(d_w, w, sizeof(double) * n, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) {
        if (d_pos) (void)hipFree(d_pos);
        if (d_w) (void)hipFree(d_w);
        return hip_fail(e, "encore_autotune: catalog upload");
    }
    double best = 1e300, best_div = 0, best_xsub = 0, dflt = 0;
    int best_nbg = 0;
    rc = ENCORE_OK;
    for (const auto& cell : kCells) {
        encore_grid tg;
        tg.ctx = ctx;
        rc = build_grid_dev(ctx->device, d_pos, d_w, n, n_data, (flags & ENCORE_DMR) != 0,
                            periodic ? box : nullptr, r_max, cell[0], cell[1], s, tg.g);
        if (rc == ENCORE_OK) rc = check_grid_edges(tg.g, edges, nbins);
        if (rc) {
            if (tg.g.P) grid_free(tg.g);
            break;
        }
        const int64_t np = k;
        rc = ensure(x.prim, sizeof(int32_t) * (size_t)k);
        if (rc == ENCORE_OK) {
            const hipError_t ce = hipMemcpyAsync(x.prim.p, sample.data(), sizeof(int32_t) * (size_t)k,
                                                 hipMemcpyHostToDevice, s);
            if (ce != hipSuccess) rc = hip_fail(ce, "encore_autotune: sample upload");
        }
        if (rc == ENCORE_OK) {
            for (size_t q = 0; q < nbgs.size() && rc == ENCORE_OK; ++q) {
                pl.nbg = nbgs[q];
                double t = 1e300;
                for (int rep = 0; rep < 3 && rc == ENCORE_OK; ++rep) {
                    std::vector<JobRows> jobs{JobRows{&tg, (const int32_t*)x.prim.p, np}};
                    HIPTRY(hipEventRecord(x.ev[0], s));
                    rc = run_jobs(ctx, jobs, pl, flags & ~ENCORE_NORMALIZE, edges, 0.0, ztmp.data());
                    t = std::min(t, ctx->timings[1] + ctx->timings[2]);
                }
                if (&cell == &kCells[0] && q == 0) dflt = t;
                if (rc == ENCORE_OK && t < best) {
                    best = t; best_div = cell[0]; best_xsub = cell[1]; best_nbg = nbgs[q];
                }
            }
        }
        (void)hipStreamSynchronize(s);
        grid_free(tg.g);
        if (rc) break;
    }
    (void)hipFree(d_pos);
    (void)hipFree(d_w);
    if (rc) return rc;
    // a shape replaces the default only when it is clearly faster on the sample:
    // the shapes near the best differ by about as much as repeated timings do, and
    // a sample-noise pick can be slower on the full pass
    if (!(best < kTuneMargin * dflt)) {
        best = dflt; best_div = kCells[0][0]; best_xsub = kCells[0][1]; best_nbg = nbgs[0];
    }
    {
        std::lock_guard<std::mutex> tl(ctx->tab_mu);
        ctx->cell_div = best_div;
        ctx->cell_xsub = best_xsub;
        ctx->tuned_nbg[std::make_tuple(lmax, gprec, nbins)] = best_nbg;
    }
    if (report) {
        report[0] = best_div;
        report[1] = best_xsub;
        report[2] = best_nbg;
        report[3] = best;
        report[4] = dflt;
    }
    return ENCORE_OK;
}

int encore_npcf_simple(const double* pos, const double* w, int64_t n, int npcf, int lmax, int nbins,
                       const double* edges, const double* box, uint32_t flags, double* zeta,
                       size_t zeta_len)
{
    int rc;
    if ((rc = check_edges(edges, nbins))) return rc;
    encore_ctx* ctx = nullptr;
    if ((rc = encore_create(0, &ctx))) return rc;
    encore_grid* g = nullptr;
    const uint32_t gflags = box ? ENCORE_PERIODIC : 0u;
    if ((rc = encore_build_grid(ctx, pos, w, n, 0, box, edges[nbins], gflags, nullptr, &g))) {
        encore_destroy(ctx);
        return rc;
    }
    rc = encore_npcf(ctx, g, npcf, lmax, nbins, edges, flags, 0.0, zeta, zeta_len, nullptr, 0, nullptr);
    std::string err = rc ? get_error() : "";
    encore_free_grid(g);
    encore_destroy(ctx);
    if (rc) set_error(err);
    return rc;
}

int encore_debug_alm(encore_ctx* ctx, const encore_grid* grid, int lmax, int nbins, const double* edges,
                     uint32_t flags, const int64_t* primaries, int64_t k, double* alm_out)
{
    if (!ctx || !grid) return fail(ENCORE_EINVAL, "NULL ctx or grid");
    if (lmax < 0 || lmax > kMaxLmax) return fail(ENCORE_EINVAL, "lmax must be 0..10");
    int rc;
    if ((rc = check_edges(edges, nbins))) return rc;
    if ((rc = check_grid_edges(grid->g, edges, nbins))) return rc;
    int cprec = 0;
    if ((rc = precision_of(flags, &cprec))) return rc;
    const int prec = gather_precision(cprec);   // the gather encore_npcf runs for this precision
    if (!primaries || k < 1 || !alm_out) return fail(ENCORE_EINVAL, "need k >= 1 primaries and alm_out");
    const bool full = flags & ENCORE_DEBUG_FULLGRID;
    std::lock_guard<std::mutex> lock(ctx->mu);
    HIPTRY(hipSetDevice(ctx->device));
    Exec& x = ctx->main;
    const hipStream_t s = x.s;
    const int nlm = (lmax + 1) * (lmax + 2) / 2;
    const int64_t per = (int64_t)nbins * nlm * 2;     // reals per primary
    // requested rows -> sorted indices (x.prim), validated
    int64_t np = 0;
    if ((rc = make_primaries(x, grid, primaries, k, &np))) return rc;
    std::vector<int32_t> sorted_rows(k);
    HIPTRY(hipMemcpy(sorted_rows.data(), x.prim.p, sizeof(int32_t) * k, hipMemcpyDeviceToHost));
    const int64_t nlaunch = full ? grid->g.n : k;
    if (full && (rc = make_primaries(x, grid, nullptr, 0, &np))) return rc;
    if ((rc = ensure(x.alm, (size_t)(nlaunch * per) * (prec == 0 ? 8 : 4)))) return rc;   // FP32 out for 1, 2
    if ((rc = ensure(x.zeta, sizeof(double) * (size_t)(nlaunch * per)))) return rc;
    if ((rc = ensure(x.wprim, sizeof(double) * (size_t)nlaunch))) return rc;
    if ((rc = ensure(x.segs, sizeof(GatherSeg)))) return rc;
    std::vector<double> kap(nlm);
    gather_tables(lmax, kap.data());
    double* d_kg = nullptr;
    HIPTRY(hipMalloc(&d_kg, sizeof(double) * nlm));
    hipError_t e = hipMemcpy(d_kg, kap.data(), sizeof(double) * nlm, hipMemcpyHostToDevice);
    const DevGrid& g = grid->g;
    GatherSeg gs;
    memset(&gs, 0, sizeof(gs));
    gs.P = g.P; gs.Pq = g.P; gs.nP = (int)g.n; gs.cell_start = g.cell_start; gs.prim = (const int32_t*)x.prim.p;
    gs.ncx = g.ncx; gs.ncy = g.ncy; gs.ncz = g.ncz; gs.periodic = g.periodic;
    gs.ox = g.ox; gs.oy = g.oy; gs.oz = g.oz;
    gs.csx = g.csx; gs.csy = g.csy; gs.csz = g.csz;
    gs.Lx = g.Lx; gs.Ly = g.Ly; gs.Lz = g.Lz;
    gs.row0 = 0; gs.nprim = (int)nlaunch;
    finish_seg(gs);
    if (e == hipSuccess) e = hipMemcpy(x.segs.p, &gs, sizeof(gs), hipMemcpyHostToDevice);
    GatherArgs ga;
    memset(&ga, 0, sizeof(ga));
    ga.nbins = nbins;
    for (int b = 0; b <= nbins; ++b) {
        ga.e2[b] = edges[b] * edges[b];
        ga.e1[b] = edges[b];
    }
    ga.kappa = d_kg;
    ga.alm = x.alm.p;
    ga.wprim = (double*)x.wprim.p;
    ga.segs = (const GatherSeg*)x.segs.p;
    ga.nseg = 1;
    ga.nrows = (int)nlaunch;
    NpcfPlan gpl;
    gpl.lmax = lmax; gpl.prec = cprec; gpl.nbins = nbins;
    const int nbg = ctx_nbg(ctx, gpl);   // the configuration encore_npcf launches
    if (e == hipSuccess) e = (hipError_t)launch_gather(ga, lmax, prec, nbg, false, s);
    if (e == hipSuccess)
        e = (hipError_t)launch_to_double(x.alm.p, prec == 0 ? 0 : 1, nlaunch * per, (double*)x.zeta.p, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    for (int64_t r = 0; r < k && e == hipSuccess; ++r) {
        // full launch: row of sorted index sorted_rows[r]; else row r
        const int64_t row = full ? sorted_rows[r] : r;
        e = hipMemcpy(alm_out + r * per, (double*)x.zeta.p + row * per, sizeof(double) * per,
                      hipMemcpyDeviceToHost);
    }
    (void)hipFree(d_kg);
    if (e != hipSuccess) return hip_fail(e, "encore_debug_alm");
    return ENCORE_OK;
}

int encore_last_timings(const encore_ctx* ctx, double* out, size_t out_len)
{
    if (!ctx || !out) return fail(ENCORE_EINVAL, "NULL ctx or out");
    if (out_len < 6) return fail(ENCORE_ESIZE, "timings need 6 entries");
    for (int i = 0; i < 6; ++i) out[i] = ctx->timings[i];
    return ENCORE_OK;
}

}  // extern "C"
