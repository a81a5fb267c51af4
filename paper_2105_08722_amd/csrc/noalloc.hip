// Allocation-free form of encore_npcf (encore_npcf_noalloc): every device buffer
// of the call -- coupling tables, primary list, harmonic coefficients of a slice,
// coupling partial sums, the per-job sums and zeta -- is carved from one static
// device array of fixed size, so the call makes no device allocation and frees
// nothing.  The array is a file-scope __device__ variable: each GPU that loads the
// library holds its own copy, at its own address, until the process ends.  Host
// code must never use the array's name as a device address; the address of each
// device's copy is looked up once per device (noalloc_init, from encore_create)
// and only that address is passed to kernels and copies.
//
// Calls that overlap on one GPU share the array and race; calls on one context
// are serialised by the context's lock.  Nothing in the array is assumed to be
// zero: every buffer the hot path accumulates into is cleared by a fill kernel
// on the call's stream first, as in encore_npcf.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "engine.h"

namespace encore {

namespace {

constexpr size_t kScratchBytes = (size_t)256 << 20;   // 256 MiB per device

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
std::map<int, char*> g_scratch;   // device -> address of that device's copy of scratch

char* scratch_of(int device)
{
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch.find(device);
    return it == g_scratch.end() ? nullptr : it->second;
}

// Device bytes one slice of `rows` rows needs (as prepare_slice sizes them) and
// the rows such a slice takes, for a job of nprim primaries and slice cap `cap`.
struct SliceNeed {
    int64_t rows = 0, nsplit = 0, split_rows = 0;
    size_t bytes = 0;
};

SliceNeed slice_need(const NpcfPlan& pl, const DevTables* tb, int64_t nprim, int64_t cap)
{
    SliceNeed n;
    n.split_rows = job_split_rows(pl, tb, nprim, cap);
    n.rows = std::min<int64_t>(nprim, std::max<int64_t>(cap / n.split_rows, 1) * n.split_rows);
    n.nsplit = (n.rows + n.split_rows - 1) / n.split_rows;
    const size_t align = 256;
    auto up = [&](size_t b) { return (std::max<size_t>(b, 256) + align - 1) / align * align; };
    n.bytes = up(alm_row_bytes(pl) * (size_t)n.rows) + up(sizeof(double) * (size_t)n.rows) +
              up(sizeof(double) * (size_t)n.nsplit * (size_t)acc_len(pl, tb)) + up(sizeof(GatherSeg)) +
              up(sizeof(int32_t) * (size_t)(2 * n.nsplit + 2)) + up(sizeof(double*)) + 2 * up(64);
    if (pl.prec == 2) {
        const int64_t nblk = (n.rows + kBlkRows - 1) / kBlkRows;
        n.bytes += up((size_t)nblk * blk_bytes(tb->mf_nent) + 1024);
    }
    return n;
}

}  // namespace

int noalloc_init(int device)
{
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch.count(device)) return ENCORE_OK;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));   // on the current device
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    g_scratch[device] = static_cast<char*>(p);
    return ENCORE_OK;
}

size_t noalloc_scratch_bytes() { return kScratchBytes; }

}  // namespace encore

using namespace encore;

extern "C" int encore_npcf_noalloc(encore_ctx* ctx, const encore_grid* grid, int npcf, int lmax, int nbins,
                                   const double* edges, uint32_t flags, double volume, double* zeta,
                                   size_t zeta_len, const int64_t* primary_subset, int64_t n_subset,
                                   void* stream)
{
    if (!ctx || !grid) return fail(ENCORE_EINVAL, "NULL ctx or grid");
    if (grid->ctx != ctx) return fail(ENCORE_EINVAL, "grid belongs to another context");
    NpcfPlan pl;
    int rc;
    if ((rc = plan_call(npcf, lmax, nbins, edges, flags, &pl))) return rc;
    pl.nbg = ctx_nbg(ctx, pl);
    if ((rc = check_grid_edges(grid->g, edges, nbins))) return rc;
    if ((flags & ENCORE_NORMALIZE) && !(volume > 0.0) && !grid->g.periodic)
        return fail(ENCORE_EINVAL, "ENCORE_NORMALIZE needs volume > 0 without a periodic box");
    if (primary_subset && n_subset < 0) return fail(ENCORE_EINVAL, "n_subset < 0");
    const size_t need = (size_t)(pl.nlam * pl.nB);
    if (!zeta && need > 0) return fail(ENCORE_EINVAL, "zeta is NULL");
    if (zeta_len < need) return fail(ENCORE_ESIZE, "zeta needs " + std::to_string(need) + " elements");
    std::lock_guard<std::mutex> lock(ctx->mu);
    for (double& t : ctx->timings) t = 0.0;
    if (need == 0) return ENCORE_OK;
    HIPTRY(hipSetDevice(ctx->device));
    char* base = scratch_of(ctx->device);
    if (!base) return fail(ENCORE_EDEVICE, "no scratch address for this device");
    Arena A;
    A.base = base;
    A.size = kScratchBytes;
    Exec x;
    x.s = stream ? (hipStream_t)stream : ctx->main.s;
    for (int i = 0; i < 4; ++i) x.ev[i] = ctx->main.ev[i];
    exec_use_arena(x, &A);

    HIPTRY(hipEventRecord(x.ev[0], x.s));
    DevTables tb;
    if ((rc = tables_in_arena(A, x.s, pl, tb))) return rc;
    const int64_t nprim = primary_subset ? n_subset : grid->g.n;
    if ((rc = ensure(x.prim, sizeof(int32_t) * (size_t)std::max<int64_t>(nprim, 1)))) return rc;
    if ((rc = ensure(x.misc, sizeof(int64_t) * (size_t)std::max<int64_t>(primary_subset ? n_subset : 0, 1) + 16)))
        return rc;
    int64_t np = 0;
    if ((rc = fill_primaries(x, grid, primary_subset, n_subset, (int32_t*)x.prim.p, &np))) return rc;
    // the job's sums, zeta and the normalisation table (run_jobs sizes them so)
    const int64_t outs = acc_len(pl, &tb);
    if ((rc = ensure(x.Tjob, sizeof(double) * (size_t)outs))) return rc;
    if ((rc = ensure(x.zeta, sizeof(double) * need))) return rc;
    if ((flags & ENCORE_NORMALIZE) && (rc = ensure(x.bscale, sizeof(double) * (size_t)std::max<int64_t>(pl.nB, 1))))
        return rc;
    // Slices as encore_npcf cuts them when they fit what is left (then the results
    // are the same bits), else the largest that fits (binary search over the row
    // cap); every slice workspace is carved now at that size, so the slices carve
    // nothing.
    const size_t left = A.size - std::min(A.size, (A.used + 255) / 256 * 256);
    const int64_t npx = std::max<int64_t>(np, 1);
    const int64_t step = pl.prec == 2 ? kBlkRows : 1;
    int64_t cap = cap_rows(pl);
    bool fits = slice_need(pl, &tb, npx, cap).bytes <= left;
    if (!fits) {
        int64_t lo = 0, hi = npx;
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) / 2;
            const int64_t c = std::max<int64_t>(mid / step * step, step);
            if (slice_need(pl, &tb, npx, c).bytes <= left) lo = mid;
            else hi = mid - 1;
        }
        cap = std::max<int64_t>(lo / step * step, step);
        fits = lo > 0 && slice_need(pl, &tb, npx, cap).bytes <= left;
    }
    const SliceNeed sn = slice_need(pl, &tb, npx, cap);
    if (!fits)
        return fail(ENCORE_ESIZE, "the call needs " + std::to_string(sn.bytes + A.used) +
                                      " bytes of device workspace, more than the " +
                                      std::to_string(kScratchBytes >> 20) +
                                      " MiB scratch buffer of the allocation-free entry point");
    if ((rc = ensure(x.alm, alm_row_bytes(pl) * (size_t)sn.rows)) ||
        (rc = ensure(x.wprim, sizeof(double) * (size_t)sn.rows)) ||
        (rc = ensure(x.T, sizeof(double) * (size_t)sn.nsplit * (size_t)outs)) ||
        (rc = ensure(x.segs, sizeof(GatherSeg))) || (rc = ensure(x.splits, sizeof(int32_t) * (size_t)(2 * sn.nsplit + 2))) ||
        (rc = ensure(x.redp, sizeof(double*))) || (rc = ensure(x.queues, 64)))
        return rc;
    if (pl.prec == 2 &&
        (rc = ensure(x.almb, (size_t)((sn.rows + kBlkRows - 1) / kBlkRows) * blk_bytes(tb.mf_nent) + 1024)))
        return rc;
    std::vector<JobRows> jobs{JobRows{grid, (const int32_t*)x.prim.p, np}};
    return run_jobs(ctx, x, &tb, cap, jobs, pl, flags, edges, volume, zeta);
}
