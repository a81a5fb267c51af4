// Host-side execution engine: tables on the device, workspaces, and the slice
// runner shared by the synchronous entry points and the server.
#include "engine.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <type_traits>

namespace encore {

static thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }
const char* get_error() { return g_err.c_str(); }

int fail(int code, const std::string& msg)
{
    set_error(msg);
    return code;
}

int hip_fail(hipError_t e, const char* what)
{
    return fail(e == hipErrorOutOfMemory ? ENCORE_ENOMEM : ENCORE_EDEVICE,
                std::string(what) + ": " + hipGetErrorString(e));
}

int arena_take(Arena& A, size_t bytes, void** p)
{
    const size_t off = (A.used + 255) / 256 * 256;
    if (off > A.size || bytes > A.size - off)
        return fail(ENCORE_ESIZE, "the call needs more than the " + std::to_string(A.size >> 20) +
                                      " MiB scratch buffer of the allocation-free entry point");
    *p = A.base + off;
    A.used = off + bytes;
    return ENCORE_OK;
}

int ensure(Buf& b, size_t bytes)
{
    if (b.n >= bytes && b.p) return ENCORE_OK;
    if (b.arena) {   // carved from fixed memory: never allocated or freed
        const size_t want = std::max<size_t>(bytes, 256);
        const int rc = arena_take(*b.arena, want, &b.p);
        if (rc) return rc;
        b.n = want;
        return ENCORE_OK;
    }
    dev_free(b.p, b.pool, b.s);
    b.p = nullptr;
    b.n = 0;
    // pooled buffers grow by at least half, so a lane settles after a few slices
    const size_t want = std::max<size_t>(b.pool ? std::max(bytes, bytes / 2 * 3) : bytes, 256);
    hipError_t e = dev_alloc(&b.p, want, b.pool, b.s);
    if (e != hipSuccess) {
        b.p = nullptr;
        return hip_fail(e, "workspace allocation");
    }
    b.n = want;
    return ENCORE_OK;
}

static Buf* exec_bufs(Exec& x, int i)
{
    Buf* all[] = {&x.alm, &x.wprim, &x.T, &x.segs, &x.splits, &x.redp, &x.queues,
                  &x.misc, &x.zeta, &x.bscale, &x.prim, &x.Tjob, &x.almb, &x.cache, &x.cmap,
                  &x.mesh, &x.meshd, &x.meshk, &x.egt, &x.eA, &x.eM, &x.eio};
    return i < (int)(sizeof(all) / sizeof(all[0])) ? all[i] : nullptr;
}

int exec_init(Exec& x, hipMemPool_t pool)
{
    HIPTRY(hipStreamCreateWithFlags(&x.s, hipStreamNonBlocking));
    for (int i = 0; i < 4; ++i) HIPTRY(hipEventCreate(&x.ev[i]));
    for (int i = 0; Buf* b = exec_bufs(x, i); ++i) {
        b->pool = pool;
        b->s = x.s;
    }
    return ENCORE_OK;
}

void exec_use_arena(Exec& x, Arena* A)
{
    for (int i = 0; Buf* b = exec_bufs(x, i); ++i) {
        b->arena = A;
        b->pool = nullptr;
        b->s = x.s;
    }
}

void exec_release(Exec& x)
{
    for (int i = 0; Buf* b = exec_bufs(x, i); ++i) {
        if (!b->arena) dev_free(b->p, b->pool, x.s);
        b->p = nullptr;
        b->n = 0;
    }
    if (x.s) (void)hipStreamSynchronize(x.s);
    for (int i = 0; i < 4; ++i) {
        if (x.ev[i]) (void)hipEventDestroy(x.ev[i]);
        x.ev[i] = nullptr;
    }
    if (x.s) (void)hipStreamDestroy(x.s);
    x.s = nullptr;
}

size_t exec_bytes(const Exec& x)
{
    size_t t = 0;
    for (int i = 0; Buf* b = exec_bufs(const_cast<Exec&>(x), i); ++i) t += b->n;
    return t;
}

bool valid_lmax(int N, int lmax)
{
    if (lmax < 0) return false;
    switch (N) {
    case 3: case 4: return lmax <= kMaxLmax;
    case 5: return lmax <= 5;
    case 6: return lmax <= 4;
    }
    return false;
}

int check_edges(const double* edges, int nbins)
{
    if (!edges) return fail(ENCORE_EINVAL, "edges is NULL");
    if (nbins < 1 || nbins > kMaxBins)
        return fail(ENCORE_EINVAL, "nbins must be in 1.." + std::to_string(kMaxBins));
    if (!(edges[0] > 0.0) || !std::isfinite(edges[0]))
        return fail(ENCORE_EINVAL, "edges[0] must be > 0 (zero separations have no direction)");
    for (int b = 0; b < nbins; ++b)
        if (!(edges[b + 1] > edges[b]) || !std::isfinite(edges[b + 1]))
            return fail(ENCORE_EINVAL, "edges must be finite and strictly increasing");
    return ENCORE_OK;
}

int precision_of(uint32_t flags, int* prec)
{
    switch (flags & ENCORE_PREC_MASK) {
    case ENCORE_PREC_FP64: *prec = 0; return ENCORE_OK;
    case ENCORE_PREC_FP32: *prec = 1; return ENCORE_OK;
    case ENCORE_PREC_SPLITBF16: *prec = 2; return ENCORE_OK;
    }
    return fail(ENCORE_EINVAL, "unknown precision flag");
}

int check_grid_edges(const DevGrid& g, const double* edges, int nbins)
{
    if (edges[nbins] > g.r_max * (1.0 + 1e-12))
        return fail(ENCORE_EINVAL, "edges[nbins] exceeds the r_max the grid was built for");
    if (g.periodic && (2.0 * edges[nbins] > g.Lx || 2.0 * edges[nbins] > g.Ly || 2.0 * edges[nbins] > g.Lz))
        return fail(ENCORE_EINVAL, "periodic box: edges[nbins] must be <= box/2 on every axis");
    return ENCORE_OK;
}

int gather_precision(int prec)
{
    // The FP32 path sums each lane's FP32 terms in FP64: on survey geometry the
    // data-minus-randoms terms cancel inside each coefficient, and plain FP32
    // sums then miss 1e-6 on the multiplets (measured 9e-6 on the 6PCF of the
    // survey wedge, 6e-7 with FP64 sums).  The split-bf16 path's own products carry
    // ~1e-5, far above what plain FP32 sums add, so it keeps the faster gather.
    return prec == 0 ? 0 : (prec == 1 ? 2 : 1);
}

int plan_call(int npcf, int lmax, int nbins, const double* edges, uint32_t flags, NpcfPlan* pl)
{
    if (npcf < 3 || npcf > 6) return fail(ENCORE_EINVAL, "npcf must be 3..6");
    if (!valid_lmax(npcf, lmax)) return fail(ENCORE_EINVAL, "lmax out of range for this N");
    int rc;
    if ((rc = check_edges(edges, nbins))) return rc;
    if ((rc = precision_of(flags, &pl->prec))) return rc;
    pl->N = npcf; pl->lmax = lmax; pl->nbins = nbins;
    pl->allparity = flags & ENCORE_ALLPARITY;
    pl->nlam = (int64_t)enumerate_multiplets(npcf, lmax, pl->allparity).size() / multiplet_width(npcf);
    pl->nB = binomial(nbins, npcf - 1);
    return ENCORE_OK;
}

template <typename V>
static int upload(V*& dst, const std::vector<V>& src)
{
    const size_t bytes = std::max<size_t>(1, src.size()) * sizeof(V);
    HIPTRY(hipMalloc(&dst, bytes));
    if (!src.empty()) HIPTRY(hipMemcpy(dst, src.data(), src.size() * sizeof(V), hipMemcpyHostToDevice));
    return ENCORE_OK;
}

// Device tables of (N, lmax, parity, nbins) from the host term table; `up(dst,
// vec)` puts one host vector on the device.
template <typename Up>
static int fill_tables(DevTables& d, int N, int lmax, bool allparity, int nbins, Up&& up)
{
    const TermTable& tt = term_table(N, lmax, allparity);
    d.N = N; d.lmax = lmax; d.nbins = nbins; d.allparity = allparity;
    d.nlam = tt.nlam;
    const int K = N - 1;
    std::vector<int32_t> bt = enumerate_bin_tuples(N, nbins);
    d.nB = (int64_t)bt.size() / K;
    d.ntuple = tt.ntuple;
    d.nterm = (int64_t)tt.coef.size();
    std::vector<int32_t> toff(tt.ntuple * K), tflags(tt.ntuple);
    for (int64_t t = 0; t < tt.ntuple; ++t) {
        int f = 0, neg = 0;
        for (int k = 0; k < K; ++k) {
            const int l = tt.tuple_l[t * K + k], m = tt.tuple_m[t * K + k];
            toff[t * K + k] = l * (l + 1) / 2 + std::abs(m);
            if (m < 0) {
                f |= 1 << k;                    // conjugate
                if (std::abs(m) & 1) neg ^= 1;  // (-1)^m
            }
        }
        if (neg) f |= 1 << 8;
        if (tt.tuple_odd[t]) f |= 1 << 16;
        tflags[t] = f;
    }
    // terms sorted by multiplet (they are generated in multiplet order)
    std::vector<int32_t> tstart(tt.nlam + 1, 0);
    for (int32_t l : tt.lam) tstart[l + 1]++;
    for (int64_t l = 0; l < tt.nlam; ++l) tstart[l + 1] += tstart[l];
    const int nlm = (lmax + 1) * (lmax + 2) / 2;
    std::vector<double> kap(nlm);
    gather_tables(lmax, kap.data());
    int rc;
    if ((rc = up(d.tuple_off, toff)) || (rc = up(d.tuple_flags, tflags)) || (rc = up(d.btab, bt)) ||
        (rc = up(d.term_start, tstart)) || (rc = up(d.term_tuple, tt.term_tuple)) ||
        (rc = up(d.term_coef, tt.coef)) || (rc = up(d.kappa, kap)))
        return rc;
    return ENCORE_OK;
}

bool use_gemm_coupling(int N)
{
    // Measured on the survey wedge (200k primaries, 10 bins): 5PCF lmax 4 31 ms
    // against 80 ms for the per-wave jobs, 6PCF lmax 3 132 ms against 458 ms; the
    // 4PCF lmax 5 (800k primaries, 2 + 1 factors) 22 ms against 14.4 ms: its blocks
    // are too thin.
    return N >= 5;
}

// The split-BF16 MFMA plan of the tables' (N, lmax, parity, nbins).
template <typename Up>
static int fill_mfma(DevTables& d, const NpcfPlan& pl, Up&& up)
{
    const int nent = pl.nbins * (pl.lmax + 1) * (pl.lmax + 2) / 2;
    if (nent > kMfmaMaxAllEntries)
        return fail(ENCORE_EUNSUPPORTED, "ENCORE_PREC_SPLITBF16 needs nbins * (lmax+1)(lmax+2)/2 <= " +
                                             std::to_string(kMfmaMaxAllEntries) + " (got " +
                                             std::to_string(nent) + ")");
    int rc;
    if (use_gemm_coupling(pl.N)) {
        GemmPlan G;
        if ((rc = build_gemm_plan(pl.N, pl.lmax, pl.allparity, pl.nbins, gemm_split(pl.N), G))) return rc;
        if ((rc = up(d.mf_rows, G.rows)) || (rc = up(d.mf_cols, G.cols)) || (rc = up(d.mf_tmap, G.tmap)) ||
            (rc = up(d.mf_macros, G.macros)))
            return rc;
        d.mf_gemm = true;
        d.mf_KL = G.KL;
        d.mf_KR = G.KR;
        d.mf_nmacro = (int)(G.macros.size() / kGemmMacroWidth);
        d.mf_any_odd = G.any_odd;
        d.mf_nent = G.nent;
        d.mf_dense = G.ntiles * 256;
        d.mf_ready = true;
        return ENCORE_OK;
    }
    MfmaPlan P;
    if ((rc = build_mfma_plan(pl.N, pl.lmax, pl.allparity, pl.nbins, P))) return rc;
    if ((rc = up(d.mf_rows, P.rows)) || (rc = up(d.mf_cols, P.cols)) || (rc = up(d.mf_tmap, P.tmap))) return rc;
    for (int sh = 0; sh < kNumMfmaShapes; ++sh) {
        if ((rc = up(d.mf_jobs[sh], P.jobs[sh]))) return rc;
        d.mf_njobs[sh] = (int)(P.jobs[sh].size() / kMfmaJobWidth);
    }
    d.mf_KF = P.KF;
    d.mf_nent = P.nent;
    d.mf_dense = P.ntiles * 256;
    d.mf_ready = true;
    return ENCORE_OK;
}

int get_tables(encore_ctx* ctx, int N, int lmax, bool allparity, int nbins, DevTables** out)
{
    std::lock_guard<std::mutex> lock(ctx->tab_mu);
    auto key = std::make_tuple(N, lmax, allparity, nbins);
    auto it = ctx->tables.find(key);
    if (it != ctx->tables.end()) { *out = &it->second; return ENCORE_OK; }
    DevTables d;
    const int rc = fill_tables(d, N, lmax, allparity, nbins, [](auto*& dst, const auto& v) { return upload(dst, v); });
    if (rc) return rc;
    auto res = ctx->tables.emplace(key, d);
    *out = &res.first->second;
    return ENCORE_OK;
}

int get_tables_for(encore_ctx* ctx, const NpcfPlan& pl, DevTables** out)
{
    int rc = get_tables(ctx, pl.N, pl.lmax, pl.allparity, pl.nbins, out);
    if (rc || pl.prec != 2) return rc;
    DevTables* d = *out;
    std::lock_guard<std::mutex> lock(ctx->tab_mu);
    if (d->mf_ready) return ENCORE_OK;
    return fill_mfma(*d, pl, [](auto*& dst, const auto& v) { return upload(dst, v); });
}

int tables_in_arena(Arena& A, hipStream_t s, const NpcfPlan& pl, DevTables& d)
{
    auto carve = [&](auto*& dst, const auto& v) -> int {
        using V = typename std::remove_reference_t<decltype(v)>::value_type;
        void* p = nullptr;
        const int rc = arena_take(A, std::max<size_t>(1, v.size()) * sizeof(V), &p);
        if (rc) return rc;
        dst = static_cast<V*>(p);
        // pageable source: the copy has read it when the call returns
        if (!v.empty()) HIPTRY(hipMemcpyAsync(p, v.data(), v.size() * sizeof(V), hipMemcpyHostToDevice, s));
        return ENCORE_OK;
    };
    int rc = fill_tables(d, pl.N, pl.lmax, pl.allparity, pl.nbins, carve);
    if (rc == ENCORE_OK && pl.prec == 2) rc = fill_mfma(d, pl, carve);
    if (rc == ENCORE_OK) HIPTRY(hipStreamSynchronize(s));
    return rc;
}

int acc_len_host(const NpcfPlan& pl, int64_t* out)
{
    if (pl.prec != 2) {
        *out = (int64_t)term_table(pl.N, pl.lmax, pl.allparity).ntuple * pl.nB;
        return ENCORE_OK;
    }
    static std::mutex mu;
    static std::map<std::tuple<int, int, bool, int>, int64_t> cache;
    std::lock_guard<std::mutex> lock(mu);
    const auto key = std::make_tuple(pl.N, pl.lmax, pl.allparity, pl.nbins);
    auto it = cache.find(key);
    if (it == cache.end()) {
        if (pl.nbins * (pl.lmax + 1) * (pl.lmax + 2) / 2 > kMfmaMaxAllEntries)
            return fail(ENCORE_EUNSUPPORTED, "ENCORE_PREC_SPLITBF16 needs nbins * (lmax+1)(lmax+2)/2 <= " +
                                                 std::to_string(kMfmaMaxAllEntries));
        int64_t dense = 0;
        if (use_gemm_coupling(pl.N)) {
            GemmPlan G;
            const int rc = build_gemm_plan(pl.N, pl.lmax, pl.allparity, pl.nbins, gemm_split(pl.N), G);
            if (rc) return rc;
            dense = G.ntiles * 256;
        } else {
            MfmaPlan P;
            const int rc = build_mfma_plan(pl.N, pl.lmax, pl.allparity, pl.nbins, P);
            if (rc) return rc;
            dense = P.ntiles * 256;
        }
        it = cache.emplace(key, dense).first;
    }
    *out = it->second;
    return ENCORE_OK;
}

int64_t acc_len(const NpcfPlan& pl, const DevTables* tb)
{
    return pl.prec == 2 ? tb->mf_dense : tb->ntuple * tb->nB;
}

size_t alm_row_bytes(const NpcfPlan& pl)
{
    const int nlm = (pl.lmax + 1) * (pl.lmax + 2) / 2;
    return (size_t)pl.nbins * nlm * 2 * (pl.prec == 0 ? 8 : 4);
}

int64_t cap_rows(const NpcfPlan& pl)
{
    // 8 GiB of coefficients (about 3% of the HBM) and at most 2^27 rows (row indices
    // are 32-bit in the kernels): the benchmark-size jobs run in one slice
    int64_t cap = std::max<int64_t>(1, (int64_t)((size_t)8 << 30) / alm_row_bytes(pl));
    cap = std::min<int64_t>(cap, (int64_t)1 << 27);
    if (const char* e = getenv("ENCORE_MAX_SLICE_ROWS")) {   // smaller slices (tests of slicing)
        const long long v = atoll(e);
        if (v > 0) cap = std::min<int64_t>(cap, v);
    }
    // split-BF16 couples whole 16-row K blocks: a slice holds at least one
    if (pl.prec == 2) cap = std::max<int64_t>(cap, kBlkRows);
    return cap;
}

int64_t job_split_rows(const NpcfPlan& pl, const DevTables* tb, int64_t nprim, int64_t cap)
{
    if (pl.prec == 2) {
        // MFMA coupling: one block per (split, 16 wave jobs or one macro tile); aim
        // at ~2048 blocks
        int64_t nbj = 0;
        if (tb->mf_gemm) nbj = tb->mf_nmacro;
        else
            for (int sh = 0; sh < kNumMfmaShapes; ++sh) nbj += (tb->mf_njobs[sh] + 15) / 16;
        // The launch runs splits in whole groups of 8 one per XCD (the blocks of a
        // split share its coefficients through that XCD's L2), so the count is a
        // multiple of 8; leftover splits (the last slice of a job) spread their
        // blocks over all XCDs instead.
        const int64_t want = std::max<int64_t>(1, 2048 / std::max<int64_t>(nbj, 1));
        const int64_t ns = std::min<int64_t>(1024, (want + 7) / 8 * 8);
        int64_t rows = (std::max<int64_t>(nprim, 1) + ns - 1) / ns;
        rows = std::max<int64_t>(256, (rows + kBlkRows - 1) / kBlkRows * kBlkRows);
        rows = std::min<int64_t>(cap, rows);
        return std::max<int64_t>(kBlkRows, rows / kBlkRows * kBlkRows);   // whole K blocks
    }
    return std::min<int64_t>(
        cap, couple_split_rows(pl.N - 1, pl.nbins, tb->ntuple, tb->nB, std::max<int64_t>(nprim, 1)));
}

int prepare_slice(Exec& x, Buf& segs, Buf& splits, Buf& redp, const NpcfPlan& pl, const DevTables* tb,
                  const double* edges, const std::vector<Chunk>& chunks, SliceLaunch& L)
{
    const hipStream_t s = x.s;
    const int nlm = (pl.lmax + 1) * (pl.lmax + 2) / 2;
    const int64_t outs = acc_len(pl, tb);
    std::vector<GatherSeg> hsegs;
    std::vector<int32_t> slo, shi, rlo, rhi;
    std::vector<double*> rdst;
    std::vector<CacheAdd> adds;
    int64_t rows = 0;
    // The MFMA coupling's K blocks are whole 16-row blocks of the blocked layout;
    // each job starts on a block so that its blocks, and so its FP32 sums, are the
    // same as when it runs alone.  Rows between jobs are skipped by the gather and
    // zero in the blocked copy.
    const bool blocked = pl.prec == 2;
    for (const Chunk& c : chunks) {
        const int64_t take = c.r1 - c.r0;
        if (take <= 0) continue;
        if (blocked) rows = (rows + kBlkRows - 1) / kBlkRows * kBlkRows;
        const DevGrid& g = *c.g;
        GatherSeg gs;
        memset(&gs, 0, sizeof(gs));
        gs.P = g.P; gs.cell_start = g.cell_start; gs.prim = c.prim + c.r0;
        gs.ncx = g.ncx; gs.ncy = g.ncy; gs.ncz = g.ncz; gs.periodic = g.periodic;
        gs.ox = g.ox; gs.oy = g.oy; gs.oz = g.oz;
        gs.csx = g.csx; gs.csy = g.csy; gs.csz = g.csz;
        gs.Lx = g.Lx; gs.Ly = g.Ly; gs.Lz = g.Lz;
        gs.row0 = (int)rows; gs.nprim = (int)take;
        gs.Pq = c.Pq ? c.Pq : g.P;
        gs.nP = (int)g.n;
        finish_seg(gs);
        hsegs.push_back(gs);
        if (c.cache) adds.push_back(CacheAdd{(int)rows, (int)take, c.prim + c.r0, c.cache});
        rlo.push_back((int32_t)slo.size());
        for (int64_t r = 0; r < take; r += c.split_rows) {
            slo.push_back((int32_t)(rows + r));
            shi.push_back((int32_t)(rows + std::min<int64_t>(take, r + c.split_rows)));
        }
        rhi.push_back((int32_t)slo.size());
        rdst.push_back(c.Tdst);
        rows += take;
    }
    L = SliceLaunch();
    L.rows = rows;
    L.adds = std::move(adds);
    if (rows == 0) return ENCORE_OK;
    if (rows > INT32_MAX || hsegs.size() > 65535) return fail(ENCORE_ESIZE, "slice too large");
    const int nsplit = (int)slo.size(), nred = (int)rlo.size();
    int rc;
    if ((rc = ensure(x.alm, alm_row_bytes(pl) * (size_t)rows))) return rc;
    // the MFMA coupling reads a blocked copy: whole 16-row blocks, plus 1 KiB that
    // its 1 KiB copy units may read past the last block
    const int ent_blk = blk_entries(tb->mf_nent);
    const int64_t nblk = (rows + kBlkRows - 1) / kBlkRows;
    if (blocked && (rc = ensure(x.almb, (size_t)nblk * blk_bytes(tb->mf_nent) + 1024))) return rc;
    if ((rc = ensure(x.wprim, sizeof(double) * (size_t)rows))) return rc;
    if ((rc = ensure(x.T, sizeof(double) * (size_t)nsplit * (size_t)outs))) return rc;
    if ((rc = ensure(segs, sizeof(GatherSeg) * hsegs.size()))) return rc;
    if ((rc = ensure(splits, sizeof(int32_t) * (size_t)(2 * nsplit + 2 * nred)))) return rc;
    if ((rc = ensure(redp, sizeof(double*) * (size_t)nred))) return rc;
    if ((rc = ensure(x.queues, 64))) return rc;
    if ((rc = ensure(x.misc, 64))) return rc;
    std::vector<int32_t> hsplit;
    hsplit.insert(hsplit.end(), slo.begin(), slo.end());
    hsplit.insert(hsplit.end(), shi.begin(), shi.end());
    hsplit.insert(hsplit.end(), rlo.begin(), rlo.end());
    hsplit.insert(hsplit.end(), rhi.begin(), rhi.end());
    HIPTRY(hipMemcpyAsync(segs.p, hsegs.data(), sizeof(GatherSeg) * hsegs.size(), hipMemcpyHostToDevice, s));
    HIPTRY(hipMemcpyAsync(splits.p, hsplit.data(), sizeof(int32_t) * hsplit.size(), hipMemcpyHostToDevice, s));
    HIPTRY(hipMemcpyAsync(redp.p, rdst.data(), sizeof(double*) * rdst.size(), hipMemcpyHostToDevice, s));
    const int32_t* dsp = (const int32_t*)splits.p;
    // several catalogs: the persistent grid (work stealing across XCD queues) unless
    // ENCORE_GATHER_PERSISTENT says otherwise (0: static grid, 1: always persistent)
    L.persistent = hsegs.size() > 1;
    if (const char* e = getenv("ENCORE_GATHER_PERSISTENT")) L.persistent = atoi(e) != 0;

    GatherArgs& ga = L.ga;
    memset(&ga, 0, sizeof(ga));
    ga.nbins = pl.nbins;
    for (int b = 0; b <= pl.nbins; ++b) {
        ga.e2[b] = edges[b] * edges[b];
        ga.e1[b] = edges[b];
    }
    ga.kappa = tb->kappa;
    ga.alm = x.alm.p;
    ga.wprim = (double*)x.wprim.p;
    ga.npairs = (unsigned long long*)x.misc.p;
    ga.queues = (unsigned*)x.queues.p;
    ga.segs = (const GatherSeg*)segs.p;
    ga.nseg = (int)hsegs.size();
    ga.nrows = (int)rows;

    CoupleArgs& ca = L.ca;
    memset(&ca, 0, sizeof(ca));
    ca.alm = x.alm.p;
    ca.wprim = (const double*)x.wprim.p;
    ca.nbins = pl.nbins; ca.nlm = nlm; ca.nk = pl.N - 1;
    ca.ntuple = (int)tb->ntuple; ca.nB = (int)tb->nB;
    ca.tuple_off = tb->tuple_off; ca.tuple_flags = tb->tuple_flags; ca.btab = tb->btab;
    ca.T = (double*)x.T.p;
    ca.nsplit = nsplit;
    ca.split_lo = dsp;
    ca.split_hi = dsp + nsplit;

    MfmaArgs& ma = L.ma;
    memset(&ma, 0, sizeof(ma));
    ma.alm = (const float*)x.almb.p;
    ma.ent_blk = ent_blk;
    ma.nent = tb->mf_nent;
    ma.rows = tb->mf_rows;
    ma.cols = tb->mf_cols;
    ma.nsplit = nsplit;
    ma.split_lo = dsp;
    ma.split_hi = dsp + nsplit;
    ma.D = (double*)x.T.p;
    ma.dense = tb->mf_dense;
    ma.any_odd = pl.allparity ? 1 : 0;
    if (tb->mf_gemm) {
        ma.jobs = tb->mf_macros;
        ma.njobs = tb->mf_nmacro;
        ma.any_odd = tb->mf_any_odd ? 1 : 0;
    }

    ReduceArgs& ra = L.ra;
    ra.T = (const double*)x.T.p;
    ra.per = outs;
    ra.nred = nred;
    ra.red_lo = dsp + 2 * nsplit;
    ra.red_hi = dsp + 2 * nsplit + nred;
    ra.dst = (double* const*)redp.p;
    return ENCORE_OK;
}

int launch_slice_gather(const SliceLaunch& L, const NpcfPlan& pl, hipStream_t s)
{
    if (L.rows == 0) return ENCORE_OK;
    HIPTRY((hipError_t)launch_gather(L.ga, pl.lmax, gather_precision(pl.prec), pl.nbg, L.persistent, s));
    const int row_cplx = pl.nbins * (pl.lmax + 1) * (pl.lmax + 2) / 2;
    for (const CacheAdd& c : L.adds)
        HIPTRY((hipError_t)launch_add_cached(L.ga.alm, pl.prec == 0 ? 0 : 1, c.row0, c.nrows, c.prim, c.cache,
                                             row_cplx, s));
    return ENCORE_OK;
}

int launch_slice_couple(const SliceLaunch& L, const NpcfPlan& pl, const DevTables* tb, hipStream_t s)
{
    if (L.rows == 0) return ENCORE_OK;
    if (pl.prec == 2) {
        HIPTRY((hipError_t)launch_to_blocked((const float2*)L.ga.alm, L.ga.wprim, L.ga.segs, L.ga.nseg,
                                             (int)L.rows, L.ma.nent, (float*)L.ma.alm, s));
        if (tb->mf_gemm) {
            HIPTRY((hipError_t)launch_couple_gemm(L.ma, tb->mf_KL, tb->mf_KR, s));
        } else {
            MfmaArgs ma = L.ma;
            for (int sh = 0; sh < kNumMfmaShapes; ++sh) {
                ma.jobs = tb->mf_jobs[sh];
                ma.njobs = tb->mf_njobs[sh];
                HIPTRY((hipError_t)launch_couple_mfma(ma, tb->mf_KF, sh, s));
            }
        }
    } else {
        HIPTRY((hipError_t)launch_couple(L.ca, pl.prec, s));
    }
    HIPTRY((hipError_t)launch_reduce(L.ra, s));
    return ENCORE_OK;
}

int run_slice(Exec& x, const NpcfPlan& pl, const DevTables* tb, const double* edges,
              const std::vector<Chunk>& chunks, double* ms_gather, double* ms_couple)
{
    SliceLaunch L;
    int rc;
    if ((rc = prepare_slice(x, x.segs, x.splits, x.redp, pl, tb, edges, chunks, L))) return rc;
    if (L.rows == 0) return ENCORE_OK;
    const hipStream_t s = x.s;
    HIPTRY(hipEventRecord(x.ev[1], s));
    if ((rc = launch_slice_gather(L, pl, s))) return rc;
    HIPTRY(hipEventRecord(x.ev[2], s));
    if ((rc = launch_slice_couple(L, pl, tb, s))) return rc;
    HIPTRY(hipEventRecord(x.ev[3], s));
    HIPTRY(hipEventSynchronize(x.ev[3]));   // the host tables above are reused by the next slice
    float ms = 0.f;
    HIPTRY(hipEventElapsedTime(&ms, x.ev[1], x.ev[2]));
    if (ms_gather) *ms_gather += ms;
    HIPTRY(hipEventElapsedTime(&ms, x.ev[2], x.ev[3]));
    if (ms_couple) *ms_couple += ms;
    return ENCORE_OK;
}

int contract_job(Exec& x, const NpcfPlan& pl, const DevTables* tb, const double* T,
                 const double* bscale, double* zeta)
{
    ContractArgs xa;
    xa.nsplit = 1; xa.ntuple = (int)tb->ntuple; xa.nB = (int)tb->nB; xa.nlam = (int)pl.nlam;
    xa.term_start = tb->term_start; xa.term_tuple = tb->term_tuple; xa.term_coef = tb->term_coef;
    xa.T = T;
    xa.bscale = bscale;
    xa.tmap = pl.prec == 2 ? tb->mf_tmap : nullptr;
    xa.zeta = zeta;
    HIPTRY((hipError_t)launch_contract(xa, x.s));
    return ENCORE_OK;
}

std::vector<double> bin_scale(const NpcfPlan& pl, const double* edges, double V)
{
    const std::vector<int32_t> bt = enumerate_bin_tuples(pl.N, pl.nbins);
    const int K = pl.N - 1;
    std::vector<double> sc((size_t)pl.nB);
    for (int64_t b = 0; b < pl.nB; ++b) {
        double v = V;
        for (int k = 0; k < K; ++k) {
            const double lo = edges[bt[b * K + k]], hi = edges[bt[b * K + k] + 1];
            v *= 4.0 * M_PI / 3.0 * (hi * hi * hi - lo * lo * lo);
        }
        sc[b] = 1.0 / v;
    }
    return sc;
}

double cell_divisor(double tuned)
{
    const char* s = getenv("ENCORE_CELL_DIVISOR");
    if (s) {
        const double v = atof(s);
        if (v >= 1.0 && v <= 32.0) return v;
    }
    if (tuned >= 1.0 && tuned <= 32.0) return tuned;
    return 5.0;   // cell side r_max / 5
}

double cell_x_subdiv(double tuned)
{
    // Cells are split further along x, the axis along which a cell row is one
    // contiguous particle range: this trims the x extent of each row piece to
    // the shell's chord more tightly at no extra row set-up cost.
    const char* s = getenv("ENCORE_CELL_XSUB");
    if (s) {
        const int v = atoi(s);
        if (v >= 1 && v <= 32) return v;
    }
    if (tuned >= 1.0 && tuned <= 32.0) return tuned;
    return 16.0;
}

int ctx_nbg(encore_ctx* ctx, const NpcfPlan& pl)
{
    std::lock_guard<std::mutex> lock(ctx->tab_mu);
    auto it = ctx->tuned_nbg.find(std::make_tuple(pl.lmax, gather_precision(pl.prec), pl.nbins));
    return it == ctx->tuned_nbg.end() ? 0 : it->second;
}

void ctx_cells(encore_ctx* ctx, double* div, double* xsub)
{
    std::lock_guard<std::mutex> lock(ctx->tab_mu);
    *div = cell_divisor(ctx->cell_div);
    *xsub = cell_x_subdiv(ctx->cell_xsub);
}

int build_grid_dev(int device, const double* d_pos, const double* d_w, int64_t n, int64_t n_data,
                   bool dmr, const double* box, double r_max, double div, double xsub, hipStream_t s,
                   DevGrid& out, hipMemPool_t pool)
{
    HIPTRY(hipSetDevice(device));
    double bx[3] = {0, 0, 0};
    if (box)
        for (int a = 0; a < 3; ++a) bx[a] = box[a];
    char err[256] = {0};
    const int rc = grid_build(out, d_pos, d_w, n, n_data, dmr, box != nullptr, bx, r_max,
                              r_max / div, r_max / (div * xsub), s,
                              err, sizeof(err), pool);
    if (rc != 0) return fail(rc == -1 ? ENCORE_EINVAL : (rc == -3 ? ENCORE_ENOMEM : ENCORE_EDEVICE), err);
    return ENCORE_OK;
}

}  // namespace encore
