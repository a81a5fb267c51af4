// C ABI of libencore (declared in include/encore.h).
//
// One encore_npcf call runs, on one HIP stream:
//   primary list -> [gather a~ for a batch of primaries -> couple into T] x batches
//   -> contract T with the coupling terms -> zeta (FP64) -> host.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/encore.h"
#include "device.h"
#include "internal.h"

namespace encore {

static thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }
const char* get_error() { return g_err.c_str(); }

}  // namespace encore

using namespace encore;

namespace {

// device copies of the tables for one (N, lmax, parity, nbins)
struct DevTables {
    int N = 0, lmax = 0, nbins = 0;
    bool allparity = false;
    int64_t nlam = 0, nB = 0, ntuple = 0, nterm = 0;
    int32_t* tuple_off = nullptr;
    int32_t* tuple_flags = nullptr;
    int32_t* btab = nullptr;
    int32_t* term_start = nullptr;
    int32_t* term_tuple = nullptr;
    double* term_coef = nullptr;
    double* kappa = nullptr;
    double* gamma = nullptr;
};

struct Buf {
    void* p = nullptr;
    size_t n = 0;
};

}  // namespace

struct encore_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::map<std::tuple<int, int, bool, int>, DevTables> tables;
    Buf alm, T, zeta, prim, bscale, misc;
    double timings[6] = {0, 0, 0, 0, 0, 0};
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    int live_grids = 0;
    std::mutex mu;
};

struct encore_grid {
    encore_ctx* ctx = nullptr;
    DevGrid g;
};

namespace {

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

#define HIPTRY(x)                                          \
    do {                                                   \
        hipError_t e__ = (x);                              \
        if (e__ != hipSuccess) return hip_fail(e__, #x);   \
    } while (0)

int ensure(Buf& b, size_t bytes)
{
    if (b.n >= bytes && b.p) return ENCORE_OK;
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.n = 0;
    const size_t want = std::max<size_t>(bytes, 256);
    hipError_t e = hipMalloc(&b.p, want);
    if (e != hipSuccess) return hip_fail(e, "hipMalloc(workspace)");
    b.n = want;
    return ENCORE_OK;
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

template <typename V>
int upload(V*& dst, const std::vector<V>& src)
{
    const size_t bytes = std::max<size_t>(1, src.size()) * sizeof(V);
    HIPTRY(hipMalloc(&dst, bytes));
    if (!src.empty()) HIPTRY(hipMemcpy(dst, src.data(), src.size() * sizeof(V), hipMemcpyHostToDevice));
    return ENCORE_OK;
}

int get_tables(encore_ctx* ctx, int N, int lmax, bool allparity, int nbins, DevTables** out)
{
    auto key = std::make_tuple(N, lmax, allparity, nbins);
    auto it = ctx->tables.find(key);
    if (it != ctx->tables.end()) { *out = &it->second; return ENCORE_OK; }
    const TermTable& tt = term_table(N, lmax, allparity);
    DevTables d;
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
                f |= 1 << k;                 // conjugate
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
    std::vector<double> kap(nlm), gam(nlm);
    gather_tables(lmax, kap.data(), gam.data());
    int rc;
    if ((rc = upload(d.tuple_off, toff)) || (rc = upload(d.tuple_flags, tflags)) ||
        (rc = upload(d.btab, bt)) || (rc = upload(d.term_start, tstart)) ||
        (rc = upload(d.term_tuple, tt.term_tuple)) || (rc = upload(d.term_coef, tt.coef)) ||
        (rc = upload(d.kappa, kap)) || (rc = upload(d.gamma, gam)))
        return rc;
    auto res = ctx->tables.emplace(key, d);
    *out = &res.first->second;
    return ENCORE_OK;
}

void free_tables(DevTables& d)
{
    for (void* p : {(void*)d.tuple_off, (void*)d.tuple_flags, (void*)d.btab, (void*)d.term_start,
                    (void*)d.term_tuple, (void*)d.term_coef, (void*)d.kappa, (void*)d.gamma})
        if (p) (void)hipFree(p);
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
    case ENCORE_PREC_SPLITBF16:
        return fail(ENCORE_EUNSUPPORTED, "ENCORE_PREC_SPLITBF16 coupling is not built in this version");
    }
    return fail(ENCORE_EINVAL, "unknown precision flag");
}

int check_grid_edges(const encore_grid* grid, const double* edges, int nbins)
{
    const DevGrid& g = grid->g;
    if (edges[nbins] > g.r_max * (1.0 + 1e-12))
        return fail(ENCORE_EINVAL, "edges[nbins] exceeds the r_max the grid was built for");
    if (g.periodic && (2.0 * edges[nbins] > g.Lx || 2.0 * edges[nbins] > g.Ly || 2.0 * edges[nbins] > g.Lz))
        return fail(ENCORE_EINVAL, "periodic box: edges[nbins] must be <= box/2 on every axis");
    return ENCORE_OK;
}

// Primary list (sorted indices) into ctx->prim; returns count in *np.
int make_primaries(encore_ctx* ctx, const encore_grid* grid, const int64_t* subset, int64_t k,
                   int64_t* np, hipStream_t s)
{
    const int64_t n = grid->g.n;
    if (!subset) {
        int rc = ensure(ctx->prim, sizeof(int32_t) * std::max<int64_t>(n, 1));
        if (rc) return rc;
        HIPTRY((hipError_t)launch_iota((int32_t*)ctx->prim.p, n, s));
        *np = n;
        return ENCORE_OK;
    }
    if (k < 0) return fail(ENCORE_EINVAL, "n_subset < 0");
    int rc = ensure(ctx->prim, sizeof(int32_t) * std::max<int64_t>(k, 1));
    if (rc) return rc;
    if ((rc = ensure(ctx->misc, sizeof(int64_t) * std::max<int64_t>(k, 1) + 16))) return rc;
    int* d_bad = (int*)ctx->misc.p;
    int64_t* d_idx = (int64_t*)((char*)ctx->misc.p + 16);
    int bad = 0;
    HIPTRY(hipMemcpyAsync(d_bad, &bad, sizeof(int), hipMemcpyHostToDevice, s));
    if (k > 0) {
        HIPTRY(hipMemcpyAsync(d_idx, subset, sizeof(int64_t) * k, hipMemcpyHostToDevice, s));
        HIPTRY((hipError_t)launch_map_subset(d_idx, k, grid->g.inv, n, (int32_t*)ctx->prim.p, d_bad, s));
    }
    HIPTRY(hipMemcpyAsync(&bad, d_bad, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPTRY(hipStreamSynchronize(s));
    if (bad) return fail(ENCORE_EINVAL, "primary_subset holds an index outside [0, n)");
    *np = k;
    return ENCORE_OK;
}

void fill_gather_args(GatherArgs& a, const DevGrid& g, const double* edges, int nbins)
{
    memset(&a, 0, sizeof(a));
    a.P = g.P;
    a.cell_start = g.cell_start;
    a.ncx = g.ncx; a.ncy = g.ncy; a.ncz = g.ncz;
    a.ox = g.ox; a.oy = g.oy; a.oz = g.oz;
    a.csx = g.csx; a.csy = g.csy; a.csz = g.csz;
    a.periodic = g.periodic;
    a.Lx = g.Lx; a.Ly = g.Ly; a.Lz = g.Lz;
    a.nbins = nbins;
    for (int b = 0; b <= nbins; ++b) a.e2[b] = edges[b] * edges[b];
}

double cell_divisor()
{
    const char* s = getenv("ENCORE_CELL_DIVISOR");
    if (s) {
        const double v = atof(s);
        if (v >= 1.0 && v <= 32.0) return v;
    }
    return 6.0;   // cell side r_max / 6: measured best of {4, 6, 8, 10}
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
    double bx[3] = {0, 0, 0};
    if (periodic) {
        if (!box) return fail(ENCORE_EINVAL, "ENCORE_PERIODIC needs box");
        for (int a = 0; a < 3; ++a) {
            if (!(box[a] > 0.0) || !std::isfinite(box[a])) return fail(ENCORE_EINVAL, "box must be > 0");
            bx[a] = box[a];
        }
    }
    HIPTRY(hipSetDevice(ctx->device));
    hipStream_t s = stream ? (hipStream_t)stream : ctx->stream;
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
    char err[256] = {0};
    const int rc = grid_build(gr->g, d_pos, d_w, n, n_data, (flags & ENCORE_DMR) != 0, periodic, bx, r_max,
                              r_max / cell_divisor(), s, err, sizeof(err));
    if (tmp_pos) (void)hipFree(tmp_pos);
    if (tmp_w) (void)hipFree(tmp_w);
    if (rc != 0) {
        delete gr;
        return fail(rc == -1 ? ENCORE_EINVAL : (rc == -3 ? ENCORE_ENOMEM : ENCORE_EDEVICE), err);
    }
    {
        std::lock_guard<std::mutex> lock(ctx->mu);
        ctx->live_grids++;
    }
    *out = gr;
    return ENCORE_OK;
}

}  // namespace

extern "C" {

const char* encore_last_error(void) { return get_error(); }

const char* encore_version(void) { return "encore-mi355x 0.1 (gfx950)"; }

int encore_create(int hip_device, encore_ctx** out)
{
    if (!out) return fail(ENCORE_EINVAL, "out is NULL");
    int ndev = 0;
    HIPTRY(hipGetDeviceCount(&ndev));
    if (hip_device < 0 || hip_device >= ndev)
        return fail(ENCORE_EINVAL, "hip_device out of range (" + std::to_string(ndev) + " devices)");
    HIPTRY(hipSetDevice(hip_device));
    auto* c = new encore_ctx();
    c->device = hip_device;
    hipError_t e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
    for (int i = 0; i < 4 && e == hipSuccess; ++i) e = hipEventCreate(&c->ev[i]);
    if (e != hipSuccess) {
        delete c;
        return hip_fail(e, "encore_create");
    }
    *out = c;
    return ENCORE_OK;
}

int encore_destroy(encore_ctx* ctx)
{
    if (!ctx) return ENCORE_OK;
    if (ctx->live_grids > 0) return fail(ENCORE_EINVAL, "free every grid before destroying the context");
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    for (auto& kv : ctx->tables) free_tables(kv.second);
    for (Buf* b : {&ctx->alm, &ctx->T, &ctx->zeta, &ctx->prim, &ctx->bscale, &ctx->misc})
        if (b->p) (void)hipFree(b->p);
    for (int i = 0; i < 4; ++i)
        if (ctx->ev[i]) (void)hipEventDestroy(ctx->ev[i]);
    (void)hipStreamDestroy(ctx->stream);
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
    (void)hipSetDevice(grid->ctx->device);
    (void)hipDeviceSynchronize();
    grid_free(grid->g);
    {
        std::lock_guard<std::mutex> lock(grid->ctx->mu);
        grid->ctx->live_grids--;
    }
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
    if (grid->ctx != ctx) return fail(ENCORE_EINVAL, "grid belongs to another context");
    if (npcf < 3 || npcf > 6) return fail(ENCORE_EINVAL, "npcf must be 3..6");
    if (!valid_lmax(npcf, lmax)) return fail(ENCORE_EINVAL, "lmax out of range for this N");
    int rc;
    if ((rc = check_edges(edges, nbins))) return rc;
    if ((rc = check_grid_edges(grid, edges, nbins))) return rc;
    int prec = 0;
    if ((rc = precision_of(flags, &prec))) return rc;
    const bool allparity = flags & ENCORE_ALLPARITY;
    const int64_t nlam = (int64_t)enumerate_multiplets(npcf, lmax, allparity).size() / multiplet_width(npcf);
    const int64_t nB = binomial(nbins, npcf - 1);
    const size_t need = (size_t)(nlam * nB);
    if (!zeta && need > 0) return fail(ENCORE_EINVAL, "zeta is NULL");
    if (zeta_len < need) return fail(ENCORE_ESIZE, "zeta needs " + std::to_string(need) + " elements");
    double V = 0.0;
    if (flags & ENCORE_NORMALIZE) {
        V = volume;
        if (!(V > 0.0)) {
            if (!grid->g.periodic) return fail(ENCORE_EINVAL, "ENCORE_NORMALIZE needs volume > 0 without a periodic box");
            V = grid->g.Lx * grid->g.Ly * grid->g.Lz;
        }
    }
    std::lock_guard<std::mutex> lock(ctx->mu);
    for (double& t : ctx->timings) t = 0.0;
    if (need == 0) return ENCORE_OK;
    HIPTRY(hipSetDevice(ctx->device));
    hipStream_t s = stream ? (hipStream_t)stream : ctx->stream;
    HIPTRY(hipEventRecord(ctx->ev[0], s));

    DevTables* tb = nullptr;
    if ((rc = get_tables(ctx, npcf, lmax, allparity, nbins, &tb))) return rc;
    int64_t nprim = 0;
    if ((rc = make_primaries(ctx, grid, primary_subset, n_subset, &nprim, s))) return rc;

    const int nlm = (lmax + 1) * (lmax + 2) / 2;
    const size_t per_prim = (size_t)nbins * nlm * 2 * (prec == 0 ? 8 : 4);
    const int64_t batch = std::max<int64_t>(1, std::min<int64_t>(nprim, (int64_t)((size_t)2 << 30) / per_prim));
    // splits of the primary range in the coupling kernel (parallelism of the sum over i)
    const int64_t outs = tb->ntuple * tb->nB;
    const int64_t nsplit = couple_nsplit(npcf - 1, nbins, tb->ntuple, tb->nB, batch);

    if ((rc = ensure(ctx->alm, per_prim * (size_t)batch))) return rc;
    if ((rc = ensure(ctx->T, sizeof(double) * (size_t)(nsplit * outs)))) return rc;
    if ((rc = ensure(ctx->zeta, sizeof(double) * need))) return rc;
    HIPTRY((hipError_t)launch_fill((double*)ctx->T.p, nsplit * outs, 0.0, s));
    const double* d_bscale = nullptr;
    if (flags & ENCORE_NORMALIZE) {
        std::vector<int32_t> bt = enumerate_bin_tuples(npcf, nbins);
        std::vector<double> sc(nB);
        const int K = npcf - 1;
        for (int64_t b = 0; b < nB; ++b) {
            double v = V;
            for (int k = 0; k < K; ++k) {
                const double lo = edges[bt[b * K + k]], hi = edges[bt[b * K + k] + 1];
                v *= 4.0 * M_PI / 3.0 * (hi * hi * hi - lo * lo * lo);
            }
            sc[b] = 1.0 / v;
        }
        if ((rc = ensure(ctx->bscale, sizeof(double) * nB))) return rc;
        HIPTRY(hipMemcpyAsync(ctx->bscale.p, sc.data(), sizeof(double) * nB, hipMemcpyHostToDevice, s));
        HIPTRY(hipStreamSynchronize(s));
        d_bscale = (const double*)ctx->bscale.p;
    }

    GatherArgs ga;
    fill_gather_args(ga, grid->g, edges, nbins);
    ga.kappa = tb->kappa;
    ga.gamma = tb->gamma;
    ga.alm = ctx->alm.p;
    if ((rc = ensure(ctx->misc, 64))) return rc;
    unsigned long long* d_pairs = (unsigned long long*)ctx->misc.p;
    HIPTRY(hipMemsetAsync(d_pairs, 0, sizeof(unsigned long long), s));
    ga.npairs = d_pairs;
    CoupleArgs ca;
    memset(&ca, 0, sizeof(ca));
    ca.alm = ctx->alm.p;
    ca.P = grid->g.P;
    ca.nbins = nbins; ca.nlm = nlm; ca.nk = npcf - 1;
    ca.ntuple = (int)tb->ntuple; ca.nB = (int)tb->nB;
    ca.tuple_off = tb->tuple_off; ca.tuple_flags = tb->tuple_flags; ca.btab = tb->btab;
    ca.nsplit = (int)nsplit;
    ca.T = (double*)ctx->T.p;

    double t_gather = 0.0, t_couple = 0.0;
    int nlaunch = 0;
    for (int64_t p0 = 0; p0 < nprim; p0 += batch) {
        const int np = (int)std::min<int64_t>(batch, nprim - p0);
        ga.prim = (const int32_t*)ctx->prim.p + p0;
        ga.nprim = np;
        HIPTRY(hipEventRecord(ctx->ev[1], s));
        HIPTRY((hipError_t)launch_gather(ga, lmax, prec, s));
        HIPTRY(hipEventRecord(ctx->ev[2], s));
        ca.prim = ga.prim;
        ca.nprim = np;
        HIPTRY((hipError_t)launch_couple(ca, prec, s));
        HIPTRY(hipEventRecord(ctx->ev[3], s));
        HIPTRY(hipEventSynchronize(ctx->ev[3]));
        float ms = 0.f;
        HIPTRY(hipEventElapsedTime(&ms, ctx->ev[1], ctx->ev[2]));
        t_gather += ms;
        HIPTRY(hipEventElapsedTime(&ms, ctx->ev[2], ctx->ev[3]));
        t_couple += ms;
        ++nlaunch;
    }
    ContractArgs xa;
    xa.T = (const double*)ctx->T.p;
    xa.nsplit = (int)nsplit; xa.ntuple = (int)tb->ntuple; xa.nB = (int)tb->nB; xa.nlam = (int)nlam;
    xa.term_start = tb->term_start; xa.term_tuple = tb->term_tuple; xa.term_coef = tb->term_coef;
    xa.bscale = d_bscale;
    xa.zeta = (double*)ctx->zeta.p;
    HIPTRY(hipEventRecord(ctx->ev[1], s));
    HIPTRY((hipError_t)launch_contract(xa, s));
    HIPTRY(hipEventRecord(ctx->ev[2], s));
    std::vector<double> host(need);
    HIPTRY(hipMemcpyAsync(host.data(), ctx->zeta.p, sizeof(double) * need, hipMemcpyDeviceToHost, s));
    HIPTRY(hipEventRecord(ctx->ev[3], s));
    HIPTRY(hipEventSynchronize(ctx->ev[3]));
    float ms_c = 0.f, ms_tot = 0.f;
    HIPTRY(hipEventElapsedTime(&ms_c, ctx->ev[1], ctx->ev[2]));
    HIPTRY(hipEventElapsedTime(&ms_tot, ctx->ev[0], ctx->ev[3]));
    unsigned long long pairs = 0;
    HIPTRY(hipMemcpy(&pairs, d_pairs, sizeof(pairs), hipMemcpyDeviceToHost));
    std::copy(host.begin(), host.end(), zeta);
    ctx->timings[5] = (double)pairs;
    ctx->timings[0] = ms_tot;
    ctx->timings[1] = t_gather;
    ctx->timings[2] = t_couple;
    ctx->timings[3] = ms_c;
    ctx->timings[4] = nlaunch;
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
    if ((rc = check_grid_edges(grid, edges, nbins))) return rc;
    int prec = 0;
    if ((flags & ENCORE_PREC_MASK) == ENCORE_PREC_SPLITBF16) prec = 1;   // same FP32 gather
    else if ((rc = precision_of(flags, &prec))) return rc;
    if (!primaries || k < 1 || !alm_out) return fail(ENCORE_EINVAL, "need k >= 1 primaries and alm_out");
    const bool full = flags & ENCORE_DEBUG_FULLGRID;
    std::lock_guard<std::mutex> lock(ctx->mu);
    HIPTRY(hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    const int nlm = (lmax + 1) * (lmax + 2) / 2;
    const int64_t per = (int64_t)nbins * nlm * 2;     // reals per primary
    const int64_t nval = k * per;
    // requested rows -> sorted indices (ctx->prim), validated
    int64_t np = 0;
    if ((rc = make_primaries(ctx, grid, primaries, k, &np, s))) return rc;
    std::vector<int32_t> sorted_rows(k);
    HIPTRY(hipMemcpy(sorted_rows.data(), ctx->prim.p, sizeof(int32_t) * k, hipMemcpyDeviceToHost));
    const int64_t nlaunch = full ? grid->g.n : k;
    if (full) {
        if ((rc = make_primaries(ctx, grid, nullptr, 0, &np, s))) return rc;
    }
    if ((rc = ensure(ctx->alm, (size_t)(nlaunch * per) * (prec == 0 ? 8 : 4)))) return rc;
    if ((rc = ensure(ctx->zeta, sizeof(double) * (size_t)(nlaunch * per)))) return rc;
    std::vector<double> kap(nlm), gam(nlm);
    gather_tables(lmax, kap.data(), gam.data());
    double* d_kg = nullptr;
    HIPTRY(hipMalloc(&d_kg, sizeof(double) * 2 * nlm));
    hipError_t e = hipMemcpy(d_kg, kap.data(), sizeof(double) * nlm, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d_kg + nlm, gam.data(), sizeof(double) * nlm, hipMemcpyHostToDevice);
    GatherArgs ga;
    fill_gather_args(ga, grid->g, edges, nbins);
    ga.kappa = d_kg;
    ga.gamma = d_kg + nlm;
    ga.alm = ctx->alm.p;
    ga.prim = (const int32_t*)ctx->prim.p;
    ga.nprim = (int)nlaunch;
    if (e == hipSuccess) e = (hipError_t)launch_gather(ga, lmax, prec, s);
    if (e == hipSuccess)
        e = (hipError_t)launch_to_double(ctx->alm.p, prec, nlaunch * per, (double*)ctx->zeta.p, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    for (int64_t r = 0; r < k && e == hipSuccess; ++r) {
        // full launch: row of sorted index sorted_rows[r]; else row r
        const int64_t row = full ? sorted_rows[r] : r;
        e = hipMemcpy(alm_out + r * per, (double*)ctx->zeta.p + row * per, sizeof(double) * per,
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
