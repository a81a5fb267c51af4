// Edge correction (Section 3.2, eqs. edge-correction-matrix and
// edge-corrected-NPCF): host side of the device matrix build and solve.  The
// generalized Gaunt integrals come from gaunt.cpp.
//
// The device builds M_{L L''}(B) = sum_{L'} f_{L'}(B) s(L, L') E(L'') G^{L L' L''} from
// a list of the nonzero (L, L'') x L' terms grouped by (L, L'') (so each entry is a
// fixed-order sum) and solves the per-B linear system of eq. edge-correction-matrix.
// The paper's equations hold for the complex multiplets; odd multiplets are
// imaginary (Section 3.1) and enter here as their imaginary parts, so a term whose
// L and L' are both odd carries i * i = -1: s(L, L') = -1 then, +1 otherwise.  (G
// vanishes unless L, L', L'' hold an even number of odd multiplets, so the other
// factors of i cancel against the one of L''.)
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "engine.h"

using namespace encore;

namespace {

struct DevBufs {
    std::vector<void*> p;
    ~DevBufs()
    {
        for (void* q : p)
            if (q) (void)hipFree(q);
    }
    template <typename T>
    int get(T** out, size_t n)
    {
        void* q = nullptr;
        const hipError_t e = hipMalloc(&q, sizeof(T) * std::max<size_t>(n, 1));
        if (e != hipSuccess) return fail(ENCORE_ENOMEM, "hipMalloc (edge correction workspace)");
        p.push_back(q);
        *out = (T*)q;
        return ENCORE_OK;
    }
};

}  // namespace

extern "C" int encore_edge_correct(encore_ctx* ctx, int npcf, int lmax, int nbins, uint32_t flags,
                                   const double* nmult, const double* rmult, size_t mult_len, int lmax_out,
                                   double* zeta, size_t zeta_len, double* coupling, size_t coupling_len,
                                   int64_t* n_singular)
{
    if (!ctx) return fail(ENCORE_EINVAL, "ctx is NULL");
    if (npcf < 3 || npcf > 6) return fail(ENCORE_EINVAL, "npcf must be 3..6");
    if (lmax < 0 || lmax > kMaxLmax) return fail(ENCORE_EINVAL, "lmax must be 0..10");
    if (lmax_out < 0 || lmax_out > lmax) return fail(ENCORE_EINVAL, "lmax_out must be 0..lmax");
    if (nbins < 1 || nbins > kMaxBins) return fail(ENCORE_EINVAL, "nbins must be 1..16");
    if (!nmult || !rmult || !zeta) return fail(ENCORE_EINVAL, "NULL multiplets or zeta");
    const bool allp = flags & ENCORE_ALLPARITY;
    const int64_t nlam = (int64_t)enumerate_multiplets(npcf, lmax, allp).size() / multiplet_width(npcf);
    if (nlam > kEdgeMaxMultiplets)
        return fail(ENCORE_EUNSUPPORTED, "edge correction solves systems of at most " +
                                             std::to_string(kEdgeMaxMultiplets) + " multiplets (got " +
                                             std::to_string(nlam) + ")");
    const GauntTable& gt = gaunt_table(npcf, lmax, allp);
    const int n = gt.nlam;
    const int64_t nB = binomial(nbins, npcf - 1);
    const int W = multiplet_width(npcf);
    std::vector<int32_t> keep;
    for (int i = 0; i < n; ++i) {
        int ls[5];
        principal_of(npcf, &gt.lam[(size_t)i * W], ls);
        if (*std::max_element(ls, ls + npcf - 1) <= lmax_out) keep.push_back(i);
    }
    const int nout = (int)keep.size();
    if (mult_len < (size_t)n * nB)
        return fail(ENCORE_ESIZE, "mult_len too small: need " + std::to_string((size_t)n * nB));
    if (zeta_len < (size_t)nout * nB)
        return fail(ENCORE_ESIZE, "zeta_len too small: need " + std::to_string((size_t)nout * nB));
    if (coupling && coupling_len < (size_t)nB * n * n)
        return fail(ENCORE_ESIZE, "coupling_len too small: need " + std::to_string((size_t)nB * n * n));
    if (n_singular) *n_singular = 0;
    if (nB == 0) return ENCORE_OK;
    std::lock_guard<std::mutex> lock(ctx->mu);
    HIPTRY(hipSetDevice(ctx->device));
    const hipStream_t s = ctx->main.s;
    DevBufs d;
    EdgeArgs a{};
    a.nlam = n;
    a.nB = (int)nB;
    a.nout = nout;
    double *dn, *dr, *dv, *dA, *dx, *dz, *dM = nullptr;
    int64_t* drs;
    int32_t *dlp, *dk;
    unsigned* dbad;
    int rc;
    const size_t nt = gt.term_lp.size();
    if ((rc = d.get(&dn, (size_t)n * nB)) || (rc = d.get(&dr, (size_t)n * nB)) ||
        (rc = d.get(&drs, gt.row_start.size())) || (rc = d.get(&dlp, nt)) || (rc = d.get(&dv, nt)) ||
        (rc = d.get(&dA, (size_t)nB * n * n)) || (rc = d.get(&dx, (size_t)nB * n)) ||
        (rc = d.get(&dk, (size_t)nout)) || (rc = d.get(&dz, (size_t)nout * nB)) || (rc = d.get(&dbad, 1)))
        return rc;
    if (coupling && (rc = d.get(&dM, (size_t)nB * n * n))) return rc;
    HIPTRY(hipMemcpyAsync(dn, nmult, sizeof(double) * n * nB, hipMemcpyHostToDevice, s));
    HIPTRY(hipMemcpyAsync(dr, rmult, sizeof(double) * n * nB, hipMemcpyHostToDevice, s));
    HIPTRY(hipMemcpyAsync(drs, gt.row_start.data(), sizeof(int64_t) * gt.row_start.size(), hipMemcpyHostToDevice, s));
    if (nt) {
        HIPTRY(hipMemcpyAsync(dlp, gt.term_lp.data(), sizeof(int32_t) * nt, hipMemcpyHostToDevice, s));
        HIPTRY(hipMemcpyAsync(dv, gt.term_val.data(), sizeof(double) * nt, hipMemcpyHostToDevice, s));
    }
    if (nout) HIPTRY(hipMemcpyAsync(dk, keep.data(), sizeof(int32_t) * nout, hipMemcpyHostToDevice, s));
    HIPTRY((hipError_t)launch_fill_u32(dbad, 1, 0u, s));
    a.nmult = dn;
    a.rmult = dr;
    a.row_start = drs;
    a.term_lp = dlp;
    a.term_val = dv;
    a.A = dA;
    a.rhs = dx;
    a.keep = dk;
    a.zeta = dz;
    a.M_out = dM;
    a.nbad = dbad;
    HIPTRY(hipEventRecord(ctx->main.ev[0], s));
    HIPTRY((hipError_t)launch_edge(a, s));
    HIPTRY(hipEventRecord(ctx->main.ev[1], s));
    unsigned nbad = 0;
    HIPTRY(hipMemcpyAsync(zeta, dz, sizeof(double) * nout * nB, hipMemcpyDeviceToHost, s));
    if (coupling) HIPTRY(hipMemcpyAsync(coupling, dM, sizeof(double) * nB * n * n, hipMemcpyDeviceToHost, s));
    HIPTRY(hipMemcpyAsync(&nbad, dbad, sizeof(unsigned), hipMemcpyDeviceToHost, s));
    HIPTRY(hipStreamSynchronize(s));
    float ms = 0.f;
    for (double& t : ctx->timings) t = 0.0;
    if (hipEventElapsedTime(&ms, ctx->main.ev[0], ctx->main.ev[1]) == hipSuccess) ctx->timings[0] = ms;
    if (n_singular) *n_singular = nbad;
    return ENCORE_OK;
}
