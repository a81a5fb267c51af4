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

// byte offset of the next 256-byte-aligned part of a packed workspace
size_t carve(size_t& off, size_t bytes)
{
    const size_t at = off;
    off += (std::max<size_t>(bytes, 1) + 255) / 256 * 256;
    return at;
}

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
    Exec& x = ctx->main;
    EdgeArgs a{};
    a.nlam = n;
    a.nB = (int)nB;
    a.nout = nout;
    int rc;
    // Workspaces: the context's grow-only buffers, kept for later calls; the Gaunt
    // table is uploaded once per (npcf, lmax, parity) while its buffer stays put.
    const size_t nt = gt.term_lp.size(), nrs = gt.row_start.size();
    size_t go = 0;
    const size_t o_rs = carve(go, sizeof(int64_t) * nrs), o_lp = carve(go, sizeof(int32_t) * nt),
                 o_v = carve(go, sizeof(double) * nt);
    const size_t gt_n0 = x.egt.n;
    if ((rc = ensure(x.egt, go))) return rc;
    const auto gt_key = std::make_tuple(npcf, lmax, allp);
    const bool gt_fresh = ctx->edge_gt_key != gt_key || x.egt.n != gt_n0;
    size_t io = 0;
    const size_t o_n = carve(io, sizeof(double) * n * nB), o_r = carve(io, sizeof(double) * n * nB),
                 o_x = carve(io, sizeof(double) * nB * n), o_k = carve(io, sizeof(int32_t) * nout),
                 o_z = carve(io, sizeof(double) * nout * nB), o_bad = carve(io, sizeof(unsigned));
    if ((rc = ensure(x.eio, io)) || (rc = ensure(x.eA, sizeof(double) * nB * n * n))) return rc;
    if (coupling && (rc = ensure(x.eM, sizeof(double) * nB * n * n))) return rc;
    char* gb = (char*)x.egt.p;
    char* ib = (char*)x.eio.p;
    int64_t* drs = (int64_t*)(gb + o_rs);
    int32_t* dlp = (int32_t*)(gb + o_lp);
    double* dv = (double*)(gb + o_v);
    double* dn = (double*)(ib + o_n);
    double* dr = (double*)(ib + o_r);
    double* dx = (double*)(ib + o_x);
    int32_t* dk = (int32_t*)(ib + o_k);
    double* dz = (double*)(ib + o_z);
    unsigned* dbad = (unsigned*)(ib + o_bad);
    double* dA = (double*)x.eA.p;
    double* dM = coupling ? (double*)x.eM.p : nullptr;
    HIPTRY(hipMemcpyAsync(dn, nmult, sizeof(double) * n * nB, hipMemcpyHostToDevice, s));
    HIPTRY(hipMemcpyAsync(dr, rmult, sizeof(double) * n * nB, hipMemcpyHostToDevice, s));
    if (gt_fresh) {
        ctx->edge_gt_key = std::make_tuple(-1, -1, false);
        HIPTRY(hipMemcpyAsync(drs, gt.row_start.data(), sizeof(int64_t) * nrs, hipMemcpyHostToDevice, s));
        if (nt) {
            HIPTRY(hipMemcpyAsync(dlp, gt.term_lp.data(), sizeof(int32_t) * nt, hipMemcpyHostToDevice, s));
            HIPTRY(hipMemcpyAsync(dv, gt.term_val.data(), sizeof(double) * nt, hipMemcpyHostToDevice, s));
        }
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
    ctx->edge_gt_key = gt_key;   // the upload (if any) has completed
    float ms = 0.f;
    for (double& t : ctx->timings) t = 0.0;
    if (hipEventElapsedTime(&ms, ctx->main.ev[0], ctx->main.ev[1]) == hipSuccess) ctx->timings[0] = ms;
    if (n_singular) *n_singular = nbad;
    return ENCORE_OK;
}
