// Gridded-data estimator (Section 3.2, Gridded Data): the multiplets of a density
// field delta given on a periodic mesh of n^3 cells.
//
//  1. Kernel fields K^b_lm(u) = Y_lm(u^) Theta^b(|u|) on the mesh offsets u
//     (minimum image, FP64, bins decided exactly as the discrete path does:
//     edges[b]^2 <= r^2 < edges[b+1]^2 with r^2 = (ux*ux + uy*uy) + uz*uz, no FMA).
//  2. The harmonic coefficients of every cell as one correlation per (b, lm),
//     a~^b_lm(s) = sum_u delta(s + u) K^b_lm(u) (eq. alm-binned-def, raw), done with
//     FFTs (eq. alm-binned-def-fft): F[a~](k) = F[delta](k) F[K](-k), and F[K](-k) =
//     (-1)^l F[K](k) because K(-u) = (-1)^l K(u).  Batched FP64 complex transforms
//     (hipFFT) over all nbins * nlm fields at once.
//  3. Every cell is a primary of weight delta(s) (cells with delta = 0 add exactly
//     zero), and the coupling of the discrete path sums the products of N - 1
//     coefficients over cells (eq. NPCF-mult-binned-estimator, sum over cells for
//     the integral over s).
//
// Layout: delta[(ix * n + iy) * n + iz]; the fields are contiguous, F[b][lm][cell]
// (complex FP64), one batched transform over all of them; each slice of cells is
// transposed through LDS into the coupling's rows [cell][b][lm].
#include <hip/hip_runtime.h>
#include <hipfft/hipfft.h>
#include <type_traits>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "engine.h"

namespace encore {

namespace {

constexpr int kMeshBlock = 256;
constexpr int kMaxNlm = (kMaxLmax + 1) * (kMaxLmax + 2) / 2;

struct MeshKernelArgs {
    int n, nbins, nlm, lmax;
    double h;
    double e2[kMaxBins + 1];
    double kappa[kMaxNlm];
    double gamma[kMaxNlm];
    int lm_l[kMaxNlm], lm_m[kMaxNlm];
};

__device__ __forceinline__ double mesh_dist2(double dx, double dy, double dz)
{
#pragma clang fp contract(off)
    return (dx * dx + dy * dy) + dz * dz;
}

__device__ __forceinline__ int min_image(int i, int n) { return 2 * i < n ? i : i - n; }

// One thread per (field f = b * nlm + lm, cell offset): K^b_lm at that offset.
__global__ void __launch_bounds__(kMeshBlock) k_mesh_kernels(MeshKernelArgs a, double2* __restrict__ F, int64_t total,
                                                   int64_t ncell)
{
    const int64_t e = (int64_t)blockIdx.x * kMeshBlock + threadIdx.x;
    if (e >= total) return;
    const int f = (int)(e / ncell);
    const int64_t c = e - (int64_t)f * ncell;
    const int b = f / a.nlm, lm = f - b * a.nlm;
    const int n = a.n;
    const int iz = (int)(c % n), iy = (int)((c / n) % n), ix = (int)(c / ((int64_t)n * n));
    const double ux = min_image(ix, n) * a.h, uy = min_image(iy, n) * a.h, uz = min_image(iz, n) * a.h;
    const double r2 = mesh_dist2(ux, uy, uz);
    double2 out = make_double2(0.0, 0.0);
    if (r2 >= a.e2[b] && r2 < a.e2[b + 1]) {   // edges[0] > 0: r2 > 0 here
        const double inv = 1.0 / sqrt(r2);
        const double x = ux * inv, y = uy * inv, z = uz * inv;
        const int l = a.lm_l[lm], m = a.lm_m[lm];
        // (x + i y)^m
        double pr = 1.0, pi = 0.0;
        for (int k = 0; k < m; ++k) {
            const double nr = pr * x - pi * y, ni = pr * y + pi * x;
            pr = nr; pi = ni;
        }
        // monic Legendre recurrence in z: R_mm = 1, R_{m+1,m} = z, R_lm = z R_{l-1,m} - gamma_lm R_{l-2,m}
        double r0 = 1.0, r1 = z;
        double rl = (l == m) ? r0 : r1;
        for (int q = m + 2; q <= l; ++q) {
            const double rn = z * r1 - a.gamma[q * (q + 1) / 2 + m] * r0;
            r0 = r1; r1 = rn; rl = rn;
        }
        const double s = a.kappa[lm] * rl;
        out = make_double2(s * pr, s * pi);
    }
    F[e] = out;
}

// delta (real) -> complex
__global__ void __launch_bounds__(kMeshBlock) k_mesh_complex(const double* __restrict__ d, double2* __restrict__ D, int64_t ncell)
{
    const int64_t c = (int64_t)blockIdx.x * kMeshBlock + threadIdx.x;
    if (c < ncell) D[c] = make_double2(d[c], 0.0);
}

// F[f][k] <- (-1)^l(f) F[delta](k) K[f][k] / n^3   (k-space; K, the transformed
// kernel fields, is kept for later calls of the same shape)
__global__ void __launch_bounds__(kMeshBlock) k_mesh_product(const double2* __restrict__ D,
                                                   const double2* __restrict__ K, double2* __restrict__ F,
                                                   int64_t total, int64_t ncell, int nlm, uint64_t odd_mask_lo,
                                                   uint64_t odd_mask_hi, double scale)
{
    const int64_t e = (int64_t)blockIdx.x * kMeshBlock + threadIdx.x;
    if (e >= total) return;
    const int f = (int)(e / ncell);
    const int64_t c = e - (int64_t)f * ncell;
    const int lm = f % nlm;
    const bool odd = lm < 64 ? ((odd_mask_lo >> lm) & 1) : ((odd_mask_hi >> (lm - 64)) & 1);
    const double s = odd ? -scale : scale;
    const double2 d = D[c], v = K[e];
    F[e] = make_double2(s * (d.x * v.x - d.y * v.y), s * (d.x * v.y + d.y * v.x));
}

// Rows [0, rows) of a slice: row r is cell prim[r]; its coefficients (FP64, or FP32
// for the FP32 and split-bf16 couplings) and weight delta(cell).  A block moves a
// tile of kRowTile rows x kFieldTile fields through LDS: reads along the cells of a
// field, writes along the fields of a row.
constexpr int kRowTile = 64, kFieldTile = 16;
template <typename T>
__global__ void __launch_bounds__(kMeshBlock) k_mesh_rows(const double2* __restrict__ F, const double* __restrict__ delta,
                                                const int32_t* __restrict__ prim, int64_t rows, int nf,
                                                int64_t ncell, T* __restrict__ alm, double* __restrict__ wprim)
{
    __shared__ double2 tile[kFieldTile][kRowTile + 1];
    const int64_t r0 = (int64_t)blockIdx.x * kRowTile;
    const int f0 = blockIdx.y * kFieldTile;
    for (int i = threadIdx.x; i < kFieldTile * kRowTile; i += kMeshBlock) {
        const int fi = i / kRowTile, ri = i - fi * kRowTile;
        const int64_t r = r0 + ri;
        const int f = f0 + fi;
        tile[fi][ri] = (r < rows && f < nf) ? F[(int64_t)f * ncell + prim[r]] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kFieldTile * kRowTile; i += kMeshBlock) {
        const int ri = i / kFieldTile, fi = i - ri * kFieldTile;
        const int64_t r = r0 + ri;
        const int f = f0 + fi;
        if (r < rows && f < nf) {
            // one 8- or 16-byte store per complex value
            using V2 = typename std::conditional<std::is_same<T, float>::value, float2, double2>::type;
            const double2 v = tile[fi][ri];
            V2 o;
            o.x = (T)v.x;
            o.y = (T)v.y;
            reinterpret_cast<V2*>(alm)[r * nf + f] = o;
        }
    }
    if (blockIdx.y == 0)
        for (int ri = threadIdx.x; ri < kRowTile; ri += kMeshBlock)
            if (r0 + ri < rows) wprim[r0 + ri] = delta[prim[r0 + ri]];
}

unsigned nblk(int64_t n) { return (unsigned)((n + kMeshBlock - 1) / kMeshBlock); }

const char* fft_msg(hipfftResult r)
{
    switch (r) {
    case HIPFFT_SUCCESS: return "success";
    case HIPFFT_ALLOC_FAILED: return "allocation failed";
    case HIPFFT_INVALID_VALUE: return "invalid value";
    case HIPFFT_EXEC_FAILED: return "execution failed";
    case HIPFFT_SETUP_FAILED: return "setup failed";
    case HIPFFT_INVALID_SIZE: return "invalid size";
    default: return "error";
    }
}

#define FFTTRY(x)                                                                      \
    do {                                                                               \
        hipfftResult r__ = (x);                                                        \
        if (r__ != HIPFFT_SUCCESS) {                                                   \
            rc = fail(r__ == HIPFFT_ALLOC_FAILED ? ENCORE_ENOMEM : ENCORE_EDEVICE,    \
                      std::string(#x) + ": " + fft_msg(r__));                          \
            goto done;                                                                 \
        }                                                                              \
    } while (0)

#define HIPTRY_DONE(x)                                \
    do {                                              \
        hipError_t e__ = (x);                         \
        if (e__ != hipSuccess) {                      \
            rc = hip_fail(e__, #x);                   \
            goto done;                                \
        }                                             \
    } while (0)

#define RCTRY(x)                 \
    do {                         \
        if ((rc = (x))) goto done; \
    } while (0)

}  // namespace

}  // namespace encore

using namespace encore;

extern "C" int encore_npcf_mesh(encore_ctx* ctx, const double* delta, int nmesh, double box, int npcf, int lmax,
                                int nbins, const double* edges, uint32_t flags, double* zeta, size_t zeta_len,
                                void* stream)
{
    if (!ctx || !delta) return fail(ENCORE_EINVAL, "NULL ctx or delta");
    if (nmesh < 2 || nmesh > 1024) return fail(ENCORE_EINVAL, "nmesh must be 2..1024");
    if (!(box > 0.0) || !std::isfinite(box)) return fail(ENCORE_EINVAL, "box must be finite and > 0");
    if (flags & ENCORE_NORMALIZE) return fail(ENCORE_EUNSUPPORTED, "encore_npcf_mesh returns raw Z");
    NpcfPlan pl;
    int rc;
    if ((rc = plan_call(npcf, lmax, nbins, edges, flags, &pl))) return rc;
    if (2.0 * edges[nbins] > box) return fail(ENCORE_EINVAL, "edges[nbins] must be <= box/2");
    const size_t need = (size_t)(pl.nlam * pl.nB);
    if (!zeta && need > 0) return fail(ENCORE_EINVAL, "zeta is NULL");
    if (zeta_len < need) return fail(ENCORE_ESIZE, "zeta needs " + std::to_string(need) + " elements");
    const int nlm = (lmax + 1) * (lmax + 2) / 2;
    const int nf = nbins * nlm;
    const int64_t n = nmesh;
    const int64_t ncell = n * n * n;
    if (ncell > INT32_MAX) return fail(ENCORE_EINVAL, "mesh too large");
    std::lock_guard<std::mutex> lock(ctx->mu);
    for (double& t : ctx->timings) t = 0.0;
    if (need == 0) return ENCORE_OK;
    HIPTRY(hipSetDevice(ctx->device));
    Exec& x = ctx->main;
    const hipStream_t s = stream ? (hipStream_t)stream : x.s;
    hipfftHandle plan = 0, plan1 = 0;
    DevTables* tb = nullptr;
    double2* F = nullptr;
    double2* D = nullptr;
    double2* K = nullptr;
    const int64_t total = ncell * nf;
    float ms_fft = 0.f, ms_cpl = 0.f, ms_c = 0.f, ms_tot = 0.f;
    double t_couple = 0.0;
    int nslice = 0;
    rc = ENCORE_OK;
    {
        if ((rc = get_tables_for(ctx, pl, &tb))) return rc;
        // fields and the transform of delta: the context's grow-only mesh buffers
        // The kernel fields and their transforms depend on the shape alone: a call
        // with the shape of the previous one reuses them from meshk.
        std::vector<double> key{(double)nmesh, box, (double)lmax, (double)nbins};
        key.insert(key.end(), edges, edges + nbins + 1);
        const bool warm = ctx->mesh_key == key;
        if (!warm) ctx->mesh_key.clear();
        RCTRY(ensure(x.meshk, sizeof(double2) * (size_t)total));
        RCTRY(ensure(x.mesh, sizeof(double2) * (size_t)total));
        RCTRY(ensure(x.meshd, sizeof(double2) * (size_t)ncell));
        F = (double2*)x.mesh.p;
        D = (double2*)x.meshd.p;
        K = (double2*)x.meshk.p;
        MeshKernelArgs ka;
        std::memset(&ka, 0, sizeof(ka));
        ka.n = nmesh; ka.nbins = nbins; ka.nlm = nlm; ka.lmax = lmax;
        ka.h = box / (double)nmesh;
        for (int b = 0; b <= nbins; ++b) ka.e2[b] = edges[b] * edges[b];
        gather_tables(lmax, ka.kappa);
        uint64_t odd_lo = 0, odd_hi = 0;
        for (int l = 0; l <= lmax; ++l)
            for (int m = 0; m <= l; ++m) {
                const int lm = l * (l + 1) / 2 + m;
                ka.lm_l[lm] = l; ka.lm_m[lm] = m;
                if (l >= m + 2) {
                    // gamma_lm = b_lm kappa_{l-2,m} / kappa_{l-1,m} of the recurrence
                    const double l1 = l - 1;
                    const double bl = std::sqrt((l1 * l1 - (double)m * m) / (4.0 * l1 * l1 - 1.0));
                    const double den = (l == m + 2) ? std::sqrt(2.0 * m + 3.0)
                                                    : std::sqrt((4.0 * l1 * l1 - 1.0) / (l1 * l1 - (double)m * m));
                    ka.gamma[lm] = bl / den;
                }
                if (l & 1) (lm < 64 ? odd_lo : odd_hi) |= (uint64_t)1 << (lm & 63);
            }
        // batched transforms over the nf interleaved fields (element stride nf)
        // the plans (and their work areas) of the last (nmesh, nf) are kept
        if (!(ctx->mesh_plan && ctx->mesh_plan1 && ctx->mesh_plan_n == nmesh && ctx->mesh_plan_nf == nf)) {
            mesh_release(ctx);
            int dims[3] = {nmesh, nmesh, nmesh};
            hipfftHandle p = 0, p1 = 0;
            FFTTRY(hipfftCreate(&p));
            ctx->mesh_plan = p;
            size_t work = 0;
            FFTTRY(hipfftMakePlanMany(p, 3, dims, dims, 1, (int)ncell, dims, 1, (int)ncell, HIPFFT_Z2Z, nf, &work));
            FFTTRY(hipfftPlan3d(&p1, nmesh, nmesh, nmesh, HIPFFT_Z2Z));
            ctx->mesh_plan1 = p1;
            ctx->mesh_plan_n = nmesh;
            ctx->mesh_plan_nf = nf;
        }
        plan = (hipfftHandle)ctx->mesh_plan;
        plan1 = (hipfftHandle)ctx->mesh_plan1;
        FFTTRY(hipfftSetStream(plan, s));
        FFTTRY(hipfftSetStream(plan1, s));
        HIPTRY_DONE(hipEventRecord(x.ev[0], s));
        if (!warm) {
            hipLaunchKernelGGL(k_mesh_kernels, dim3(nblk(total)), dim3(kMeshBlock), 0, s, ka, K, total, ncell);
            HIPTRY_DONE(hipGetLastError());
        }
        hipLaunchKernelGGL(k_mesh_complex, dim3(nblk(ncell)), dim3(kMeshBlock), 0, s, delta, D, ncell);
        HIPTRY_DONE(hipGetLastError());
        FFTTRY(hipfftExecZ2Z(plan1, (hipfftDoubleComplex*)D, (hipfftDoubleComplex*)D, HIPFFT_FORWARD));
        if (!warm) FFTTRY(hipfftExecZ2Z(plan, (hipfftDoubleComplex*)K, (hipfftDoubleComplex*)K, HIPFFT_FORWARD));
        hipLaunchKernelGGL(k_mesh_product, dim3(nblk(total)), dim3(kMeshBlock), 0, s, D, K, F, total, ncell, nlm,
                           odd_lo, odd_hi, 1.0 / (double)ncell);
        HIPTRY_DONE(hipGetLastError());
        FFTTRY(hipfftExecZ2Z(plan, (hipfftDoubleComplex*)F, (hipfftDoubleComplex*)F, HIPFFT_BACKWARD));
        HIPTRY_DONE(hipEventRecord(x.ev[1], s));

        // every cell is a primary: coupling over slices of cells, as for a catalog
        const int64_t outs = acc_len(pl, tb);
        const int64_t cap = cap_rows(pl);
        RCTRY(ensure(x.prim, sizeof(int32_t) * (size_t)ncell));
        RCTRY(ensure(x.Tjob, sizeof(double) * (size_t)outs));
        RCTRY(ensure(x.zeta, sizeof(double) * need));
        HIPTRY_DONE((hipError_t)launch_iota((int32_t*)x.prim.p, ncell, s));
        HIPTRY_DONE((hipError_t)launch_fill((double*)x.Tjob.p, outs, 0.0, s));
        DevGrid cells;   // segment descriptor of the slices (no gather runs on it)
        cells.n = ncell;
        const int64_t sr = job_split_rows(pl, tb, ncell, cap);
        const hipStream_t own = x.s;
        x.s = s;
        for (int64_t r0 = 0; r0 < ncell && rc == ENCORE_OK;) {
            int64_t take = std::min<int64_t>(ncell - r0, std::max<int64_t>(cap / sr, 1) * sr);
            std::vector<Chunk> chunks{Chunk{&cells, (const int32_t*)x.prim.p, r0, r0 + take, sr, (double*)x.Tjob.p}};
            SliceLaunch L;
            rc = prepare_slice(x, x.segs, x.splits, x.redp, pl, tb, edges, chunks, L);
            if (rc) break;
            hipError_t e = hipEventRecord(x.ev[2], s);
            if (e == hipSuccess) {
                const dim3 grid((unsigned)((take + kRowTile - 1) / kRowTile), (unsigned)((nf + kFieldTile - 1) / kFieldTile));
                if (pl.prec == 0)
                    hipLaunchKernelGGL(k_mesh_rows<double>, grid, dim3(kMeshBlock), 0, s, F, delta,
                                       (const int32_t*)x.prim.p + r0, take, nf, ncell, (double*)x.alm.p,
                                       (double*)x.wprim.p);
                else
                    hipLaunchKernelGGL(k_mesh_rows<float>, grid, dim3(kMeshBlock), 0, s, F, delta,
                                       (const int32_t*)x.prim.p + r0, take, nf, ncell, (float*)x.alm.p,
                                       (double*)x.wprim.p);
                e = hipGetLastError();
            }
            if (e == hipSuccess) rc = launch_slice_couple(L, pl, tb, s);
            else rc = hip_fail(e, "mesh rows");
            if (rc == ENCORE_OK) {
                e = hipEventRecord(x.ev[3], s);
                if (e == hipSuccess) e = hipEventSynchronize(x.ev[3]);   // host slice tables are reused
                float ms = 0.f;
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, x.ev[2], x.ev[3]);
                if (e != hipSuccess) rc = hip_fail(e, "mesh slice");
                t_couple += ms;
            }
            r0 += take;
            ++nslice;
        }
        x.s = own;
        if (rc) goto done;
        HIPTRY_DONE(hipEventRecord(x.ev[2], s));
        {
            const hipStream_t keep = x.s;
            x.s = s;
            rc = contract_job(x, pl, tb, (const double*)x.Tjob.p, nullptr, (double*)x.zeta.p);
            x.s = keep;
            if (rc) goto done;
        }
        HIPTRY_DONE(hipEventRecord(x.ev[3], s));
        HIPTRY_DONE(hipMemcpyAsync(zeta, x.zeta.p, sizeof(double) * need, hipMemcpyDeviceToHost, s));
        HIPTRY_DONE(hipStreamSynchronize(s));
        HIPTRY_DONE(hipEventElapsedTime(&ms_fft, x.ev[0], x.ev[1]));
        HIPTRY_DONE(hipEventElapsedTime(&ms_c, x.ev[2], x.ev[3]));
        HIPTRY_DONE(hipEventElapsedTime(&ms_tot, x.ev[0], x.ev[3]));
        (void)ms_cpl;
        ctx->timings[0] = ms_tot;
        ctx->timings[1] = ms_fft;    // kernel fields + transforms + products
        ctx->timings[2] = t_couple;  // rows + coupling + in-order reduction
        ctx->timings[3] = ms_c;
        ctx->timings[4] = nslice;
        ctx->timings[5] = warm ? 1.0 : 0.0;   // kernel-field transforms reused
        ctx->mesh_key = key;                   // meshk holds this shape's transforms
    }
done:
    return rc;
}

void encore::mesh_release(encore_ctx* ctx)
{
    if (ctx->mesh_plan) (void)hipfftDestroy((hipfftHandle)ctx->mesh_plan);
    if (ctx->mesh_plan1) (void)hipfftDestroy((hipfftHandle)ctx->mesh_plan1);
    ctx->mesh_plan = nullptr;
    ctx->mesh_plan1 = nullptr;
    ctx->mesh_plan_n = 0;
    ctx->mesh_plan_nf = 0;
}
