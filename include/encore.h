/*
 * encore.h -- C ABI of the MI355X (gfx950) N-point correlation function hot path.
 *
 * The library computes the multiplets of the discrete isotropic NPCF estimator of
 * Philcox, Slepian, Hou, Warner, Cahn & Eisenstein (2021), Section 3.2.1 (eq.
 * NPCF-mult-discrete-binned-estimator with the harmonic coefficients of eq.
 * binned-discrete-alm), for N = 3..6:
 *
 *   Z^B_L = sum_i w_i sum_M E(L) C^L_M prod_{k=1}^{N-1} a~^{b_k}_{l_k m_k}(i),
 *   a~^b_lm(i) = sum_{j != i} w_j Y_lm((r_j - s_i)^) Theta^b(|r_j - s_i|),
 *
 * with L a multiplet (Section 2.1), B = (b_1 < ... < b_{N-1}) distinct radial bins
 * (Section 3.2.1), C^L_M the coupling of eq. basis-coupling.  By default Z is raw
 * (no 1/V, no 1/v_b); ENCORE_NORMALIZE divides by V prod_k v_{b_k}.
 *
 * Conventions shared by every entry point
 *  - Every function returns an int status: ENCORE_OK (0) or a negative code.  No
 *    C++ exception crosses the ABI.  encore_last_error() returns a message for the
 *    last failure on the calling thread.
 *  - The caller owns every buffer it passes (host or device); the library owns
 *    the handles it returns (free them with the matching destroy/free call).
 *  - Outputs are written only on success.
 *  - Positions are FP64, row-major [n][3]; weights FP64 [n].
 *  - A radial bin b holds pairs with edges[b]^2 <= r^2 < edges[b+1]^2, r^2 formed
 *    in FP64 as (dx*dx + dy*dy) + dz*dz; edges[0] > 0 excludes the self pair.
 *  - Periodic boxes use the minimum image; they need 0 <= x < box and
 *    edges[nbins] <= box/2 on every axis.
 *  - Output layout: multiplet-major, zeta[l_index * n_bin_tuples + b_index].
 *    Multiplets are ordered lexicographically over (l1, l2, (l12), l3, (l123), l4,
 *    l5) with the last entry fastest; bin tuples lexicographically with the last
 *    bin fastest.  Parity-even multiplets report Re Z, parity-odd ones Im Z
 *    (Section 3.1: even multiplets are real, odd ones imaginary).
 */
#ifndef ENCORE_H
#define ENCORE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define ENCORE_OK            0
#define ENCORE_EINVAL       -1   /* bad argument (message says which) */
#define ENCORE_ESIZE        -2   /* output buffer too small (message gives the size) */
#define ENCORE_ENOMEM       -3   /* device or host allocation failed */
#define ENCORE_EDEVICE      -4   /* HIP runtime error */
#define ENCORE_EUNSUPPORTED -5   /* combination not built */
#define ENCORE_EAGAIN       -6   /* encore_server_wait: job not finished within the timeout */

/* flags */
#define ENCORE_PERIODIC        0x1u   /* periodic box (minimum image), box[] required */
#define ENCORE_ALLPARITY       0x2u   /* odd-parity multiplets too (Section 3.1) */
#define ENCORE_DMR             0x4u   /* data-minus-randoms weighting, see build_grid */
#define ENCORE_NORMALIZE       0x8u   /* zeta = Z / (V prod_k v_{b_k}) */
#define ENCORE_PREC_FP64       0x00u  /* plain path: FP64 everywhere */
#define ENCORE_PREC_FP32       0x10u  /* FP32 a_lm and products, FP64 sum over primaries */
#define ENCORE_PREC_SPLITBF16  0x20u  /* FP32 a_lm, split-bf16 MFMA coupling */
#define ENCORE_PREC_MASK       0x30u
#define ENCORE_DEBUG_FULLGRID  0x100u /* encore_debug_alm: gather every point as in encore_npcf */

typedef struct encore_ctx encore_ctx;   /* device, stream, table and workspace cache */
typedef struct encore_grid encore_grid; /* device-resident cell-sorted catalog */

/* Message for the last failing call on this thread ("" if none).  Owned by the
 * library, valid until the next call on this thread. */
const char* encore_last_error(void);

/* Library version string (static). */
const char* encore_version(void);

/* Create a context on HIP device `hip_device` (>= 0).  *out receives the handle.
 * Errors: EINVAL (bad device or NULL out), EDEVICE. */
int encore_create(int hip_device, encore_ctx** out);

/* Destroy a context.  Every grid built on it must be freed first.  NULL is a no-op. */
int encore_destroy(encore_ctx* ctx);

/*
 * Build the device-resident cell grid of one catalog (Section 4.1: particles are
 * placed on a Cartesian grid for the neighbour search).
 *
 *  pos    [n][3] FP64 positions, host memory.
 *  w      [n] FP64 weights, host memory.
 *  n      number of points (>= 1).
 *  n_data with ENCORE_DMR: points [0, n_data) are data, [n_data, n) randoms with
 *         positive input weights; the library replaces the random weights by
 *         -w_R * sum(w_D) / sum(w_R) on the device in FP64, so the total weight is
 *         zero (Section 4.2, data-minus-randoms field).  Ignored without ENCORE_DMR.
 *  box    [3] periodic box side lengths (required with ENCORE_PERIODIC, else ignored).
 *  r_max  largest separation any later encore_npcf call on this grid will bin
 *         (> 0; sets the cell size).
 *  flags  ENCORE_PERIODIC, ENCORE_DMR.
 *  stream hipStream_t to order the work on (NULL: the context's stream).  The call
 *         returns after the grid is built.
 *  out    receives the grid handle.
 * Errors: EINVAL (non-finite input, n < 1, point outside a periodic box, bad
 * n_data, zero data or random weight sum), ENOMEM, EDEVICE.
 */
int encore_build_grid(encore_ctx* ctx, const double* pos, const double* w, int64_t n,
                      int64_t n_data, const double* box, double r_max, uint32_t flags,
                      void* stream, encore_grid** out);

/* As encore_build_grid, but pos and w are device pointers (e.g. torch data_ptr())
 * on the context's device; they are read, not adopted. */
int encore_build_grid_device(encore_ctx* ctx, const double* pos, const double* w, int64_t n,
                             int64_t n_data, const double* box, double r_max, uint32_t flags,
                             void* stream, encore_grid** out);

/* Free a grid (NULL is a no-op). */
int encore_free_grid(encore_grid* grid);

/* Number of points of a grid (>= 0), or a negative status. */
int64_t encore_grid_size(const encore_grid* grid);

/*
 * NPCF multiplets of a grid's catalog (eq. NPCF-mult-discrete-binned-estimator).
 *
 *  npcf    N, 3..6.
 *  lmax    largest principal ell, 0..10 (N = 3, 4), 0..5 (N = 5), 0..4 (N = 6).
 *  nbins   number of radial bins (1..16); nbins < N-1 gives zero bin tuples.
 *  edges   [nbins+1] host FP64, strictly increasing, edges[0] > 0,
 *          edges[nbins] <= r_max of the grid.
 *  flags   ENCORE_ALLPARITY, ENCORE_NORMALIZE, one ENCORE_PREC_* value.
 *  volume  V for ENCORE_NORMALIZE (<= 0: the periodic box volume); else ignored.
 *  zeta    host FP64 output [n_multiplets * n_bin_tuples].
 *  zeta_len length of zeta in elements; ESIZE (with the needed length in the
 *          message) if too small.
 *  primary_subset  NULL: every point is a primary.  Otherwise [n_subset] indices
 *          into the catalog (input order) of the primaries to sum over (the sum over
 *          i restricted; secondaries are always the whole catalog).
 *  stream  hipStream_t (NULL: the context's stream).  Synchronous: returns once zeta
 *          is on the host.
 * Errors: EINVAL, ESIZE, ENOMEM, EDEVICE, EUNSUPPORTED (ENCORE_PREC_SPLITBF16 when
 * the coupling's output tiles outnumber its 32-bit index, e.g. the 6PCF at lmax 4
 * with 16 bins).  The split-bf16 coupling stages each 16-primary block of
 * coefficients in LDS up to 256 coefficients per primary and reads larger blocks
 * (up to 16 bins x 66 coefficients) in global memory.
 *
 * Precision modes (the precision of the harmonic coefficients, the coupling
 * products and the sum over primaries): FP64 / FP64 / FP64 (plain path); FP32 /
 * FP32 / FP64; FP32 / split-bf16 matrix-core products (hi*hi + hi*lo + lo*hi, FP32
 * accumulation over 256 primaries) / FP64.
 */
int encore_npcf(encore_ctx* ctx, const encore_grid* grid, int npcf, int lmax, int nbins,
                const double* edges, uint32_t flags, double volume, double* zeta,
                size_t zeta_len, const int64_t* primary_subset, int64_t n_subset,
                void* stream);

/*
 * The same multiplets for several catalogs at once (one job per grid).  All jobs
 * share npcf, lmax, the bins and the flags.  The gather runs as ONE persistent launch per slice of primaries: waves
 * pull (catalog, primary, bin group) work items from device work queues, so
 * catalogs of uneven size and neighbour count share the GPU without per-job
 * launches.  The coupling and FP64 sums stay per job.
 *  grids   [njobs] grids built on ctx (may repeat).
 *  zeta    host FP64 [njobs][n_multiplets * n_bin_tuples].
 *  zeta_len length of zeta in elements (>= njobs * n_multiplets * n_bin_tuples).
 *  primary_subsets  NULL: every point of every catalog is a primary.  Otherwise
 *          [njobs] host pointers, each NULL (every point of that catalog) or
 *          [n_subsets[j]] catalog indices (input order) of job j's primaries, as
 *          primary_subset of encore_npcf.
 *  n_subsets  [njobs] (read where primary_subsets[j] is not NULL).
 * ENCORE_NORMALIZE uses each periodic grid's box volume.  Errors as encore_npcf.
 */
int encore_npcf_batch(encore_ctx* ctx, const encore_grid* const* grids, int njobs, int npcf,
                      int lmax, int nbins, const double* edges, uint32_t flags, double* zeta,
                      size_t zeta_len, const int64_t* const* primary_subsets,
                      const int64_t* n_subsets, void* stream);

/*
 * Serving loop.  A server accepts catalog jobs from any thread and runs them on
 * its lanes (worker threads, each with its own HIP stream and workspaces) on the
 * context's device.  Every job is the estimator of encore_npcf over every point
 * of its catalog (Section 3.2.1), with its own N, lmax, bins and precision.
 *
 *  - Admission: jobs wait in arrival order; the head is admitted while its
 *    device-memory footprint fits in hbm_budget minus what admitted jobs hold,
 *    and fewer than max_active jobs are admitted.  An admitted job keeps its grid
 *    and accumulated sums on the device until it completes.
 *  - Continuous batching: each lane iteration runs one slice of at most
 *    slice_rows primaries taken, oldest job first, from every admitted idle job
 *    of the same class (same npcf, lmax, bins, precision and parity) in one
 *    persistent gather launch; jobs that arrive meanwhile join at the next
 *    iteration.  Lanes run concurrently, so their work overlaps on the device.
 *  - A job's rows are reduced in a fixed order that depends only on the job, so
 *    its result is bit-identical to encore_npcf on the same catalog whatever it
 *    shares the device with.
 *  - A job that fails (invalid catalog, device allocation failure) fails alone;
 *    its error is returned by encore_server_wait.
 * Lane workspaces (a~ of one slice, coupling partial sums) come on top of the
 * budget: at most slice_rows x (nbins x (lmax+1)(lmax+2)/2 x 8 bytes in FP32,
 * 16 in FP64) each, plus a few MB.
 */
typedef struct encore_server encore_server;

/* Create a server on ctx (which must outlive it).
 *  hbm_budget  device bytes that admitted jobs may hold together (> 0).
 *  n_lanes     worker threads / streams (1..8).
 *  max_active  admitted jobs at once (>= 1).
 *  slice_rows  primaries per lane iteration (>= 1).
 * Errors: EINVAL, ENOMEM, EDEVICE. */
int encore_server_create(encore_ctx* ctx, size_t hbm_budget, int n_lanes, int max_active,
                         int64_t slice_rows, encore_server** out);

/* Submit one job; the catalog (host pos [n][3], w [n], box[3] when periodic) and
 * edges are copied, so the caller may free them on return.  flags: precision,
 * ENCORE_ALLPARITY, ENCORE_PERIODIC (box required), ENCORE_DMR (n_data as in
 * encore_build_grid), ENCORE_NORMALIZE (periodic only: V = box volume).  r_max is
 * edges[nbins].  *job_id receives the job's id.
 * Errors: EINVAL (bad arguments, server shutting down), ESIZE (footprint larger
 * than the whole budget), EUNSUPPORTED.  Errors found while the job runs
 * (non-finite input, points outside the box) are reported by encore_server_wait. */
int encore_server_submit(encore_server* srv, const double* pos, const double* w, int64_t n,
                         int64_t n_data, const double* box, int npcf, int lmax, int nbins,
                         const double* edges, uint32_t flags, int64_t* job_id);

/* Wait for a job (timeout_s < 0: no limit; 0: poll).  On success writes zeta
 * (host FP64 [n_multiplets * n_bin_tuples], layout as encore_npcf) and, if times
 * is not NULL, times[4] = submit, admit, first slice start, done, in seconds since
 * the server was created; the job's record is then released (wait once per job).
 * Errors: EAGAIN (not finished: the record is kept), ESIZE (zeta_len too small:
 * record kept), EINVAL (unknown or collected id), or the job's own failure code
 * (record released). */
int encore_server_wait(encore_server* srv, int64_t job_id, double timeout_s, double* zeta,
                       size_t zeta_len, double* times);

/* Counters: out[12] = submitted, done, failed, queued, admitted, bytes held by
 * admitted jobs, peak of that, primaries run, slices run, gather ms, coupling ms
 * (summed over lanes), lane workspace bytes.  Errors: EINVAL, ESIZE (out_len < 12). */
int encore_server_stats(encore_server* srv, double* out, size_t out_len);

/* Finish every submitted job, stop the lanes and free the server (NULL: no-op).
 * Results not collected with encore_server_wait are discarded. */
int encore_server_destroy(encore_server* srv);

/*
 * Graph-captured job step: the computation of encore_npcf over every point of one
 * grid (gather -> coupling -> FP64 sum over primaries -> contraction, eq.
 * NPCF-mult-discrete-binned-estimator), prepared once and recorded into a HIP
 * graph on the plan's own stream, then replayed by encore_plan_execute: repeated
 * runs of one job cost one graph launch and no host-side preparation.
 *  grid     must outlive the plan (encore_free_grid refuses while plans exist);
 *           grids are immutable, so every replay computes the same zeta.
 *  other arguments as encore_npcf (all points are primaries; no stream argument).
 * The plan owns its workspaces (sized at creation; replays allocate nothing) and a
 * pinned host copy of zeta.
 * Errors: as encore_npcf; EDEVICE if the capture fails.
 */
typedef struct encore_plan encore_plan;
int encore_plan_create(encore_ctx* ctx, encore_grid* grid, int npcf, int lmax, int nbins,
                       const double* edges, uint32_t flags, double volume, encore_plan** out);
/* Replay the plan's graph and wait for it; zeta as encore_npcf.  Errors: EINVAL,
 * ESIZE, EDEVICE.  Calls on one plan must not overlap. */
int encore_plan_execute(encore_plan* plan, double* zeta, size_t zeta_len);
/* Destroy a plan (NULL: no-op). */
int encore_plan_destroy(encore_plan* plan);

/*
 * Work of the split-BF16 MFMA coupling for (npcf, lmax, nbins, ENCORE_ALLPARITY in
 * flags), host only: out[0] = 16x16 output tiles computed per 16 primaries (three
 * 16x16x32 bf16 MFMAs each), out[1] = 16-row operand tiles formed per 16
 * primaries, out[2] = entries of T used (tuples x bin tuples), out[3] = dense
 * entries accumulated.  Errors: EINVAL, ESIZE (out_len < 4), EUNSUPPORTED.
 */
int encore_mfma_plan_stats(int npcf, int lmax, int nbins, uint32_t flags, int64_t* out, size_t out_len);

/*
 * Autotuner of the launch shapes: builds trial grids of the catalog (host arrays,
 * as encore_build_grid) with 8 cell shapes (cell side r_max/d on y and z,
 * r_max/(d*s) on x, where one cell row is a contiguous particle range; (d, s) =
 * (5, 16) -- the default without tuning --, (5, 8), (6, 16), (6, 8), (8, 8),
 * (8, 4), (5, 24), (4, 16)) and times,
 * for each, the gather + coupling of this job (as encore_npcf) over a sample of
 * n_sample primaries (16 runs of consecutive cell-sorted primaries spread over the
 * grid, so that neighbouring work items share cells as in a full pass), for every compiled
 * bins-per-work-item value of the gather.  The fastest (d, s) becomes the cell
 * shape of later grids built on ctx; the fastest bins-per-item value is used by
 * later calls with the same lmax, gather precision and nbins.  The default shape
 * and bins per item are kept unless the fastest is more than 2% faster on the
 * sample (sample timings of nearby shapes differ by about that much).  The choice changes
 * only the order of floating-point operations, never what is computed.
 *  report  NULL or [5]: d, s, bins per item, best ms, ms of the default shape.
 * Errors: as encore_build_grid and encore_npcf; ESIZE if report_len < 5.
 */
int encore_autotune(encore_ctx* ctx, const double* pos, const double* w, int64_t n, int64_t n_data,
                    const double* box, int npcf, int lmax, int nbins, const double* edges, uint32_t flags,
                    int64_t n_sample, double* report, size_t report_len);

/*
 * Allocation-free encore_npcf, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Arguments, layout, result and errors as encore_npcf (zeta on the
 * host; the grid is built beforehand), but the call makes no device allocation and
 * frees nothing: the coupling tables, the primary list, the per-slice
 * coefficients and partial sums, the job's sums and zeta all live in one static
 * scratch array of 256 MiB per device (held from the first encore_create on that
 * device until the process ends), and slices are sized to fit it.
 *  - Errors: ESIZE (with the bytes needed) when one slice of at least one coupling
 *    split no longer fits, e.g. N = 6 at lmax 4 with many bins.
 *  - Results equal encore_npcf's bit for bit when both run the job as one slice;
 *    with more slices only the rounding order of the reduced-precision sums
 *    differs.
 *  - Every call on a device shares that device's array and leaves its contents
 *    behind; calls on one context are serialised, calls that overlap on one GPU
 *    from different contexts or threads race and must not be made.
 */
int encore_npcf_noalloc(encore_ctx* ctx, const encore_grid* grid, int npcf, int lmax, int nbins,
                        const double* edges, uint32_t flags, double volume, double* zeta,
                        size_t zeta_len, const int64_t* primary_subset, int64_t n_subset,
                        void* stream);

/*
 * Gridded data (Section 3.2, Gridded Data): the multiplets of a density field
 * given on a periodic mesh, with the harmonic coefficients of every cell from FFTs
 * (eq. alm-binned-def-fft): a~^b_lm(s) = sum_u delta(s + u) Y_lm(u^) Theta^b(|u|)
 * over the mesh offsets u (minimum image), computed as batched FP64 complex
 * transforms, then Z^B_L = sum_s delta(s) sum_M E(L) C^L_M prod_k a~ with every
 * cell a primary of weight delta(s) (eq. NPCF-mult-binned-estimator, raw: no
 * 1/V, no 1/v_b), coupled as encore_npcf couples a catalog.  The bin rule is the
 * discrete one (edges[b]^2 <= |u|^2 < edges[b+1]^2, |u|^2 in FP64), so a catalog
 * assigned to the mesh cell by cell gives encore_npcf's result for the catalog
 * moved to its cell centres (h (i + 1/2)).
 *  delta  device FP64 [nmesh][nmesh][nmesh], delta[(ix * nmesh + iy) * nmesh + iz],
 *         cell (ix, iy, iz) spanning [ix h, (ix + 1) h) x ..., h = box / nmesh.
 *  nmesh  2..1024; box > 0 the period; edges[nbins] <= box / 2.
 *  npcf, lmax, nbins, edges, zeta, zeta_len  as encore_npcf; flags: ENCORE_ALLPARITY
 *         and one ENCORE_PREC_* (the precision of the coupling; the transforms are
 *         FP64).  ENCORE_NORMALIZE is EUNSUPPORTED.
 *  stream hipStream_t (NULL: the context's stream); synchronous.
 * Device memory: 2 nbins * (lmax+1)(lmax+2)/2 + 1 complex FP64 fields of nmesh^3
 * cells and the transform plans with their work areas, kept by the context for
 * later calls (the plans per (nmesh, number of fields)).  The
 * transforms of the kernel fields Y_lm Theta^b depend on (nmesh, box, lmax, edges)
 * alone: a call with the shape of the context's previous mesh call reuses them and
 * transforms only delta and the products.
 * Timings: [1] the fields, transforms and products, [2] the coupling, [5] 1 when
 * the kernel-field transforms were reused, else 0.
 * Errors: EINVAL, ESIZE, ENOMEM, EDEVICE, EUNSUPPORTED.
 */
int encore_npcf_mesh(encore_ctx* ctx, const double* delta, int nmesh, double box, int npcf, int lmax,
                     int nbins, const double* edges, uint32_t flags, double* zeta, size_t zeta_len,
                     void* stream);

/* One-shot form: build a grid from host arrays, run encore_npcf, free the grid.
 * r_max = edges[nbins]; box may be NULL for a non-periodic catalog. */
int encore_npcf_simple(const double* pos, const double* w, int64_t n, int npcf, int lmax,
                       int nbins, const double* edges, const double* box, uint32_t flags,
                       double* zeta, size_t zeta_len);

/* |multiplets| for (N, lmax, flags & ENCORE_ALLPARITY), or a negative status. */
int64_t encore_num_multiplets(int npcf, int lmax, uint32_t flags);

/* |bin tuples| = C(nbins, N-1), or a negative status. */
int64_t encore_num_bin_tuples(int npcf, int nbins);

/* Multiplet table in output order: out[k * width + c], width = 2N-5 for N >= 4
 * ((l1, l2, l12, l3, l123, l4, l5) truncated to N), width 2 for N = 3.
 * out_len in elements; ESIZE if too small. */
int encore_multiplet_table(int npcf, int lmax, uint32_t flags, int32_t* out, size_t out_len);

/*
 * The coupling terms the device path sums (Appendix B half sum): for every
 * multiplet and every M with m_{N-1} >= 0 and C^L_M != 0,
 *   coef = 2 S(m_{N-1}) E(L) C^L_M,  S(0) = 1/2, S(m > 0) = 1,
 * applied to Re (even L) or Im (odd L) of prod_k a~^{b_k}_{l_k m_k}.
 * With out arrays NULL, only *n_terms is written.  Otherwise (capacity cap):
 *   lam[t], l[t*(N-1)+k], m[t*(N-1)+k], coef[t].
 * Host-only (no device needed).
 */
int encore_coupling_terms(int npcf, int lmax, uint32_t flags, int64_t* n_terms, int64_t cap,
                          int32_t* lam, int32_t* l, int32_t* m, double* coef);

/* Wigner 3j symbol (j1 j2 j3; m1 m2 m3) as the library's host tables use it. */
double encore_wigner3j(int j1, int j2, int j3, int m1, int m2, int m3);

/*
 * Raw harmonic coefficients a~^b_lm (eq. binned-discrete-alm without 1/v_b) of k
 * primaries, computed by the device gather kernel of the given precision.
 * With ENCORE_DEBUG_FULLGRID the gather runs over every point of the catalog in
 * the launch configuration encore_npcf uses (one launch), and the requested
 * primaries' rows are returned.
 *  primaries [k] catalog indices (input order).
 *  alm_out   host FP64 [k][nbins][(lmax+1)(lmax+2)/2][2] (re, im), m >= 0 only,
 *            index l(l+1)/2 + m.
 */
int encore_debug_alm(encore_ctx* ctx, const encore_grid* grid, int lmax, int nbins,
                     const double* edges, uint32_t flags, const int64_t* primaries, int64_t k,
                     double* alm_out);

/*
 * Edge correction (Section 3.2, eqs. edge-correction-matrix and
 * edge-corrected-NPCF).  From the multiplets N_L^B of the data-minus-randoms field
 * and R_L^B of the randoms alone (both as encore_npcf returns them, same flags),
 * builds per bin tuple B the coupling matrix
 *     M_{L L''}(B) = sum_{L'} (R_{L'}^B / R_0^B) s(L, L') E(L'') G^{L L' L''}
 * with the generalized Gaunt integrals G of eq. generalized-gaunt-def (closed forms
 * of Appendix A for N = 3, 4, 5; for N = 6 the same construction with one 9j
 * symbol per node of the coupling tree), built once per (npcf, lmax, parity) on
 * the host and kept, and solves N_{L''}^B / R_0^B = sum_L zeta_L^B M_{L L''}
 * for zeta on the device (FP64, Gaussian elimination with partial pivoting and back substitution).
 * The paper's equations are written for the complex multiplets; odd multiplets are
 * imaginary and are passed and returned as their imaginary parts, which gives the
 * factor s(L, L') = i * i = -1 to terms with L and L' both odd (+1 otherwise).  In
 * these real numbers M is symmetric.
 * L, L', L'' run over the multiplets of (npcf, lmax, flags & ENCORE_ALLPARITY);
 * zeta is returned for those with every principal ell <= lmax_out (the paper
 * measures at lmax_out + 1), in the same order.
 *  nmult, rmult  host FP64 [nlam][nB] (encore_num_multiplets x the bin tuples),
 *                mult_len elements each; row 0 of rmult is R_0.
 *  zeta          host FP64 [nout][nB]; B with R_0 = 0 or a singular matrix get NaN.
 *  coupling      NULL or host FP64 [nB][nlam][nlam]: M[B][L][L''].
 *  n_singular    NULL or the number of B without a solution.
 * Device memory: the nB matrices of nlam^2 FP64 values (twice when coupling is
 * requested), the Gaunt table and the multiplets, in grow-only workspaces kept by
 * the context for later calls; the table is uploaded once per (npcf, lmax, parity).
 * Errors: EINVAL, ESIZE (a buffer too small; the message gives the size),
 * EUNSUPPORTED (more than 4096 multiplets, e.g. npcf = 6 at lmax 4), ENOMEM, EDEVICE.
 */
int encore_edge_correct(encore_ctx* ctx, int npcf, int lmax, int nbins, uint32_t flags,
                        const double* nmult, const double* rmult, size_t mult_len, int lmax_out,
                        double* zeta, size_t zeta_len, double* coupling, size_t coupling_len,
                        int64_t* n_singular);

/*
 * Random-split co-adding (Section 4.2, Reconstructing the geometry-corrected
 * NPCF): the random catalog is cut into disjoint parts R_1..R_K; part k gives the
 * data-minus-randoms catalog D + R_k, whose multiplets N^(k) are measured as by
 * encore_npcf, and the mean (1/K) sum_k N^(k) is returned.  The data's share of
 * the harmonic coefficients of every data primary is the same in each part: it is
 * gathered ONCE (from data_grid) and kept on the device (n_data rows of
 * nbins * (lmax+1)(lmax+2)/2 complex values, FP64 or FP32 by precision, in a
 * grow-only workspace of the context, freed with it).  In each
 * part the data primaries are then gathered against the part's randoms alone (a
 * grid of R_k with its D-R weights, built from the split grid on first use and
 * freed with it) and get the kept rows added; the random primaries are gathered
 * against D + R_k.  Data-data pairs are thus visited once, not K times.  This is
 * done with ENCORE_PREC_FP64 when the parts hold at least 6,000 points per r_max^3
 * on average (r_max = edges[nbins]); below that a work item's cost is mostly its
 * cell geometry, not its pairs, and in the FP32 modes the separate data and random
 * shares of a coefficient, each much larger than their D-R sum, would cost accuracy
 * (1.6e-3 instead of 1e-6 of max|Z| measured on a dense catalog).  Otherwise each
 * part runs as one catalog (same result up to rounding order).  The environment
 * variable ENCORE_SPLIT_CACHE=1 / 0 forces either way.
 *
 *  data_grid   grid of the data alone (built without ENCORE_DMR).
 *  split_grids [nsplit] grids built with ENCORE_DMR on D + R_k: the first n_data
 *              input points are the data catalog, in data_grid's input order, with
 *              the same positions and weights (checked on the device).  Same
 *              periodic box as data_grid.
 *  nsplit      K >= 1.
 *  npcf, lmax, nbins, edges, flags, volume  as encore_npcf (edges within the
 *              r_max of every grid).
 *  zeta        host FP64 [n_multiplets * n_bin_tuples]: the mean over the parts.
 *  zeta_splits NULL, or host FP64 [nsplit][n_multiplets * n_bin_tuples]: N^(k).
 *  stream      as encore_npcf.
 * Timings: [1] includes the data gather, [5] its pairs; [0] excludes building
 * the randoms-only grids (with the data part kept).
 * Errors: EINVAL (grids that do not match as above), ESIZE, ENOMEM, EDEVICE,
 * EUNSUPPORTED as encore_npcf.
 */
int encore_npcf_splits(encore_ctx* ctx, const encore_grid* data_grid,
                       const encore_grid* const* split_grids, int nsplit, int npcf, int lmax,
                       int nbins, const double* edges, uint32_t flags, double volume,
                       double* zeta, size_t zeta_len, double* zeta_splits,
                       size_t zeta_splits_len, void* stream);

/* Timings (milliseconds, HIP events on the work stream) of the last encore_npcf
 * call on this context: [0] total, [1] gather, [2] coupling, [3] reduce/contract,
 * [4] number of gather launches, [5] number of accepted (primary, secondary) pairs.
 * After encore_edge_correct, [0] is the device time of its matrix build and solves
 * and [1..5] are zero.  out_len >= 6. */
int encore_last_timings(const encore_ctx* ctx, double* out, size_t out_len);

#ifdef __cplusplus
}
#endif
#endif /* ENCORE_H */
