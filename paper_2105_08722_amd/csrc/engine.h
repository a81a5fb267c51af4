// Host-side execution engine of libencore (internal, not part of the ABI).
//
// An Exec is one HIP stream with its own workspaces; the context owns one for
// the synchronous entry points and the server owns one per lane.  run_slice()
// runs gather -> coupling -> in-order reduction for a list of row chunks that
// may come from several catalogs; contract_job() turns a job's accumulated T
// into zeta.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/encore.h"
#include "device.h"
#include "internal.h"

namespace encore {

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
    // split-BF16 MFMA plan (built on first use)
    bool mf_ready = false;
    int mf_KF = 0, mf_nent = 0;
    int64_t mf_dense = 0;
    int32_t* mf_rows = nullptr;
    int32_t* mf_cols = nullptr;
    int32_t* mf_jobs[kNumMfmaShapes] = {nullptr, nullptr, nullptr, nullptr};
    int mf_njobs[kNumMfmaShapes] = {0, 0, 0, 0};
    int32_t* mf_tmap = nullptr;
    // macro-tiled GEMM plan (used instead of the wave jobs when mf_gemm): mf_rows /
    // mf_cols hold its rows and columns, mf_macros its macro tiles
    bool mf_gemm = false;
    int mf_KL = 0, mf_KR = 0, mf_nmacro = 0;
    bool mf_any_odd = false;
    int32_t* mf_macros = nullptr;
};
// whether the split-BF16 coupling of N runs as the macro-tiled GEMM
bool use_gemm_coupling(int N);


// Fixed device memory handed out front to back (the scratch buffer of the
// allocation-free entry point): nothing in it is allocated or freed.
struct Arena {
    char* base = nullptr;
    size_t size = 0, used = 0;
};
// bytes from the arena (256-byte aligned) or ESIZE
int arena_take(Arena& A, size_t bytes, void** p);

// A grow-only device buffer.  With a pool it is allocated and freed stream-ordered
// on stream s (no device-wide synchronisation when it grows); with an arena it is
// carved from it (growing takes new room; nothing is freed).
struct Buf {
    void* p = nullptr;
    size_t n = 0;
    hipMemPool_t pool = nullptr;
    hipStream_t s = nullptr;
    Arena* arena = nullptr;
};

// One stream and the workspaces of the hot path on it.
struct Exec {
    hipStream_t s = nullptr;
    Buf alm, wprim, T, segs, splits, redp, queues, misc, zeta, bscale, prim, Tjob, almb;
    Buf cache, cmap;   // random splits: the data part of a~ and the row maps
    Buf mesh, meshd;   // gridded data: the coefficient fields and the transform of delta
    Buf meshk;         // gridded data: transforms of the kernel fields (kept between calls)
    Buf egt, eA, eM, eio;   // edge correction: Gaunt table, matrices, matrix copies, small arrays
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
};
// pool: null for plain hipMalloc workspaces, else a stream-ordered pool the
// workspaces come from (on x.s)
int exec_init(Exec& x, hipMemPool_t pool = nullptr);
// every workspace of x carved from A instead (x.s must be set)
void exec_use_arena(Exec& x, Arena* A);
void exec_release(Exec& x);
// bytes held by the workspaces
size_t exec_bytes(const Exec& x);

int fail(int code, const std::string& msg);
int hip_fail(hipError_t e, const char* what);

#define HIPTRY(x)                                                    \
    do {                                                             \
        hipError_t e__ = (x);                                        \
        if (e__ != hipSuccess) return ::encore::hip_fail(e__, #x);   \
    } while (0)

// grow-only device buffer
int ensure(Buf& b, size_t bytes);

bool valid_lmax(int N, int lmax);
int check_edges(const double* edges, int nbins);
int precision_of(uint32_t flags, int* prec);
int check_grid_edges(const DevGrid& g, const double* edges, int nbins);

// Validated call parameters shared by every entry point that computes zeta.
struct NpcfPlan {
    int N = 0, lmax = 0, nbins = 0, prec = 0;
    int nbg = 0;   // gather bins per work item (0: the compiled default)
    bool allparity = false;
    int64_t nlam = 0, nB = 0;
};
int plan_call(int npcf, int lmax, int nbins, const double* edges, uint32_t flags, NpcfPlan* pl);
// Gather variant of a call precision (0 FP64, 1 FP32, 2 split-BF16): 0 FP64
// accumulators, 1 FP32 (split-BF16), 2 FP32 terms in FP64 sums (FP32); see launch_gather.
int gather_precision(int prec);

// per-job accumulator length: ntuple * nB (VALU coupling) or the dense MFMA tiles
int64_t acc_len(const NpcfPlan& pl, const DevTables* tb);
// the same before any device tables exist (host plan, cached)
int acc_len_host(const NpcfPlan& pl, int64_t* out);

// bytes of a~ per primary row
size_t alm_row_bytes(const NpcfPlan& pl);
// rows of a~ held at once (8 GiB of coefficients, at most 2^27 rows;
// ENCORE_MAX_SLICE_ROWS may lower it)
int64_t cap_rows(const NpcfPlan& pl);
// Coupling split length of a job: a function of the job alone, so that a job's
// zeta does not depend on what shares a launch with it.
int64_t job_split_rows(const NpcfPlan& pl, const DevTables* tb, int64_t nprim, int64_t cap);

// Rows [r0, r1) of one job's primary list inside a slice.  r0 is a multiple of
// split_rows; Tdst receives += (in split order) the job's T over those rows.
struct Chunk {
    const DevGrid* g;
    const int32_t* prim;   // device: the job's sorted primary indices
    int64_t r0, r1;
    int64_t split_rows;
    double* Tdst;          // device [ntuple * nB]
    // primaries from another point array (null: the grid's own points; prim then
    // indexes Pq), and cache rows added to the gathered rows (row of primary p +=
    // cache row p; null: none)
    const double4* Pq = nullptr;
    const void* cache = nullptr;
};
// Gather + couple + reduce for the chunks (at most cap_rows rows in total).
// Synchronises x.s before returning; adds the gather / coupling milliseconds.
// x.misc holds the accepted-pair counter (cleared by the caller).
int run_slice(Exec& x, const NpcfPlan& pl, const DevTables* tb, const double* edges,
              const std::vector<Chunk>& chunks, double* ms_gather, double* ms_couple);

// The same in two parts: prepare_slice builds the slice's host tables, copies them
// (asynchronously on x.s) into segs / splits / redp and grows x's workspaces;
// launch_slice_* then only launch kernels (no allocation, no host synchronisation),
// so they can be recorded into a HIP graph.
struct CacheAdd {
    int row0, nrows;
    const int32_t* prim;
    const void* cache;
};
struct SliceLaunch {
    int64_t rows = 0;
    bool persistent = false;
    std::vector<CacheAdd> adds;   // after the gather
    GatherArgs ga;
    CoupleArgs ca;
    MfmaArgs ma;
    ReduceArgs ra;
};
int prepare_slice(Exec& x, Buf& segs, Buf& splits, Buf& redp, const NpcfPlan& pl, const DevTables* tb,
                  const double* edges, const std::vector<Chunk>& chunks, SliceLaunch& L);
int launch_slice_gather(const SliceLaunch& L, const NpcfPlan& pl, hipStream_t s);
int launch_slice_couple(const SliceLaunch& L, const NpcfPlan& pl, const DevTables* tb, hipStream_t s);
// zeta[nlam][nB] (device) from a job's T (device); bscale[nB] (device) or null.
int contract_job(Exec& x, const NpcfPlan& pl, const DevTables* tb, const double* T,
                 const double* bscale, double* zeta);
// 1 / (V prod_k shell volume) per bin tuple (normalisation of eq. 2.7's estimator)
std::vector<double> bin_scale(const NpcfPlan& pl, const double* edges, double V);

// Cell grid of a catalog already on the device (pos [n][3], w [n]).
// cell sides r_max / div (y, z) and r_max / (div * xsub) (x)
// (pool: see grid_build)
int build_grid_dev(int device, const double* d_pos, const double* d_w, int64_t n, int64_t n_data,
                   bool dmr, const double* box, double r_max, double div, double xsub, hipStream_t s,
                   DevGrid& out, hipMemPool_t pool = nullptr);
// cell shape: ENCORE_CELL_DIVISOR / ENCORE_CELL_XSUB, else the tuned value (> 0),
// else the default
double cell_divisor(double tuned = 0.0);
double cell_x_subdiv(double tuned = 0.0);   // x cell side = yz side / this

}  // namespace encore

struct encore_ctx {
    int device = 0;
    encore::Exec main;
    // autotuned launch shapes (encore_autotune); guarded by tab_mu
    double cell_div = 0.0, cell_xsub = 0.0;               // 0: defaults
    std::map<std::tuple<int, int, int>, int> tuned_nbg;  // (lmax, gather precision, nbins) -> bins per item
    std::map<std::tuple<int, int, bool, int>, encore::DevTables> tables;
    std::mutex tab_mu;   // tables
    std::mutex mu;       // main exec, timings
    double timings[6] = {0, 0, 0, 0, 0, 0};
    // gridded data: (nmesh, box, lmax, nbins, edges) whose kernel-field transforms
    // main.meshk holds; empty when it holds none (guarded by mu)
    std::vector<double> mesh_key;
    // gridded data: the transform plans (hipfftHandle) of the last (nmesh, number of
    // fields), with their work areas, kept for later calls (guarded by mu; freed by
    // mesh_release): a batch of mesh_plan_nf fields and a single field
    void* mesh_plan = nullptr;
    void* mesh_plan1 = nullptr;
    int mesh_plan_n = 0, mesh_plan_nf = 0;
    // edge correction: (npcf, lmax, all parities) of the Gaunt table held in
    // main.egt; (-1, ...) when it holds none (guarded by mu)
    std::tuple<int, int, bool> edge_gt_key{-1, -1, false};
    std::atomic<int> live_grids{0};
};

struct encore_grid {
    encore_ctx* ctx = nullptr;
    encore::DevGrid g;
    std::atomic<int> plans{0};   // live encore_plan objects on this grid
    // random-split co-adding: the grid of this D-R catalog's randoms alone (with
    // their D-R weights), built on first use and freed with this grid
    mutable encore_grid* rand_only = nullptr;
};

namespace encore {
// Looks up, once per device (the device current), the address of that device's
// copy of the scratch array of encore_npcf_noalloc.
int noalloc_init(int device);
size_t noalloc_scratch_bytes();

// Primaries of one job as cell-sorted indices at dst (device, room for the count):
// every point (subset NULL) or the subset given in input order (validated; uses
// x.misc).  *np: the count.
int fill_primaries(Exec& x, const encore_grid* grid, const int64_t* subset, int64_t k, int32_t* dst,
                   int64_t* np);

// One job's rows for run_jobs.
struct JobRows {
    const encore_grid* grid;
    const int32_t* prim;   // device
    int64_t nprim;
    const double4* Pq = nullptr;   // random-split jobs (see Chunk)
    const void* cache = nullptr;
};

// The hot path over several jobs on exec x with tables tb (the caller holds
// ctx->mu): slices of at most cap rows, cut only at each job's split boundaries,
// then one contraction per job; zeta [njobs][nlam][nB] to the host; the
// context's timings are set.
int run_jobs(encore_ctx* ctx, Exec& x, const DevTables* tb, int64_t cap, const std::vector<JobRows>& jobs,
             const NpcfPlan& pl, uint32_t flags, const double* edges, double volume, double* zeta);

// tuned bins per work item for a call (0: default); thread-safe
int ctx_nbg(encore_ctx* ctx, const NpcfPlan& pl);
// destroy the context's gridded-data transform plans
void mesh_release(encore_ctx* ctx);
void ctx_cells(encore_ctx* ctx, double* div, double* xsub);
// thread-safe; the returned tables live as long as the context
int get_tables(encore_ctx* ctx, int N, int lmax, bool allparity, int nbins, DevTables** out);
// tables of the call's precision (the MFMA plan too for split-BF16)
int get_tables_for(encore_ctx* ctx, const NpcfPlan& pl, DevTables** out);
// the same tables carved from an arena and copied on stream s (waits for the copies)
int tables_in_arena(Arena& A, hipStream_t s, const NpcfPlan& pl, DevTables& d);
}  // namespace encore
