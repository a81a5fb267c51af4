// Device-side data structures and kernel launchers of libencore (internal).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <vector>

#include "mfma_plan.h"

namespace encore {

constexpr int kMaxBins = 16;     // radial bins per call
constexpr int kMaxLmax = 10;     // largest principal ell built
constexpr int kWave = 64;        // CDNA wavefront
// NaN records after a grid's points: the gather maps candidate positions up to
// 2 * kWave - 1 past a batch's last candidate onto distinct sentinels, which no
// bin accepts
constexpr int kSentinels = 2 * kWave;
// largest catalog of one grid: the gather packs a point index (sentinels
// included) and a 6-bit image code into 32 bits
constexpr int64_t kMaxGridPoints = (int64_t(1) << 26) - kSentinels;

// Cell-sorted catalog on the device.  Particles are sorted by cell index
// (cz * ncy + cy) * ncx + cx, so the cells of one (cy, cz) row are contiguous.
struct DevGrid {
    int64_t n = 0;
    double4* P = nullptr;        // sorted (x, y, z, w) in FP64; P[n .. n+kSentinels) are NaN
    int32_t* perm = nullptr;     // sorted index -> input index
    int32_t* inv = nullptr;      // input index -> sorted index
    int32_t* cell_start = nullptr;  // [ncell + 1]
    int ncx = 1, ncy = 1, ncz = 1;
    double ox = 0, oy = 0, oz = 0;  // grid origin
    double csx = 1, csy = 1, csz = 1;  // cell sizes
    int periodic = 0;
    double Lx = 0, Ly = 0, Lz = 0;
    double r_max = 0;
    int64_t n_data = 0;   // with dmr: input points [0, n_data) are data
    int dmr = 0;          // built as a data-minus-randoms catalog
    hipMemPool_t pool = nullptr;   // arrays from this stream-ordered pool (null: hipMalloc)
};

// Device memory from a stream-ordered pool on stream s (no device-wide
// synchronisation, unlike hipMalloc/hipFree), or plain hipMalloc/hipFree when
// pool is null.
hipError_t dev_alloc(void** p, size_t bytes, hipMemPool_t pool, hipStream_t s);
void dev_free(void* p, hipMemPool_t pool, hipStream_t s);

// ------------------------------------------------------------------ grid build
// With a pool, every array of the grid and every temporary comes from it on
// `stream`; grid_free must then be given a stream ordered after the grid's last use.
int grid_build(DevGrid& g, const double* d_pos, const double* d_w, int64_t n, int64_t n_data,
               bool dmr, bool periodic, const double box[3], double r_max, double cell_size,
               double cell_size_x,
               hipStream_t stream, char* errbuf, size_t errlen, hipMemPool_t pool = nullptr);
void grid_free(DevGrid& g, hipStream_t s = nullptr);
// small utility kernels
int launch_iota(int32_t* out, int64_t n, hipStream_t stream);
// out[k] = inv[idx[k]]; sets *bad if any idx is outside [0, n)
int launch_map_subset(const int64_t* idx, int64_t k, const int32_t* inv, int64_t n, int32_t* out,
                      int* bad, hipStream_t stream);
int launch_fill(double* p, int64_t n, double v, hipStream_t stream);
int launch_fill_u32(unsigned* p, int64_t n, unsigned v, hipStream_t stream);
int launch_to_double(const void* src, int precision, int64_t n, double* dst, hipStream_t stream);
// Random-split catalog S (data + one random part, built with dmr) against the
// data-only grid D: *bad = 1 if a data point of S differs from D's (position or
// weight, same input index).
int launch_split_check(const DevGrid& S, const DevGrid& D, int* bad, hipStream_t stream);
// The random points of S (input order) as arrays pos [n - n_data][3], w (S's
// data-minus-randoms weights).
int launch_split_randoms(const DevGrid& S, double* pos, double* w, hipStream_t stream);

// ------------------------------------------------------------------ gather
// Harmonic coefficient gather (eq. binned-discrete-alm).  A launch covers a
// "slice" of primaries that may come from several catalogs (jobs): segment s
// holds nprim consecutive slice rows starting at row0, all from one catalog.
// Work item = (slice row, bin group); rows are written as complex
// alm[row][nbins][nlm] plus the primary's weight wprim[row].
struct GatherSeg {
    const double4* P;      // secondaries (cell-sorted, n points + kSentinels NaN records)
    const int32_t* cell_start;
    const double4* Pq;     // primary records (P, or another grid's points)
    const int32_t* prim;   // indices into Pq of this segment's primaries
    int ncx, ncy, ncz, periodic;
    double ox, oy, oz, csx, csy, csz;
    double Lx, Ly, Lz;
    int row0, nprim;
    int nP, pad_;          // points of P (index of the first sentinel)
    // derived by finish_seg: reciprocal cell sizes, the pad of the culling radius
    // and the FP32 row set-up margin (both in length units)
    double icsx, icsy, icsz, cull_pad, frame_eps;
};
inline void finish_seg(GatherSeg& s)
{
    s.icsx = 1.0 / s.csx;
    s.icsy = 1.0 / s.csy;
    s.icsz = 1.0 / s.csz;
    const double cmin = s.csx < s.csy ? (s.csx < s.csz ? s.csx : s.csz) : (s.csy < s.csz ? s.csy : s.csz);
    const int nmax = s.ncx > s.ncy ? (s.ncx > s.ncz ? s.ncx : s.ncz) : (s.ncy > s.ncz ? s.ncy : s.ncz);
    s.cull_pad = 1e-7 * cmin;
    // FP32 rounding of coordinates relative to the grid origin is about
    // nmax * 2^-23 cells; the margin is far above it
    const double margin = 1e-6 * nmax > 1e-3 ? 1e-6 * nmax : 1e-3;
    s.frame_eps = margin * cmin;
}
struct GatherArgs {
    const GatherSeg* segs;   // device array
    int nseg;
    int nrows;               // slice rows (sum of segment nprim)
    int nbins;
    int ngroups;             // bin groups per primary (work items per primary)
    int group_bins;          // bins per group (last group may have fewer)
    double e2[kMaxBins + 1]; // squared edges
    double e1[kMaxBins + 1]; // edges
    void* alm;               // output rows
    double* wprim;           // output: weight of each row's primary
    const double* kappa;     // [nlm] final scale of the monic recurrence
    unsigned long long* npairs;  // optional: += accepted pairs (null: not counted)
    // persistent mode (queues != null): waves pull items from 8 queues (one per
    // XCD, contiguous item ranges) and steal from the others when theirs is empty
    unsigned* queues;        // [8] counters, zero at launch
};
// precision: 0 = FP64, 1 = FP32.  nbg: bins per work item (0 or a value without
// a compiled variant: the default).  persistent: grid sized to the resident waves.
int launch_gather(const GatherArgs& a, int lmax, int precision, int nbg, bool persistent, hipStream_t stream);
// alm row row0 + r += cache row prim[r], r < nrows (rows of row_cplx complex
// values; precision 0: FP64, else FP32)
int launch_add_cached(void* alm, int precision, int row0, int nrows, const int32_t* prim, const void* cache,
                      int row_cplx, hipStream_t stream);
int gather_group_bins(int lmax, int precision, int nbg);
// compiled bins-per-item values for (lmax, precision), the default first
std::vector<int> gather_nbg_options(int lmax, int precision);
void gather_tables(int lmax, double* kappa);

// ------------------------------------------------------------------ coupling
// For every split y: T[y][t][B] = sum over rows p in [split_lo[y], split_hi[y]) of
// w_p Q_t[prod_k a~^{b_k}_{l_k m_k}(p)], Q_t = Re or Im (written, not accumulated).
struct CoupleArgs {
    const void* alm;          // [nrows][nbins][nlm] complex
    const double* wprim;      // [nrows]
    int nbins, nlm, nk;       // nk = N - 1
    int ntuple, nB;
    const int32_t* tuple_off;   // [ntuple][nk] lm index of factor k
    const int32_t* tuple_flags; // [ntuple] bit k: factor k has m < 0 (conjugate); bit 8:
                                // overall (-1)^m sign negative; bit 16: take Im
    const int32_t* btab;      // [nB][nk]
    int nsplit;
    const int32_t* split_lo;  // [nsplit]
    const int32_t* split_hi;  // [nsplit]
    double* T;                // [nsplit][ntuple][nB]
};
int launch_couple(const CoupleArgs& a, int precision, hipStream_t stream);

// Split-BF16 MFMA coupling (couple_mfma.hip): per split y, D[y][tile][16][16] of
// the wave jobs of one shape (RT row tiles x NC column tiles per wave).
// Blocked layout of the FP32 coefficients read by the MFMA coupling: rows in
// blocks of kBlkRows; a block holds, for each entry e < ent_blk, the 16 rows'
// complex values (16 float2) and 16 bytes of padding, so an entry spans 144 bytes
// (16-byte LDS reads of 16 different entries then spread over the banks).  The
// padding of entries 0..3 holds the rows' weights as FP32 (row r: entry r / 4,
// float r % 4).  A block is copied to LDS as it is.
constexpr int kBlkRows = 16;
constexpr int kBlkEntFloats = 36;
inline int blk_entries(int nent) { return nent < 4 ? 4 : nent; }
inline size_t blk_bytes(int nent) { return (size_t)blk_entries(nent) * kBlkEntFloats * 4; }

struct MfmaArgs {
    const float* alm;         // blocked coefficients and weights of the slice rows
    int ent_blk;              // entries per block (blk_entries(nent))
    int nent;
    const int32_t* rows;      // [.][KF + 1]: factor entries, flags
    const int32_t* cols;      // [.]: entry of the last factor (-1: padding)
    const int32_t* jobs;      // [njobs][kMfmaJobWidth] of this shape
    int njobs;
    int nsplit;
    const int32_t* split_lo;  // [nsplit]
    const int32_t* split_hi;  // [nsplit]
    double* D;                // [nsplit][dense]
    int64_t dense;            // ntiles * 256
    int any_odd;              // some rows take the Im part (all-parity multiplets)
};
int launch_couple_mfma(const MfmaArgs& a, int KF, int shape, hipStream_t stream);
// The macro-tiled GEMM of a GemmPlan (mfma_plan.h): rows / cols hold the plan's rows
// and columns, jobs its macro tiles (njobs of them), KL + KR factors.
int launch_couple_gemm(const MfmaArgs& a, int KL, int KR, hipStream_t stream);

// Edge correction (one workgroup per bin tuple B): builds the coupling matrix from
// the Gaunt terms and the random multiplets, solves for zeta (NaN for B with R_0 = 0
// or a singular matrix, counted in *nbad).
// Largest multiplet count of the edge-correction solve (its factor column sits in LDS).
constexpr int kEdgeMaxMultiplets = 4096;
struct EdgeArgs {
    int nlam, nB, nout;
    const double* nmult;        // [nlam][nB] data-minus-random multiplets
    const double* rmult;        // [nlam][nB] random multiplets (row 0: L = 0)
    const int64_t* row_start;   // [nlam * nlam + 1] terms of entry (L, L'')
    const int32_t* term_lp;     // L'
    const double* term_val;     // E(L'') G^{L L' L''}
    double* A;                  // workspace [nB][nlam][nlam]
    double* rhs;                // workspace [nB][nlam]
    const int32_t* keep;        // [nout] output multiplets (indices into the list)
    double* zeta;               // [nout][nB]
    double* M_out;              // optional [nB][nlam][nlam], M[L][L'']
    unsigned* nbad;             // += number of B without a solution
};
int launch_edge(const EdgeArgs& a, hipStream_t stream);
// Row-major FP32 coefficients ([nrows][nent] complex) and weights -> blocked layout
// (out: ceil(nrows / 16) blocks); rows outside every segment's [row0, row0 + nprim)
// and past nrows become zero with weight zero.
int launch_to_blocked(const float2* alm, const double* wprim, const GatherSeg* segs, int nseg, int nrows,
                      int nent, float* out, hipStream_t stream);
// rows per split that keep the coupling kernels' blocks busy
int couple_split_rows(int nk, int nbins, int64_t ntuple, int64_t nB, int64_t nrows);
int couple_ptile(int nbins, int nlm, int precision);

// dst[r][..] += sum over splits y in [red_lo[r], red_hi[r]) of T[y][..], left to
// right starting from the current dst[r] (one entry per job and slice).
struct ReduceArgs {
    const double* T;          // [nsplit][ntuple * nB]
    int64_t per;              // ntuple * nB
    int nred;
    const int32_t* red_lo;
    const int32_t* red_hi;
    double* const* dst;       // [nred] device pointers, each [per]
};
int launch_reduce(const ReduceArgs& a, hipStream_t stream);

struct ContractArgs {
    const double* T;          // [nsplit][ntuple][nB]
    int nsplit, ntuple, nB, nlam;
    const int32_t* term_start;  // [nlam + 1] CSR over terms sorted by multiplet
    const int32_t* term_tuple;  // [nterm]
    const double* term_coef;    // [nterm]
    const double* bscale;       // [nB] or null
    const int32_t* tmap;        // null, or [ntuple][nB]: index into T (bit 31: negate); nsplit must be 1
    double* zeta;             // [nlam][nB]
};
int launch_contract(const ContractArgs& a, hipStream_t stream);

}  // namespace encore
