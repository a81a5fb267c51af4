// Device-side data structures and kernel launchers of libencore (internal).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace encore {

constexpr int kMaxBins = 16;     // radial bins per call
constexpr int kMaxLmax = 10;     // largest principal ell built
constexpr int kWave = 64;        // CDNA wavefront

// Cell-sorted catalog on the device.  Particles are sorted by cell index
// (cz * ncy + cy) * ncx + cx, so the cells of one (cy, cz) row are contiguous.
struct DevGrid {
    int64_t n = 0;
    double4* P = nullptr;        // sorted (x, y, z, w) in FP64
    int32_t* perm = nullptr;     // sorted index -> input index
    int32_t* inv = nullptr;      // input index -> sorted index
    int32_t* cell_start = nullptr;  // [ncell + 1]
    int ncx = 1, ncy = 1, ncz = 1;
    double ox = 0, oy = 0, oz = 0;  // grid origin
    double csx = 1, csy = 1, csz = 1;  // cell sizes
    int periodic = 0;
    double Lx = 0, Ly = 0, Lz = 0;
    double r_max = 0;
};

// ------------------------------------------------------------------ grid build
int grid_build(DevGrid& g, const double* d_pos, const double* d_w, int64_t n, int64_t n_data,
               bool dmr, bool periodic, const double box[3], double r_max, double cell_size,
               hipStream_t stream, char* errbuf, size_t errlen);
void grid_free(DevGrid& g);
// small utility kernels
int launch_iota(int32_t* out, int64_t n, hipStream_t stream);
// out[k] = inv[idx[k]]; sets *bad if any idx is outside [0, n)
int launch_map_subset(const int64_t* idx, int64_t k, const int32_t* inv, int64_t n, int32_t* out,
                      int* bad, hipStream_t stream);
int launch_fill(double* p, int64_t n, double v, hipStream_t stream);
int launch_to_double(const void* src, int precision, int64_t n, double* dst, hipStream_t stream);
int couple_ptile(int nbins, int nlm, int precision);
// primary splits of the coupling kernels (parallelism across the sum over primaries)
int couple_nsplit(int nk, int nbins, int64_t ntuple, int64_t nB, int64_t nprim);

// ------------------------------------------------------------------ gather
// Harmonic coefficient gather (eq. binned-discrete-alm): for every primary of the
// launch, a~^b_lm over all secondaries, written as complex [nprim][nbins][nlm].
struct GatherArgs {
    const double4* P;
    const int32_t* cell_start;
    int ncx, ncy, ncz;
    double ox, oy, oz, csx, csy, csz;
    int periodic;
    double Lx, Ly, Lz;
    const int32_t* prim;   // sorted indices of the primaries
    int nprim;
    int nbins;
    int ngroups;           // bin groups per primary (work items per primary)
    int group_bins;        // bins per group (last group may have fewer)
    double e2[kMaxBins + 1];  // squared edges
    void* alm;             // output
    const double* kappa;   // [nlm] final scale of the monic recurrence
    const double* gamma;   // [nlm] recurrence coefficients
    unsigned long long* npairs;  // optional: += accepted pairs (null: not counted)
};
// precision: 0 = FP64, 1 = FP32.  Returns hipError_t as int.
int launch_gather(const GatherArgs& a, int lmax, int precision, hipStream_t stream);
// bins per work item the kernel for (lmax, precision) keeps in registers
int gather_group_bins(int lmax, int precision);
// fill kappa/gamma tables for the monic Legendre recurrence used by the gather
void gather_tables(int lmax, double* kappa, double* gamma);

// ------------------------------------------------------------------ coupling
// T[split][t][B] = sum over the split's primaries p of w_p Q_t[prod_k a^{b_k}_{l_k m_k}(p)],
// Q_t = Re or Im; then zeta[L][B] = sum_terms coef * sum_split T.
struct CoupleArgs {
    const void* alm;          // [nprim][nbins][nlm] complex
    const double4* P;         // for the primary weights
    const int32_t* prim;      // sorted indices of the primaries
    int nprim;
    int nbins, nlm, nk;       // nk = N - 1
    int ntuple, nB;
    const int32_t* tuple_off;   // [ntuple][nk] lm index of factor k
    const int32_t* tuple_flags; // [ntuple] bit k: factor k has m < 0; bits 8..12: (-1)^m sign of
                                // factor k negative; bit 16: take Im
    const int32_t* btab;      // [nB][nk]
    int nsplit;
    double* T;                // [nsplit][ntuple][nB]  (accumulated: +=)
};
int launch_couple(const CoupleArgs& a, int precision, hipStream_t stream);

struct ContractArgs {
    const double* T;          // [nsplit][ntuple][nB]
    int nsplit, ntuple, nB, nlam;
    const int32_t* term_start;  // [nlam + 1] CSR over terms sorted by multiplet
    const int32_t* term_tuple;  // [nterm]
    const double* term_coef;    // [nterm]
    const double* bscale;       // [nB] or null
    double* zeta;             // [nlam][nB]
};
int launch_contract(const ContractArgs& a, hipStream_t stream);

}  // namespace encore
