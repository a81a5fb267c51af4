// Host plan of the split-BF16 MFMA coupling (internal; no HIP types, so host
// unit tests can build it with a plain C++ compiler).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace encore {

constexpr int kMfmaMaxEntries = 256;      // coefficients per primary of a K block staged in LDS
constexpr int kMfmaMaxAllEntries = 1056;  // any call: 16 bins x 66 coefficients (lmax 10)
constexpr int kNumMfmaShapes = 4;
constexpr int kMfmaJobWidth = 4;       // row_base, col_base, tile_base, valid row tiles
struct MfmaShape { int RT, NC; };      // row tiles x column tiles of one wave job
extern const MfmaShape kMfmaShapes[kNumMfmaShapes];

// Rows hold KF = N-2 factor entries (bin * nlm + lm index of |m|) and a flags word
// (bit k: factor k has m < 0 and is conjugated, bit 8: the Im part, bit 9: a real
// row, not padding).  Columns hold the entry of the last factor (-1: padding).
// tmap[t * nB + b] is the dense index (tile * 256 + i * 16 + j) of T[t][b], bit 31
// set when the tuple's (-1)^m signs of its conjugated factors multiply to -1.
struct MfmaPlan {
    int K = 0, KF = 0, nlm = 0, nbins = 0, nent = 0;
    std::vector<int32_t> rows;                  // [nrow][KF + 1]
    std::vector<int32_t> cols;                  // [ncol]
    std::vector<int32_t> jobs[kNumMfmaShapes];  // [njob][kMfmaJobWidth]
    int64_t ntiles = 0;
    std::vector<int32_t> tmap;                  // [ntuple * nB]
};
int build_mfma_plan(int N, int lmax, bool allparity, int nbins, MfmaPlan& P);

// Plan of the macro-tiled coupling GEMM.  The K = N-1 factors of a tuple are split
// after the first KL: rows are the products of the first KL factors (their (l, m),
// the Re or Im part, the bins b_1 < .. < b_KL), columns w times the products of
// the other KR = K - KL factors (their (l, m), bins b_KL < b_{KL+1} < .. < b_K).
// Rows and columns are grouped in blocks of fixed (sum of the row factors' m, b_KL):
// a tuple's row and column meet only inside its block.  Each block is cut into
// macro tiles of MR x MC 16 x 16 output tiles, MR + MC <= kGemmMaxOps and at most
// kGemmMaxOps blocks of 2 x 2 output tiles (ceil(MR/2) ceil(MC/2)); one workgroup
// forms a macro tile's MR + MC operand tiles once per 16 primaries and computes all
// its output tiles from them, one 2 x 2 block per wave.  The shape is chosen per
// block: thin blocks (few row tiles) take long macro tiles, so that their row
// operands are formed fewer times.
constexpr int kGemmMaxOps = 16;      // operand tiles of a macro tile (one per wave)
constexpr int kGemmMacroWidth = 5;   // row_start, col_start, row tiles, column tiles, tile_base
struct GemmPlan {
    int K = 0, KL = 0, KR = 0, nlm = 0, nbins = 0, nent = 0;
    bool any_odd = false;
    std::vector<int32_t> rows;     // [nrow][KL + 1]: entries (bin * nlm + lm of |m|), flags
    std::vector<int32_t> cols;     // [ncol][KR + 1]: entries, flags
    std::vector<int32_t> macros;   // [nmacro][kGemmMacroWidth]
    std::vector<int32_t> blocks;   // [nblock][2]: row tiles, column tiles of each block
    int64_t ntiles = 0;
    std::vector<int32_t> tmap;     // [ntuple * nB], as MfmaPlan::tmap
};
// flags of a row or column: bit k = factor k has m < 0 (conjugated), bit 8 = the Im
// part (rows only), bit 9 = a real row or column (not padding)
int build_gemm_plan(int N, int lmax, bool allparity, int nbins, int KL, GemmPlan& P);
// the split used for N (rows from the first KL factors)
int gemm_split(int N);
// macro tile shape (row tiles, column tiles) for a block of nrt x nct output tiles
void gemm_macro_shape(int nrt, int nct, int* mr, int* mc);

int fail(int code, const std::string& msg);

}  // namespace encore
