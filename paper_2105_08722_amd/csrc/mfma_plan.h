// Host plan of the split-BF16 MFMA coupling (internal; no HIP types, so host
// unit tests can build it with a plain C++ compiler).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace encore {

constexpr int kMfmaMaxEntries = 256;   // nbins * (lmax+1)(lmax+2)/2 staged per primary
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

int fail(int code, const std::string& msg);

}  // namespace encore
