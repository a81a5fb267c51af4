// Host plan of the split-BF16 MFMA coupling (the reassociated contraction of eq.
// NPCF-mult-discrete-binned-estimator, Appendix B half sum), N = 3..6.
//
// The accumulated tensor T[t][B] = sum_i w_i Q_t[prod_k a~^{b_k}_{l_k m_k}(i)] is
// computed as a set of real GEMMs over K = (primary, re/im):
//
//   rows    (rho, q, b_1 .. b_{K-1}): the product P = prod_{k<K} a~ of the first
//           K-1 factors of a tuple (rho = their (l_k, m_k)), q = Re or Im part;
//   columns (l_K, b_K) of the last factor at fixed m_K = mu >= 0;
//   A[row][(i, c)] = (Re P, -Im P) for q = Re, (Im P, Re P) for q = Im;
//   B[(i, c)][col] = (Re, Im)(w_i a~^{b_K}_{l_K mu}(i)),
//
// so that sum_K A B = sum_i w_i Q[P a~].  Rows and columns are grouped in blocks
// of fixed (mu, beta = b_{K-1}); a block's columns are the bins b_K > beta, so
// every computed entry has strictly increasing bins.  The blocks are cut into
// 16 x 16 output tiles; one wave owns up to four tiles of one block (a "wave
// job") and forms each of its row operands once per primary.
#include "mfma_plan.h"

#include "../../include/encore.h"
#include "internal.h"

#include <algorithm>
#include <cstdlib>
#include <map>
#include <vector>

namespace encore {

namespace {

int lm_of(int l, int m) { return l * (l + 1) / 2 + m; }

// combinations of size k from [0, n), lexicographic
std::vector<std::vector<int>> combos(int n, int k)
{
    std::vector<std::vector<int>> out;
    if (k < 0 || k > n) return out;
    std::vector<int> c(k);
    for (int i = 0; i < k; ++i) c[i] = i;
    while (true) {
        out.push_back(c);
        int i = k - 1;
        while (i >= 0 && c[i] == n - k + i) --i;
        if (i < 0) break;
        ++c[i];
        for (int j = i + 1; j < k; ++j) c[j] = c[j - 1] + 1;
    }
    return out;
}

}  // namespace

const MfmaShape kMfmaShapes[kNumMfmaShapes] = {{4, 1}, {2, 2}, {1, 3}, {1, 4}};

int build_mfma_plan(int N, int lmax, bool allparity, int nbins, MfmaPlan& P)
{
    const TermTable& tt = term_table(N, lmax, allparity);
    const int K = N - 1, KF = K - 1;
    const int nlm = (lmax + 1) * (lmax + 2) / 2;
    P = MfmaPlan();
    P.K = K; P.KF = KF; P.nlm = nlm; P.nbins = nbins; P.nent = nbins * nlm;

    // row keys (rho, q) and column ells per mu
    std::map<int, std::map<std::vector<int>, int>> rowkeys;   // mu -> key -> index
    std::map<int, std::map<int, int>> colells;                // mu -> l_K -> index
    for (int64_t t = 0; t < tt.ntuple; ++t) {
        const int mu = tt.tuple_m[t * K + K - 1];
        std::vector<int> key;
        for (int k = 0; k < KF; ++k) {
            key.push_back(tt.tuple_l[t * K + k]);
            key.push_back(tt.tuple_m[t * K + k]);
        }
        key.push_back(tt.tuple_odd[t]);
        auto& rk = rowkeys[mu];
        if (!rk.count(key)) { const int id = (int)rk.size(); rk[key] = id; }
        auto& ce = colells[mu];
        const int lK = tt.tuple_l[t * K + K - 1];
        if (!ce.count(lK)) { const int id = (int)ce.size(); ce[lK] = id; }
    }
    // index of a prefix bin tuple (b_1 .. b_{K-2}) among those below beta
    struct BlockInfo {
        int64_t row0 = 0;     // first row in P.rows
        int nrow = 0;
        std::vector<int64_t> cg_job0;   // per column group: first wave job (global list order)
        std::vector<int> cg_shape, cg_nct;
        std::map<std::vector<int>, int> pre_index;
        int nrho = 0, nell = 0;
    };
    std::map<std::pair<int, int>, BlockInfo> blocks;
    const int W = KF + 1;
    std::vector<std::vector<int32_t>> shape_jobs(kNumMfmaShapes);
    struct JobRef { int shape; int64_t idx; };
    std::vector<JobRef> joblist;
    int64_t ntiles = 0;

    for (auto& kv : rowkeys) {
        const int mu = kv.first;
        // Row keys ordered by the factor that takes bin beta (the last row factor),
        // then the rest: consecutive rows of a tile then share that factor, whose
        // LDS read is a broadcast.  The key index is the row key's position here.
        std::vector<const std::vector<int>*> keys;
        for (auto& e : kv.second) keys.push_back(&e.first);
        std::stable_sort(keys.begin(), keys.end(), [&](const std::vector<int>* x, const std::vector<int>* y) {
            const int o = 2 * (KF - 1);
            if ((*x)[o] != (*y)[o]) return (*x)[o] < (*y)[o];
            if ((*x)[o + 1] != (*y)[o + 1]) return (*x)[o + 1] < (*y)[o + 1];
            return *x < *y;
        });
        for (size_t i = 0; i < keys.size(); ++i) kv.second[*keys[i]] = (int)i;
        std::vector<int> ells(colells[mu].size());
        for (auto& e : colells[mu]) ells[e.second] = e.first;
        for (int beta = K - 2; beta <= nbins - 2; ++beta) {
            const std::vector<std::vector<int>> pres = combos(beta, K - 2);
            const int nrow = (int)(pres.size() * keys.size());
            const int ncol = (int)(ells.size() * (nbins - 1 - beta));
            if (nrow == 0 || ncol == 0) continue;
            BlockInfo bi;
            bi.nrho = (int)keys.size();
            bi.nell = (int)ells.size();
            for (size_t p = 0; p < pres.size(); ++p) bi.pre_index[pres[p]] = (int)p;
            bi.row0 = (int64_t)P.rows.size() / W;
            bi.nrow = nrow;
            // rows: (rho, q) outer, prefix bins inner; padded to a multiple of 64
            for (const auto* key : keys)
                for (const auto& pre : pres) {
                    int flags = 1 << 9;   // valid
                    for (int k = 0; k < KF; ++k) {
                        const int l = (*key)[2 * k], m = (*key)[2 * k + 1];
                        const int bin = (k < KF - 1) ? pre[k] : beta;
                        P.rows.push_back(bin * nlm + lm_of(l, std::abs(m)));
                        if (m < 0) flags |= 1 << k;
                    }
                    if ((*key)[2 * KF]) flags |= 1 << 8;
                    P.rows.push_back(flags);
                }
            const int nrow_pad = (nrow + 63) / 64 * 64;
            for (int r = nrow; r < nrow_pad; ++r)
                for (int c = 0; c < W; ++c) P.rows.push_back(0);   // flags 0: invalid
            // columns: b_K outer, l_K inner, cut into groups of at most 4 tiles
            std::vector<int32_t> cvals;
            for (int bK = beta + 1; bK < nbins; ++bK)
                for (int l : ells) cvals.push_back(bK * nlm + lm_of(l, mu));
            const int nct_all = (ncol + 15) / 16;
            const int nrt = (nrow + 15) / 16;
            for (int cg = 0; cg * 4 < nct_all; ++cg) {
                const int nct = std::min(4, nct_all - cg * 4);
                const int shape = nct - 1;   // {4,1} {2,2} {1,3} {1,4}
                const int RT = kMfmaShapes[shape].RT;
                const int64_t col_base = (int64_t)P.cols.size();
                for (int c = 0; c < 16 * nct; ++c) {
                    const int ci = cg * 64 + c;
                    P.cols.push_back(ci < ncol ? cvals[ci] : -1);
                }
                bi.cg_job0.push_back((int64_t)joblist.size());
                bi.cg_shape.push_back(shape);
                bi.cg_nct.push_back(nct);
                for (int rt0 = 0; rt0 < nrt; rt0 += RT) {
                    auto& js = shape_jobs[shape];
                    const int64_t idx = (int64_t)js.size() / kMfmaJobWidth;
                    js.push_back((int32_t)(bi.row0 + rt0 * 16));
                    js.push_back((int32_t)col_base);
                    js.push_back((int32_t)ntiles);
                    js.push_back(std::min(RT, nrt - rt0));
                    joblist.push_back(JobRef{shape, idx});
                    ntiles += (int64_t)RT * nct;
                }
            }
            blocks[{mu, beta}] = std::move(bi);
        }
    }
    if ((int64_t)P.rows.size() / W > INT32_MAX || ntiles * 256 > INT32_MAX)
        return fail(ENCORE_EUNSUPPORTED, "split-bf16 coupling plan too large for this (N, lmax, nbins)");
    P.ntiles = ntiles;
    for (int s = 0; s < kNumMfmaShapes; ++s) P.jobs[s] = std::move(shape_jobs[s]);

    // map (t, B) -> dense index, sign bit 31 = (-1)^(sum of |m| over factors with m < 0)
    const std::vector<int32_t> bt = enumerate_bin_tuples(N, nbins);
    const int64_t nB = (int64_t)bt.size() / K;
    P.tmap.assign((size_t)(tt.ntuple * nB), 0);
    for (int64_t t = 0; t < tt.ntuple; ++t) {
        const int mu = tt.tuple_m[t * K + K - 1];
        std::vector<int> key;
        int neg = 0;
        for (int k = 0; k < KF; ++k) {
            const int m = tt.tuple_m[t * K + k];
            key.push_back(tt.tuple_l[t * K + k]);
            key.push_back(m);
            if (m < 0 && (std::abs(m) & 1)) neg ^= 1;
        }
        key.push_back(tt.tuple_odd[t]);
        const int rho = rowkeys[mu][key];
        const int lidx = colells[mu][tt.tuple_l[t * K + K - 1]];
        for (int64_t b = 0; b < nB; ++b) {
            const int32_t* B = &bt[b * K];
            const int beta = B[K - 2], bK = B[K - 1];
            const BlockInfo& bi = blocks.at({mu, beta});
            const std::vector<int> pre(B, B + K - 2);
            const int row = rho * (int)bi.pre_index.size() + bi.pre_index.at(pre);
            const int col = (bK - beta - 1) * bi.nell + lidx;
            const int cg = col / 64, cc = col % 64;
            const int shape = bi.cg_shape[cg];
            const int RT = kMfmaShapes[shape].RT, nct = bi.cg_nct[cg];
            const int rtg = row / 16;
            const JobRef jr = joblist[bi.cg_job0[cg] + rtg / RT];
            const int32_t* job = &P.jobs[jr.shape][jr.idx * kMfmaJobWidth];
            const int64_t tile = job[2] + (int64_t)(rtg % RT) * nct + cc / 16;
            const int64_t dense = tile * 256 + (row % 16) * 16 + (cc % 16);
            P.tmap[(size_t)(t * nB + b)] = (int32_t)dense | (neg ? (int32_t)0x80000000 : 0);
        }
    }
    return ENCORE_OK;
}

int gemm_split(int N) { return N == 3 ? 1 : (N == 6 ? 3 : 2); }

// Cost of one K block of an MR x MC macro tile in CU cycles, a model of the
// kernel: each operand tile takes ~376 SIMD cycles of VALU to form (products,
// weights, bf16 hi + lo split), spread over the 4 SIMDs; the CU's LDS moves 128
// bytes per cycle: ~8 KiB per formed operand (factor reads, hi + lo writes), 2 KiB
// per operand tile each wave reads for its 2 x 2 output tiles, and the K block's
// copy; each output tile takes three 16-cycle MFMAs.  The LDS and the VALU bound
// it, partly overlapped; ~300 more for the barrier.
static double macro_cost(int MR, int MC)
{
    const int ops = MR + MC;
    double reads = 0.0;                          // operand tiles read, summed over the waves
    for (int bi = 0; bi < (MR + 1) / 2; ++bi)
        for (int bj = 0; bj < (MC + 1) / 2; ++bj)
            reads += std::min(2, MR - 2 * bi) + std::min(2, MC - 2 * bj);
    const double valu = 376.0 * ((ops + 3) / 4);
    const double lds = (8.0 * ops + 2.0 * reads + 16.0) * 1024.0 / 128.0;
    const double mfma = 48.0 * ((MR * MC + 3) / 4);
    return std::max({valu, lds, mfma}) + 0.25 * std::min(valu, lds) + 300.0;
}

void gemm_macro_shape(int nrt, int nct, int* mr, int* mc)
{
    double best = 0.0;
    *mr = *mc = 1;
    for (int r = 1; r <= std::min(nrt, kGemmMaxOps - 1); ++r) {
        // the widest c with r + c operand tiles and ceil(r/2) ceil(c/2) 2 x 2 output
        // blocks (one per wave) within the kernel's 16 waves
        int c = kGemmMaxOps - r;
        while (c > 1 && ((r + 1) / 2) * ((c + 1) / 2) > kGemmMaxOps) --c;
        const int nr = (nrt + r - 1) / r, nc = (nct + c - 1) / c;
        double cost = 0.0;
        for (int i = 0; i < nr; ++i)
            for (int j = 0; j < nc; ++j) cost += macro_cost(std::min(r, nrt - i * r), std::min(c, nct - j * c));
        if (r == 1 || cost < best) {
            best = cost;
            *mr = r;
            *mc = c;
        }
    }
}

int build_gemm_plan(int N, int lmax, bool allparity, int nbins, int KL, GemmPlan& P)
{
    const TermTable& tt = term_table(N, lmax, allparity);
    const int K = N - 1;
    if (KL < 1 || KL >= K) return fail(ENCORE_EINVAL, "gemm split out of range");
    const int KR = K - KL;
    const int nlm = (lmax + 1) * (lmax + 2) / 2;
    P = GemmPlan();
    P.K = K; P.KL = KL; P.KR = KR; P.nlm = nlm; P.nbins = nbins; P.nent = nbins * nlm;

    // row keys (l, m of the first KL factors, Im part) and column keys (l, m of the
    // rest) by the m-sum s of the row factors
    std::map<int, std::map<std::vector<int>, int>> rkeys, ckeys;
    auto rkey = [&](int64_t t) {
        std::vector<int> k;
        for (int f = 0; f < KL; ++f) { k.push_back(tt.tuple_l[t * K + f]); k.push_back(tt.tuple_m[t * K + f]); }
        k.push_back(tt.tuple_odd[t]);
        return k;
    };
    auto ckey = [&](int64_t t) {
        std::vector<int> k;
        for (int f = KL; f < K; ++f) { k.push_back(tt.tuple_l[t * K + f]); k.push_back(tt.tuple_m[t * K + f]); }
        return k;
    };
    auto msum = [&](int64_t t) {
        int s = 0;
        for (int f = 0; f < KL; ++f) s += tt.tuple_m[t * K + f];
        return s;
    };
    for (int64_t t = 0; t < tt.ntuple; ++t) {
        rkeys[msum(t)][rkey(t)] = 0;
        ckeys[msum(t)][ckey(t)] = 0;
        if (tt.tuple_odd[t]) P.any_odd = true;
    }
    for (auto& kv : rkeys) { int i = 0; for (auto& e : kv.second) e.second = i++; }
    for (auto& kv : ckeys) { int i = 0; for (auto& e : kv.second) e.second = i++; }

    struct Block {
        int64_t row0 = 0, col0 = 0;   // first row / column (multiples of 16)
        int nrho = 0, nsig = 0;
        std::map<std::vector<int>, int> pre, suf;   // prefix / suffix bin tuples -> index
        int64_t macro0 = 0;   // first macro tile
        int mr = 0, mc = 0;   // macro tile shape (row tiles, column tiles)
        int nmc = 0;          // macro tiles along the columns
    };
    std::map<std::pair<int, int>, Block> blocks;
    const int RW = KL + 1, CW = KR + 1;
    int64_t ntiles = 0;
    for (auto& kv : rkeys) {
        const int s = kv.first;
        if (!ckeys.count(s)) continue;
        const auto& rk = kv.second;
        const auto& ck = ckeys[s];
        for (int beta = KL - 1; beta <= nbins - 1 - KR; ++beta) {
            const std::vector<std::vector<int>> pres = combos(beta, KL - 1);
            std::vector<std::vector<int>> sufs = combos(nbins - 1 - beta, KR);
            for (auto& x : sufs)
                for (int& b : x) b += beta + 1;
            const int64_t nrow = (int64_t)pres.size() * rk.size();
            const int64_t ncol = (int64_t)sufs.size() * ck.size();
            if (nrow == 0 || ncol == 0) continue;
            Block B;
            B.nrho = (int)rk.size();
            B.nsig = (int)ck.size();
            for (size_t i = 0; i < pres.size(); ++i) B.pre[pres[i]] = (int)i;
            for (size_t i = 0; i < sufs.size(); ++i) B.suf[sufs[i]] = (int)i;
            B.row0 = (int64_t)P.rows.size() / RW;
            B.col0 = (int64_t)P.cols.size() / CW;
            // rows: key outer, prefix bins inner; padded to a multiple of 16
            for (const auto& e : rk)
                for (const auto& pre : pres) {
                    int flags = 1 << 9;
                    for (int f = 0; f < KL; ++f) {
                        const int l = e.first[2 * f], m = e.first[2 * f + 1];
                        const int bin = f < KL - 1 ? pre[f] : beta;
                        P.rows.push_back(bin * nlm + lm_of(l, std::abs(m)));
                        if (m < 0) flags |= 1 << f;
                    }
                    if (e.first[2 * KL]) flags |= 1 << 8;
                    P.rows.push_back(flags);
                }
            for (int64_t r = nrow; r % 16; ++r)
                for (int c = 0; c < RW; ++c) P.rows.push_back(0);
            // columns: key outer, suffix bins inner
            for (const auto& e : ck)
                for (const auto& suf : sufs) {
                    int flags = 1 << 9;
                    for (int f = 0; f < KR; ++f) {
                        const int l = e.first[2 * f], m = e.first[2 * f + 1];
                        P.cols.push_back(suf[f] * nlm + lm_of(l, std::abs(m)));
                        if (m < 0) flags |= 1 << f;
                    }
                    P.cols.push_back(flags);
                }
            for (int64_t c = ncol; c % 16; ++c)
                for (int k = 0; k < CW; ++k) P.cols.push_back(0);
            const int nrt = (int)((nrow + 15) / 16), nct = (int)((ncol + 15) / 16);
            P.blocks.push_back(nrt);
            P.blocks.push_back(nct);
            gemm_macro_shape(nrt, nct, &B.mr, &B.mc);
            B.nmc = (nct + B.mc - 1) / B.mc;
            B.macro0 = (int64_t)P.macros.size() / kGemmMacroWidth;
            for (int r0 = 0; r0 < nrt; r0 += B.mr)
                for (int c0 = 0; c0 < nct; c0 += B.mc) {
                    const int MR = std::min(B.mr, nrt - r0), MC = std::min(B.mc, nct - c0);
                    P.macros.push_back((int32_t)(B.row0 + (int64_t)r0 * 16));
                    P.macros.push_back((int32_t)(B.col0 + (int64_t)c0 * 16));
                    P.macros.push_back(MR);
                    P.macros.push_back(MC);
                    P.macros.push_back((int32_t)ntiles);
                    ntiles += (int64_t)MR * MC;
                }
            blocks[{s, beta}] = std::move(B);
        }
    }
    if ((int64_t)P.rows.size() / RW > INT32_MAX || (int64_t)P.cols.size() / CW > INT32_MAX ||
        ntiles * 256 > INT32_MAX)
        return fail(ENCORE_EUNSUPPORTED, "split-bf16 coupling plan too large for this (N, lmax, nbins)");
    P.ntiles = ntiles;

    // (t, B) -> dense index; bit 31: (-1)^(sum of |m| over the factors with m < 0)
    const std::vector<int32_t> bt = enumerate_bin_tuples(N, nbins);
    const int64_t nB = (int64_t)bt.size() / K;
    P.tmap.assign((size_t)(tt.ntuple * nB), 0);
    for (int64_t t = 0; t < tt.ntuple; ++t) {
        const int s = msum(t);
        const int rho = rkeys[s][rkey(t)], sig = ckeys[s][ckey(t)];
        int neg = 0;
        for (int f = 0; f < K; ++f) {
            const int m = tt.tuple_m[t * K + f];
            if (m < 0 && (std::abs(m) & 1)) neg ^= 1;
        }
        for (int64_t b = 0; b < nB; ++b) {
            const int32_t* Bt = &bt[b * K];
            const Block& B = blocks.at({s, Bt[KL - 1]});
            const std::vector<int> pre(Bt, Bt + KL - 1), suf(Bt + KL, Bt + K);
            const int64_t row = (int64_t)rho * (int64_t)B.pre.size() + B.pre.at(pre);
            const int64_t col = (int64_t)sig * (int64_t)B.suf.size() + B.suf.at(suf);
            const int64_t rt = row / 16, ct = col / 16;
            const int mi = (int)(rt / B.mr), mj = (int)(ct / B.mc);
            const int32_t* M = &P.macros[(B.macro0 + (int64_t)mi * B.nmc + mj) * kGemmMacroWidth];
            const int64_t tile = M[4] + (rt % B.mr) * M[3] + (ct % B.mc);
            const int64_t dense = tile * 256 + (row % 16) * 16 + (col % 16);
            P.tmap[(size_t)(t * nB + b)] = (int32_t)dense | (neg ? (int32_t)0x80000000 : 0);
        }
    }
    return ENCORE_OK;
}

}  // namespace encore
