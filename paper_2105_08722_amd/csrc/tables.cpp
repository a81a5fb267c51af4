// Host-side tables of the isotropic basis for the device path.
//
// * Multiplets (Section 2.1, eq. basis-coupling): principal l_i <= lmax, the
//   intermediates l_12, l_123 bounded by their triangle conditions, parity-even
//   only unless all parities are asked for (Section 3.1).
// * Coupling coefficients C^L_M of eq. basis-coupling, from Wigner 3j symbols.
//   The 3j symbols use the Racah single-sum formula (DLMF 34.2.4) evaluated in
//   long double with a table of factorials.
// * The half-sum terms of Appendix B: only M with m_{N-1} >= 0 are kept, each with
//   weight 2 S(m_{N-1}) E(L) C^L_M, S(0) = 1/2, applied to Re (even L) or Im (odd L)
//   of the product of harmonic coefficients.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <map>
#include <memory>
#include <mutex>
#include <tuple>

#include "internal.h"

namespace encore {

int multiplet_width(int N) { return N == 3 ? 2 : 2 * N - 5; }

void principal_of(int N, const int32_t* row, int* ls)
{
    switch (N) {
    case 3: ls[0] = row[0]; ls[1] = row[1]; break;
    case 4: ls[0] = row[0]; ls[1] = row[1]; ls[2] = row[2]; break;
    case 5: ls[0] = row[0]; ls[1] = row[1]; ls[2] = row[3]; ls[3] = row[4]; break;
    default: ls[0] = row[0]; ls[1] = row[1]; ls[2] = row[3]; ls[3] = row[5]; ls[4] = row[6]; break;
    }
}

std::vector<int32_t> enumerate_multiplets(int N, int lmax, bool allparity)
{
    std::vector<int32_t> out;
    auto keep = [&](int sum) { return allparity || (sum % 2 == 0); };
    if (N == 3) {
        for (int l = 0; l <= lmax; ++l) { out.push_back(l); out.push_back(l); }
        return out;
    }
    for (int l1 = 0; l1 <= lmax; ++l1)
    for (int l2 = 0; l2 <= lmax; ++l2) {
        if (N == 4) {
            for (int l3 = std::abs(l1 - l2); l3 <= std::min(l1 + l2, lmax); ++l3)
                if (keep(l1 + l2 + l3)) { out.push_back(l1); out.push_back(l2); out.push_back(l3); }
            continue;
        }
        for (int l12 = std::abs(l1 - l2); l12 <= l1 + l2; ++l12)
        for (int l3 = 0; l3 <= lmax; ++l3) {
            if (N == 5) {
                for (int l4 = std::abs(l12 - l3); l4 <= std::min(l12 + l3, lmax); ++l4)
                    if (keep(l1 + l2 + l3 + l4)) {
                        int32_t r[5] = {l1, l2, l12, l3, l4};
                        out.insert(out.end(), r, r + 5);
                    }
                continue;
            }
            for (int l123 = std::abs(l12 - l3); l123 <= l12 + l3; ++l123)
            for (int l4 = 0; l4 <= lmax; ++l4)
            for (int l5 = std::abs(l123 - l4); l5 <= std::min(l123 + l4, lmax); ++l5)
                if (keep(l1 + l2 + l3 + l4 + l5)) {
                    int32_t r[7] = {l1, l2, l12, l3, l123, l4, l5};
                    out.insert(out.end(), r, r + 7);
                }
        }
    }
    return out;
}

int64_t binomial(int n, int k)
{
    if (k < 0 || k > n) return 0;
    int64_t r = 1;
    for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
    return r;
}

std::vector<int32_t> enumerate_bin_tuples(int N, int nbins)
{
    const int k = N - 1;
    std::vector<int32_t> out;
    if (nbins < k) return out;
    std::vector<int> b(k);
    for (int i = 0; i < k; ++i) b[i] = i;
    while (true) {
        out.insert(out.end(), b.begin(), b.end());
        int i = k - 1;
        while (i >= 0 && b[i] == nbins - k + i) --i;
        if (i < 0) break;
        ++b[i];
        for (int j = i + 1; j < k; ++j) b[j] = b[j - 1] + 1;
    }
    return out;
}

// ------------------------------------------------------------------ 3j symbols
static long double fact(int n)
{
    static long double table[200];
    static std::once_flag once;
    std::call_once(once, [] {
        table[0] = 1.0L;
        for (int i = 1; i < 200; ++i) table[i] = table[i - 1] * (long double)i;
    });
    return table[n];
}

double wigner3j(int j1, int j2, int j3, int m1, int m2, int m3)
{
    if (m1 + m2 + m3 != 0) return 0.0;
    if (j3 < std::abs(j1 - j2) || j3 > j1 + j2) return 0.0;
    if (std::abs(m1) > j1 || std::abs(m2) > j2 || std::abs(m3) > j3) return 0.0;
    if (j1 + j2 + j3 + 1 >= 200) return NAN;
    // Racah: sqrt(Delta * prod (j+-m)!) * sum_k (-1)^k / [k! (j3-j2+k+m1)! (j3-j1+k-m2)!
    //        (j1+j2-j3-k)! (j1-k-m1)! (j2-k+m2)!],   overall phase (-1)^(j1-j2-m3)
    const long double tri = fact(j1 + j2 - j3) * fact(j1 - j2 + j3) * fact(-j1 + j2 + j3) /
                            fact(j1 + j2 + j3 + 1);
    const long double pre = fact(j1 + m1) * fact(j1 - m1) * fact(j2 + m2) * fact(j2 - m2) *
                            fact(j3 + m3) * fact(j3 - m3);
    const int kmin = std::max({0, j2 - j3 - m1, j1 - j3 + m2});
    const int kmax = std::min({j1 + j2 - j3, j1 - m1, j2 + m2});
    long double s = 0.0L;
    for (int k = kmin; k <= kmax; ++k) {
        const long double den = fact(k) * fact(j3 - j2 + k + m1) * fact(j3 - j1 + k - m2) *
                                fact(j1 + j2 - j3 - k) * fact(j1 - k - m1) * fact(j2 - k + m2);
        s += ((k & 1) ? -1.0L : 1.0L) / den;
    }
    long double v = std::sqrt(tri * pre) * s;
    if (((j1 - j2 - m3) % 2 + 2) % 2) v = -v;
    // values that are exactly zero by cancellation come out ~1e-19 relative
    if (std::fabs(v) < 1e-15L) return 0.0;
    return (double)v;
}

double coupling(int N, const int32_t* row, const int* M)
{
    int ls[5];
    principal_of(N, row, ls);
    int sum_l = 0, sum_m = 0;
    for (int k = 0; k < N - 1; ++k) {
        if (std::abs(M[k]) > ls[k]) return 0.0;
        sum_l += ls[k];
        sum_m += M[k];
    }
    if (sum_m != 0) return 0.0;
    const double E = (sum_l % 2) ? -1.0 : 1.0;
    if (N == 3) return E * wigner3j(ls[0], ls[1], 0, M[0], M[1], 0);
    if (N == 4) return E * wigner3j(ls[0], ls[1], ls[2], M[0], M[1], M[2]);
    // Chain with intermediates: (l1 l2 l12; m1 m2 -m12) [(l12 l3 l123; m12 m3 -m123)]
    // (l_last_int l_{N-2} l_{N-1}; m_last_int m_{N-2} m_{N-1}), phase (-1)^kappa,
    // kappa = sum over intermediates of (l_int - m_int), times prod sqrt(2 l_int + 1).
    const int nint = N - 4;
    int lint[2] = {row[2], N == 6 ? row[4] : 0};
    int mcur = M[0] + M[1];
    if (std::abs(mcur) > lint[0]) return 0.0;
    double val = wigner3j(ls[0], ls[1], lint[0], M[0], M[1], -mcur);
    int kappa = lint[0] - mcur;
    double pref = std::sqrt(2.0 * lint[0] + 1.0);
    for (int q = 1; q < nint; ++q) {
        const int mnext = mcur + M[q + 1];
        if (std::abs(mnext) > lint[q]) return 0.0;
        val *= wigner3j(lint[q - 1], ls[q + 1], lint[q], mcur, M[q + 1], -mnext);
        kappa += lint[q] - mnext;
        pref *= std::sqrt(2.0 * lint[q] + 1.0);
        mcur = mnext;
    }
    val *= wigner3j(lint[nint - 1], ls[N - 3], ls[N - 2], mcur, M[N - 3], M[N - 2]);
    if (((kappa % 2) + 2) % 2) val = -val;
    return E * pref * val;
}

// ------------------------------------------------------------------ term tables
static TermTable build_terms(int N, int lmax, bool allparity)
{
    TermTable T;
    T.N = N; T.lmax = lmax; T.allparity = allparity;
    const int W = multiplet_width(N);
    const int K = N - 1;
    std::vector<int32_t> lams = enumerate_multiplets(N, lmax, allparity);
    T.nlam = (int64_t)lams.size() / W;
    std::map<std::vector<int32_t>, int64_t> tuple_index;
    for (int64_t li = 0; li < T.nlam; ++li) {
        const int32_t* row = &lams[li * W];
        int ls[5];
        principal_of(N, row, ls);
        int sum_l = 0;
        for (int k = 0; k < K; ++k) sum_l += ls[k];
        const double E = (sum_l % 2) ? -1.0 : 1.0;
        // iterate m_1..m_{N-2} over their ranges; m_{N-1} = -sum, keep m_{N-1} >= 0
        int M[5] = {0, 0, 0, 0, 0};
        for (int k = 0; k < K - 1; ++k) M[k] = -ls[k];
        while (true) {
            int s = 0;
            for (int k = 0; k < K - 1; ++k) s += M[k];
            const int mlast = -s;
            if (mlast >= 0 && mlast <= ls[K - 1]) {
                M[K - 1] = mlast;
                const double c = coupling(N, row, M);
                if (c != 0.0) {
                    const double S = (mlast == 0) ? 0.5 : 1.0;
                    T.lam.push_back((int32_t)li);
                    std::vector<int32_t> key;
                    for (int k = 0; k < K; ++k) {
                        T.l.push_back(ls[k]);
                        T.m.push_back(M[k]);
                        key.push_back(ls[k]);
                        key.push_back(M[k]);
                    }
                    T.coef.push_back(2.0 * S * E * c);
                    auto it = tuple_index.find(key);
                    int64_t ti;
                    if (it == tuple_index.end()) {
                        ti = T.ntuple++;
                        tuple_index.emplace(key, ti);
                        for (int k = 0; k < K; ++k) {
                            T.tuple_l.push_back(ls[k]);
                            T.tuple_m.push_back(M[k]);
                        }
                        T.tuple_odd.push_back(sum_l % 2);
                    } else {
                        ti = it->second;
                    }
                    T.term_tuple.push_back((int32_t)ti);
                }
            }
            // odometer over m_1..m_{N-2}
            int k = K - 2;
            while (k >= 0 && M[k] == ls[k]) { M[k] = -ls[k]; --k; }
            if (k < 0) break;
            ++M[k];
        }
    }
    return T;
}

const TermTable& term_table(int N, int lmax, bool allparity)
{
    static std::mutex mu;
    static std::map<std::tuple<int, int, bool>, std::unique_ptr<TermTable>> cache;
    std::lock_guard<std::mutex> lock(mu);
    auto key = std::make_tuple(N, lmax, allparity);
    auto it = cache.find(key);
    if (it != cache.end()) return *it->second;
    auto t = std::make_unique<TermTable>(build_terms(N, lmax, allparity));
    const TermTable& ref = *t;
    cache.emplace(key, std::move(t));
    return ref;
}

}  // namespace encore
