// Generalized Gaunt integrals G^{L L' L''} (eq. generalized-gaunt-def) of a multiplet
// list, as the terms of the edge-correction matrix (host only: built with g++ and
// the sanitizers by the tests as well as into the library).
//
// G comes from closed forms in the manner of Appendix A: products over the N-1
// directions of sqrt((2l+1)(2l'+1)(2l''+1)) (l l' l''; 0 0 0) over (4 pi)^{(N-1)/2},
// times one 9j symbol per node of the multiplet's coupling tree (l1 l2 -> l12, l12
// l3 -> l123, ..., the last node coupling to the last principal ell) and, for every
// intermediate x, sqrt((2x+1)(2x'+1)(2x''+1)): one 9j for N = 4, two for N = 5,
// three for N = 6 (the paper writes N = 3, 4, 5 and notes that higher orders follow
// the same construction; the N = 6 form is checked against the integral's
// definition).  For N = 3 the single 3j symbol is squared over 4 pi.  6j symbols by
// Racah's single sum (DLMF 34.4.3) and 9j symbols by the sum of 6j products (DLMF
// 34.6.2), in long double.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "internal.h"

namespace encore {

namespace {

long double lfact(int n)
{
    static long double table[256];
    static std::once_flag once;
    std::call_once(once, [] {
        table[0] = 1.0L;
        for (int i = 1; i < 256; ++i) table[i] = table[i - 1] * (long double)i;
    });
    return table[n];
}

bool tri(int a, int b, int c) { return c >= std::abs(a - b) && c <= a + b; }

long double delta_sq(int a, int b, int c)
{
    return lfact(a + b - c) * lfact(a - b + c) * lfact(-a + b + c) / lfact(a + b + c + 1);
}

long double sixj(int j1, int j2, int j3, int j4, int j5, int j6)
{
    if (!tri(j1, j2, j3) || !tri(j1, j5, j6) || !tri(j4, j2, j6) || !tri(j4, j5, j3)) return 0.0L;
    const int a[4] = {j1 + j2 + j3, j1 + j5 + j6, j4 + j2 + j6, j4 + j5 + j3};
    const int b[3] = {j1 + j2 + j4 + j5, j2 + j3 + j5 + j6, j3 + j1 + j6 + j4};
    const int tlo = std::max({a[0], a[1], a[2], a[3]}), thi = std::min({b[0], b[1], b[2]});
    long double s = 0.0L;
    for (int t = tlo; t <= thi; ++t) {
        long double den = 1.0L;
        for (int x : a) den *= lfact(t - x);
        for (int y : b) den *= lfact(y - t);
        s += ((t & 1) ? -1.0L : 1.0L) * lfact(t + 1) / den;
    }
    return s * std::sqrt(delta_sq(j1, j2, j3) * delta_sq(j1, j5, j6) * delta_sq(j4, j2, j6) *
                         delta_sq(j4, j5, j3));
}

long double ninej(int j1, int j2, int j3, int j4, int j5, int j6, int j7, int j8, int j9)
{
    const int lo = std::max({std::abs(j1 - j9), std::abs(j4 - j8), std::abs(j2 - j6)});
    const int hi = std::min({j1 + j9, j4 + j8, j2 + j6});
    long double s = 0.0L;
    for (int x = lo; x <= hi; ++x)
        s += (2 * x + 1) * sixj(j1, j4, j7, j8, j9, x) * sixj(j2, j5, j8, j4, x, j6) * sixj(j3, j6, j9, x, j1, j2);
    return s;
}

// Evaluates G^{L L' L''} from Appendix A for one multiplet list; the principal and
// intermediate ells are unpacked once, the 3j symbols with zero m are tabulated and
// the 9j symbols memoised (one evaluator per thread).
struct GauntEval {
    int N;
    int np;                               // principal ells per multiplet
    std::vector<int> pl, l12, l123;       // [n][np], [n] (N >= 5), [n] (N = 6)
    std::vector<long double> w0;          // (a b c; 0 0 0), index (a * D + b) * D + c
    int D;
    std::unordered_map<uint64_t, long double> memo;

    GauntEval(int N_, const std::vector<int32_t>& lam, int W, int n) : N(N_), np(N_ - 1)
    {
        pl.resize((size_t)n * np);
        l12.assign(n, 0);
        l123.assign(n, 0);
        int lmx = 0;
        for (int i = 0; i < n; ++i) {
            principal_of(N, &lam[(size_t)i * W], &pl[(size_t)i * np]);
            if (N >= 5) l12[i] = lam[(size_t)i * W + 2];
            if (N == 6) l123[i] = lam[(size_t)i * W + 4];
            for (int k = 0; k < np; ++k) lmx = std::max(lmx, pl[(size_t)i * np + k]);
        }
        D = lmx + 1;
        w0.assign((size_t)D * D * D, 0.0L);
        for (int a = 0; a < D; ++a)
            for (int b = 0; b < D; ++b)
                for (int c = 0; c < D; ++c)
                    w0[((size_t)a * D + b) * D + c] = wigner3j(a, b, c, 0, 0, 0);
    }
    long double nine(int j1, int j2, int j3, int j4, int j5, int j6, int j7, int j8, int j9)
    {
        const int v[9] = {j1, j2, j3, j4, j5, j6, j7, j8, j9};
        uint64_t key = 0;
        for (int x : v) key = key * 64 + (uint64_t)x;
        auto it = memo.find(key);
        if (it != memo.end()) return it->second;
        const long double r = ninej(j1, j2, j3, j4, j5, j6, j7, j8, j9);
        memo.emplace(key, r);
        return r;
    }
    double operator()(int a, int b, int c)
    {
        const int* la = &pl[(size_t)a * np];
        const int* lb = &pl[(size_t)b * np];
        const int* lc = &pl[(size_t)c * np];
        long double p = 1.0L;
        for (int i = 0; i < np; ++i) {
            if ((la[i] + lb[i] + lc[i]) & 1) return 0.0;   // (l l' l''; 0 0 0) = 0
            if (!tri(la[i], lb[i], lc[i])) return 0.0;
            const long double w = w0[((size_t)la[i] * D + lb[i]) * D + lc[i]];
            if (w == 0.0L) return 0.0;
            p *= std::sqrt((long double)(2 * la[i] + 1) * (2 * lb[i] + 1) * (2 * lc[i] + 1)) * w;
        }
        const long double fourpi = 4.0L * 3.14159265358979323846264338327950288L;
        if (N == 3) {   // single direction pair {l, l}: the 3j symbol squared
            const long double w = w0[((size_t)la[0] * D + lb[0]) * D + lc[0]];
            return (double)(std::sqrt((long double)(2 * la[0] + 1) * (2 * lb[0] + 1) * (2 * lc[0] + 1)) * w * w /
                            fourpi);
        }
        if (N == 4)
            return (double)(p / std::pow(fourpi, 1.5L) *
                            nine(la[0], lb[0], lc[0], la[1], lb[1], lc[1], la[2], lb[2], lc[2]));
        // N = 5, 6: intermediates l12 (and l123)
        const int a12 = l12[a], b12 = l12[b], c12 = l12[c];
        if (!tri(a12, b12, c12)) return 0.0;
        const long double s12 = std::sqrt((long double)(2 * a12 + 1) * (2 * b12 + 1) * (2 * c12 + 1));
        if (N == 5)
            return (double)(p / (fourpi * fourpi) * s12 *
                            nine(la[0], la[1], a12, lb[0], lb[1], b12, lc[0], lc[1], c12) *
                            nine(a12, la[2], la[3], b12, lb[2], lb[3], c12, lc[2], lc[3]));
        const int a123 = l123[a], b123 = l123[b], c123 = l123[c];
        if (!tri(a123, b123, c123)) return 0.0;
        const long double s123 = std::sqrt((long double)(2 * a123 + 1) * (2 * b123 + 1) * (2 * c123 + 1));
        return (double)(p / (fourpi * fourpi * std::sqrt(fourpi)) * s12 * s123 *
                        nine(la[0], la[1], a12, lb[0], lb[1], b12, lc[0], lc[1], c12) *
                        nine(a12, la[2], a123, b12, lb[2], b123, c12, lc[2], c123) *
                        nine(a123, la[3], la[4], b123, lb[3], lb[4], c123, lc[3], lc[4]));
    }
};

}  // namespace

const GauntTable& gaunt_table(int N, int lmax, bool allparity)
{
    static std::mutex mu;
    static std::map<std::tuple<int, int, bool>, std::unique_ptr<GauntTable>> cache;
    std::lock_guard<std::mutex> lk(mu);
    const auto key = std::make_tuple(N, lmax, allparity);
    auto it = cache.find(key);
    if (it != cache.end()) return *it->second;
    auto t = std::make_unique<GauntTable>();
    const std::vector<int32_t> lam = enumerate_multiplets(N, lmax, allparity);
    const int W = multiplet_width(N);
    const int n = (int)(lam.size() / W);
    t->nlam = n;
    t->lam = lam;
    std::vector<int> E(n);
    for (int i = 0; i < n; ++i) {
        int ls[5];
        principal_of(N, &lam[(size_t)i * W], ls);
        int s = 0;
        for (int k = 0; k < N - 1; ++k) s += ls[k];
        E[i] = (s & 1) ? -1 : 1;
    }
    // multiplets by their principal ells: G vanishes unless every direction's
    // (l, l', l'') satisfies the triangle rule with an even sum, so for (L, L'') only
    // the L' whose principal ells lie in those ranges are evaluated
    const int np = N - 1;
    std::map<std::vector<int>, std::vector<int32_t>> by_principal;
    std::vector<int> pls((size_t)n * np);
    for (int i = 0; i < n; ++i) {
        principal_of(N, &lam[(size_t)i * W], &pls[(size_t)i * np]);
        by_principal[std::vector<int>(&pls[(size_t)i * np], &pls[(size_t)i * np] + np)].push_back(i);
    }
    // entry (L = a, L'' = c) -> terms over L' = b, in increasing b; rows of a are
    // evaluated on several threads and joined in order
    const int nth = std::max(1, std::min<int>(16, (int)std::thread::hardware_concurrency()));
    std::vector<std::vector<int32_t>> lp(n);
    std::vector<std::vector<double>> val(n);
    std::vector<std::vector<int64_t>> cnt(n);
    std::atomic<int> next{0};
    auto worker = [&]() {
        GauntEval ge(N, lam, W, n);
        std::vector<int> cur(np);
        std::vector<std::pair<int32_t, double>> terms;
        for (int a = next++; a < n; a = next++) {
            cnt[a].assign(n, 0);
            const int* la = &pls[(size_t)a * np];
            for (int c = 0; c < n; ++c) {
                const int* lc = &pls[(size_t)c * np];
                terms.clear();
                // every principal tuple of L' allowed by (L, L'')
                std::function<void(int)> walk = [&](int k) {
                    if (k == np) {
                        auto it = by_principal.find(cur);
                        if (it == by_principal.end()) return;
                        for (const int32_t b : it->second) {
                            const double g = ge(a, b, c);
                            if (g != 0.0) terms.emplace_back(b, (E[a] < 0 && E[b] < 0 ? -1.0 : 1.0) * E[c] * g);
                        }
                        return;
                    }
                    for (int l = std::abs(la[k] - lc[k]); l <= la[k] + lc[k] && l <= lmax; l += 2) {
                        cur[k] = l;
                        walk(k + 1);
                    }
                };
                walk(0);
                std::sort(terms.begin(), terms.end());
                for (const auto& t : terms) {
                    lp[a].push_back(t.first);
                    val[a].push_back(t.second);
                }
                cnt[a][c] = (int64_t)terms.size();
            }
        }
    };
    std::vector<std::thread> th;
    for (int k = 0; k < nth; ++k) th.emplace_back(worker);
    for (auto& x : th) x.join();
    t->row_start.assign((size_t)n * n + 1, 0);
    for (int a = 0; a < n; ++a) {
        for (int c = 0; c < n; ++c) t->row_start[(size_t)a * n + c + 1] = t->row_start[(size_t)a * n + c] + cnt[a][c];
        t->term_lp.insert(t->term_lp.end(), lp[a].begin(), lp[a].end());
        t->term_val.insert(t->term_val.end(), val[a].begin(), val[a].end());
    }
    auto* out = t.get();
    cache.emplace(key, std::move(t));
    return *out;
}

}  // namespace encore
