// Host unit test of the macro-tiled coupling GEMM plan: every macro tile's GEMM,
// evaluated in FP64 on random coefficients exactly as the kernel forms its
// operands (rows: product of the first KL factors, Re/Im part; columns: w times the
// product of the others), must reproduce T[t][B] = sum_i w_i Q_t[prod_k a~] summed
// directly over the tuples (a~_{l,-m} = (-1)^m conj(a~_{l,m}), Appendix B), and
// every (t, B) must map to its own dense entry.  Built with g++ by
// tests/test_mfma_plan_cpu.py.
#include <cmath>
#include <complex>
#include <cstdio>
#include <random>
#include <set>
#include <string>
#include <vector>

#include "../../paper_2105_08722_amd/csrc/internal.h"
#include "../../paper_2105_08722_amd/csrc/mfma_plan.h"

namespace encore {
static std::string g_err;
void set_error(const std::string& m) { g_err = m; }
const char* get_error() { return g_err.c_str(); }
int fail(int code, const std::string& m) { g_err = m; return code; }
}  // namespace encore

using namespace encore;
using cd = std::complex<double>;

static int failures = 0;

static void check_case(int N, int L, bool allp, int nbins, int KL, int nprim, unsigned seed)
{
    GemmPlan P;
    if (build_gemm_plan(N, L, allp, nbins, KL, P) != 0) {
        std::printf("FAIL plan N=%d L=%d: %s\n", N, L, g_err.c_str());
        ++failures;
        return;
    }
    const int K = N - 1, KR = K - KL, nlm = (L + 1) * (L + 2) / 2;
    std::mt19937 rng(seed);
    std::normal_distribution<double> nd;
    std::vector<cd> a((size_t)nprim * nbins * nlm);
    std::vector<double> w(nprim);
    for (auto& v : a) v = cd(nd(rng), nd(rng));
    for (auto& v : w) v = nd(rng);
    for (int p = 0; p < nprim; ++p)   // m = 0 coefficients are real for real fields
        for (int b = 0; b < nbins; ++b)
            for (int l = 0; l <= L; ++l) a[((size_t)p * nbins + b) * nlm + l * (l + 1) / 2] = nd(rng);
    auto coef = [&](int p, int b, int l, int m) {
        const cd v = a[((size_t)p * nbins + b) * nlm + l * (l + 1) / 2 + std::abs(m)];
        if (m >= 0) return v;
        return ((std::abs(m) & 1) ? -1.0 : 1.0) * std::conj(v);
    };
    auto prod_of = [&](const int32_t* e, int nf, int fl, int p) {
        cd prod = 1.0;
        for (int k = 0; k < nf; ++k) {
            cd f = a[(size_t)p * nbins * nlm + e[k]];
            if (fl & (1 << k)) f = std::conj(f);
            prod *= f;
        }
        return prod;
    };
    std::vector<double> D((size_t)P.ntiles * 256, 0.0);
    const size_t nmacro = P.macros.size() / kGemmMacroWidth;
    for (size_t mc = 0; mc < nmacro; ++mc) {
        const int32_t* M = &P.macros[mc * kGemmMacroWidth];
        if (M[2] < 1 || M[3] < 1 || M[2] + M[3] > kGemmMaxOps || ((M[2] + 1) / 2) * ((M[3] + 1) / 2) > kGemmMaxOps) {
            std::printf("FAIL N=%d L=%d: macro shape %d x %d\n", N, L, M[2], M[3]);
            ++failures;
            return;
        }
        for (int tr = 0; tr < M[2]; ++tr)
            for (int tc = 0; tc < M[3]; ++tc)
                for (int i = 0; i < 16; ++i)
                    for (int j = 0; j < 16; ++j) {
                        const int32_t* row = &P.rows[(size_t)(M[0] + tr * 16 + i) * (KL + 1)];
                        const int32_t* col = &P.cols[(size_t)(M[1] + tc * 16 + j) * (KR + 1)];
                        double s = 0.0;
                        for (int p = 0; p < nprim; ++p) {
                            // padding rows / columns: their outputs are never mapped
                            const cd pl = (row[KL] & (1 << 9)) ? prod_of(row, KL, row[KL], p) : cd(0.0);
                            const cd pr = (col[KR] & (1 << 9)) ? w[p] * prod_of(col, KR, col[KR], p) : cd(0.0);
                            const bool im = row[KL] & (1 << 8);
                            const double x0 = im ? pl.imag() : pl.real();
                            const double x1 = im ? pl.real() : -pl.imag();
                            s += x0 * pr.real() + x1 * pr.imag();
                        }
                        D[(size_t)(M[4] + tr * M[3] + tc) * 256 + i * 16 + j] = s;
                    }
    }
    const TermTable& tt = term_table(N, L, allp);
    const std::vector<int32_t> bt = enumerate_bin_tuples(N, nbins);
    const int64_t nB = (int64_t)bt.size() / K;
    if ((int64_t)P.tmap.size() != tt.ntuple * nB) {
        std::printf("FAIL tmap size N=%d L=%d\n", N, L);
        ++failures;
        return;
    }
    std::set<int32_t> seen;
    double maxerr = 0.0, maxval = 0.0;
    for (int64_t t = 0; t < tt.ntuple; ++t)
        for (int64_t b = 0; b < nB; ++b) {
            double s = 0.0;
            for (int p = 0; p < nprim; ++p) {
                cd prod = 1.0;
                for (int k = 0; k < K; ++k)
                    prod *= coef(p, bt[b * K + k], tt.tuple_l[t * K + k], tt.tuple_m[t * K + k]);
                s += w[p] * (tt.tuple_odd[t] ? prod.imag() : prod.real());
            }
            const int32_t mv = P.tmap[t * nB + b];
            const int32_t idx = mv & 0x7fffffff;
            if (idx >= P.ntiles * 256 || !seen.insert(idx).second) {
                std::printf("FAIL N=%d L=%d: dense index %d out of range or repeated\n", N, L, idx);
                ++failures;
                return;
            }
            const double got = (mv < 0 ? -1.0 : 1.0) * D[idx];
            maxerr = std::max(maxerr, std::fabs(got - s));
            maxval = std::max(maxval, std::fabs(s));
        }
    const bool ok = maxerr <= 1e-12 * std::max(maxval, 1.0);
    std::printf("%s N=%d lmax=%d allparity=%d nbins=%d KL=%d: tuples %lld, macros %zu, tiles %lld, "
                "useful %.3f, max|dT| %.2e of %.2e\n",
                ok ? "ok  " : "FAIL", N, L, (int)allp, nbins, KL, (long long)tt.ntuple, nmacro,
                (long long)P.ntiles, (double)(tt.ntuple * nB) / std::max<double>(1.0, P.ntiles * 256.0), maxerr, maxval);
    if (!ok) ++failures;
}

int main()
{
    check_case(3, 4, false, 10, 1, 3, 1);
    check_case(3, 3, true, 7, 1, 3, 2);
    check_case(4, 5, false, 10, 2, 2, 3);
    check_case(4, 3, true, 7, 2, 3, 4);
    check_case(4, 3, false, 6, 1, 2, 5);
    check_case(5, 2, true, 6, 2, 2, 6);
    check_case(5, 3, false, 7, 2, 2, 7);
    check_case(6, 2, false, 6, 2, 2, 8);
    check_case(6, 1, true, 6, 2, 2, 9);
    check_case(6, 2, false, 6, 3, 2, 10);
    check_case(6, 2, true, 7, 3, 2, 12);
    check_case(5, 2, false, 10, 2, 1, 13);   // long thin blocks
    check_case(4, 3, false, 2, 2, 2, 11);   // nbins < N-1: no bin tuples
    if (failures) {
        std::printf("%d failures\n", failures);
        return 1;
    }
    std::printf("all passed\n");
    return 0;
}
