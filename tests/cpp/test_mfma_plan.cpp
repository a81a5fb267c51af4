// Host unit test of the split-BF16 MFMA coupling plan: the tile GEMMs the plan
// describes, evaluated in FP64 on random coefficients exactly as the kernel
// combines its operands, must reproduce T[t][B] = sum_i w_i Q_t[prod_k a~] summed
// directly over the tuples (with a~_{l,-m} = (-1)^m conj(a~_{l,m}), Appendix B),
// and every (t, B) must map to its own dense entry.  Built with g++ by
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

static void check_case(int N, int L, bool allp, int nbins, int nprim, unsigned seed)
{
    MfmaPlan P;
    if (build_mfma_plan(N, L, allp, nbins, P) != 0) {
        std::printf("FAIL plan N=%d L=%d: %s\n", N, L, g_err.c_str());
        ++failures;
        return;
    }
    const int K = N - 1, KF = K - 1, nlm = (L + 1) * (L + 2) / 2;
    std::mt19937 rng(seed);
    std::normal_distribution<double> nd;
    std::vector<cd> a((size_t)nprim * nbins * nlm);
    std::vector<double> w(nprim);
    for (auto& v : a) v = cd(nd(rng), nd(rng));
    for (auto& v : w) v = nd(rng);
    for (int p = 0; p < nprim; ++p)          // m = 0 coefficients are real for real fields
        for (int b = 0; b < nbins; ++b)
            for (int l = 0; l <= L; ++l) a[((size_t)p * nbins + b) * nlm + l * (l + 1) / 2] = nd(rng);
    auto coef = [&](int p, int b, int l, int m) {
        const cd v = a[((size_t)p * nbins + b) * nlm + l * (l + 1) / 2 + std::abs(m)];
        if (m >= 0) return v;
        return ((std::abs(m) & 1) ? -1.0 : 1.0) * std::conj(v);
    };
    // the tile GEMMs, in FP64
    std::vector<double> D((size_t)P.ntiles * 256, 0.0);
    for (int sh = 0; sh < kNumMfmaShapes; ++sh) {
        const int NC = kMfmaShapes[sh].NC;
        const size_t njob = P.jobs[sh].size() / kMfmaJobWidth;
        for (size_t jb = 0; jb < njob; ++jb) {
            const int32_t* J = &P.jobs[sh][jb * kMfmaJobWidth];
            for (int rt = 0; rt < J[3]; ++rt)
                for (int ct = 0; ct < NC; ++ct)
                    for (int i = 0; i < 16; ++i)
                        for (int j = 0; j < 16; ++j) {
                            const int64_t r = J[0] + rt * 16 + i;
                            const int c = P.cols[J[1] + ct * 16 + j];
                            const int32_t* row = &P.rows[r * (KF + 1)];
                            const int fl = row[KF];
                            if (!(fl & (1 << 9)) || c < 0) continue;
                            double s = 0.0;
                            for (int p = 0; p < nprim; ++p) {
                                cd prod = 1.0;
                                for (int k = 0; k < KF; ++k) {
                                    cd f = a[(size_t)p * nbins * nlm + row[k]];
                                    if (fl & (1 << k)) f = std::conj(f);
                                    prod *= f;
                                }
                                const bool im = fl & (1 << 8);
                                const double x0 = im ? prod.imag() : prod.real();
                                const double x1 = im ? prod.real() : -prod.imag();
                                const cd bv = w[p] * a[(size_t)p * nbins * nlm + c];
                                s += x0 * bv.real() + x1 * bv.imag();
                            }
                            D[(size_t)(J[2] + rt * NC + ct) * 256 + i * 16 + j] = s;
                        }
        }
    }
    // direct T over the tuples
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
    std::printf("%s N=%d lmax=%d allparity=%d nbins=%d: tuples %lld, tiles %lld, max|dT| %.2e of %.2e\n",
                ok ? "ok  " : "FAIL", N, L, (int)allp, nbins, (long long)tt.ntuple, (long long)P.ntiles,
                maxerr, maxval);
    if (!ok) ++failures;
}

int main()
{
    check_case(3, 4, false, 10, 3, 1);
    check_case(3, 3, true, 7, 3, 2);
    check_case(4, 5, false, 10, 2, 3);
    check_case(4, 3, true, 7, 3, 4);
    check_case(4, 2, false, 3, 3, 5);
    check_case(5, 2, true, 6, 2, 6);
    check_case(5, 3, false, 5, 2, 7);
    check_case(6, 2, false, 6, 2, 8);
    check_case(6, 1, true, 5, 2, 9);
    check_case(4, 3, false, 2, 2, 10);   // nbins < N-1: no bin tuples
    if (failures) {
        std::printf("%d failures\n", failures);
        return 1;
    }
    std::printf("all passed\n");
    return 0;
}
