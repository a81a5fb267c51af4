// Host unit test of the edge-correction Gaunt table (gaunt.cpp): every term of
// gaunt_table(N, lmax, parity) against the oracle's closed-form values, read from
// a text file written by tests/test_gaunt_cpu.py (entries above 1e-14 of the
// largest), and no such (L, L', L'') missing; terms the oracle lists as zero must
// be below that level (exact cancellations in the 9j sums).  Built with g++ under ASan + UBSan and under TSan
// (the table is built on several threads).
#include <cmath>
#include <cstdio>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "../../paper_2105_08722_amd/csrc/internal.h"

namespace encore {
static std::string g_err;
void set_error(const std::string& m) { g_err = m; }
const char* get_error() { return g_err.c_str(); }
int fail(int code, const std::string& m) { g_err = m; return code; }
}  // namespace encore

using namespace encore;

int main(int argc, char** argv)
{
    if (argc < 2) return 2;
    FILE* f = std::fopen(argv[1], "r");
    if (!f) return 2;
    int failures = 0, N, lmax, allp, n;
    long long nnz;
    while (std::fscanf(f, "%d %d %d %d %lld", &N, &lmax, &allp, &n, &nnz) == 5) {
        // oracle: (a, b, c) -> s(a, b) E(c) G(a, b, c), the value a table term holds
        std::map<std::tuple<int, int, int>, double> want;
        for (long long k = 0; k < nnz; ++k) {
            int a, b, c;
            double v;
            if (std::fscanf(f, "%d %d %d %lf", &a, &b, &c, &v) != 4) return 2;
            want[std::make_tuple(a, b, c)] = v;
        }
        const GauntTable& t = gaunt_table(N, lmax, allp != 0);
        if (t.nlam != n) {
            std::printf("FAIL N=%d lmax=%d: %d multiplets, oracle %d\n", N, lmax, t.nlam, n);
            ++failures;
            continue;
        }
        double worst = 0.0, scale = 0.0;
        long long found = 0;
        for (int a = 0; a < n; ++a)
            for (int c = 0; c < n; ++c)
                for (int64_t e = t.row_start[(size_t)a * n + c]; e < t.row_start[(size_t)a * n + c + 1]; ++e) {
                    const int b = t.term_lp[e];
                    if (e > t.row_start[(size_t)a * n + c] && t.term_lp[e - 1] >= b) {
                        std::printf("FAIL N=%d: terms of (%d, %d) not in increasing L'\n", N, a, c);
                        ++failures;
                    }
                    auto it = want.find(std::make_tuple(a, b, c));
                    const double w = it == want.end() ? 0.0 : it->second;
                    if (it != want.end()) ++found;
                    worst = std::max(worst, std::fabs(t.term_val[e] - w));
                    scale = std::max(scale, std::fabs(w));
                }
        const bool ok = found == nnz && worst <= 1e-13 * std::max(scale, 1e-30);
        if (found != nnz) std::printf("  %lld of %lld oracle terms found\n", found, nnz);
        std::printf("%s N=%d lmax=%d allparity=%d: %d multiplets, %lld terms (oracle %lld), max diff %.2e of %.2e\n",
                    ok ? "ok  " : "FAIL", N, lmax, allp, n, (long long)t.term_lp.size(), nnz, worst, scale);
        if (!ok) ++failures;
    }
    std::fclose(f);
    if (failures) return 1;
    std::printf("all passed\n");
    return 0;
}
