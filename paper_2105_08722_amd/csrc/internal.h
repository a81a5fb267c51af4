// Internal declarations shared by the host side of libencore (not part of the ABI).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace encore {

// ---------------------------------------------------------------- error state
void set_error(const std::string& msg);
const char* get_error();

struct Error {
    int code;
    std::string msg;
};

// ---------------------------------------------------------------- host tables
// Multiplets L in output order; each row has width(N) entries laid out as
// (l1, l2, (l12), l3, (l123), l4, l5) truncated to N.
int multiplet_width(int N);
std::vector<int32_t> enumerate_multiplets(int N, int lmax, bool allparity);
// principal ells of row r (N-1 of them)
void principal_of(int N, const int32_t* row, int* ls);

// Radial-bin tuples b_1 < ... < b_{N-1}, lexicographic, last fastest.
std::vector<int32_t> enumerate_bin_tuples(int N, int nbins);
int64_t binomial(int n, int k);

double wigner3j(int j1, int j2, int j3, int m1, int m2, int m3);
// C^L_M of the coupling chain (E(L) included).
double coupling(int N, const int32_t* lam_row, const int* M);

// Half-sum coupling terms (Appendix B): coef = 2 S(m_{N-1}) E(L) C^L_M.
struct TermTable {
    int N = 0, lmax = 0;
    bool allparity = false;
    int64_t nlam = 0;
    std::vector<int32_t> lam;     // [nterm]
    std::vector<int32_t> l, m;    // [nterm][N-1]
    std::vector<double> coef;     // [nterm]
    // distinct (l_k, m_k)_k tuples with m_{N-1} >= 0 (the device accumulates one
    // real component per tuple) and the contraction term -> tuple
    int64_t ntuple = 0;
    std::vector<int32_t> tuple_l, tuple_m;   // [ntuple][N-1]
    std::vector<int32_t> tuple_odd;          // [ntuple]  1: Im part, 0: Re part
    std::vector<int32_t> term_tuple;         // [nterm]
};
const TermTable& term_table(int N, int lmax, bool allparity);

// Generalized Gaunt integrals of the multiplet list (N, lmax, allparity), N = 3..6,
// as the terms of the edge-correction matrix: entry (L, L'') = a * nlam + c holds
// terms [row_start[e], row_start[e+1]) of (L' = term_lp, E(L'') G^{L L' L''} = term_val).
struct GauntTable {
    int nlam = 0;
    std::vector<int32_t> lam;          // [nlam][width(N)]
    std::vector<int64_t> row_start;    // [nlam * nlam + 1]
    std::vector<int32_t> term_lp;
    std::vector<double> term_val;
};
const GauntTable& gaunt_table(int N, int lmax, bool allparity);

}  // namespace encore
