// Edge correction on the device (Section 3.2, eqs. edge-correction-matrix and
// edge-corrected-NPCF), one workgroup per radial-bin tuple B, FP64 throughout.
//
// k_edge_matrix: A[B][L''][L] = M_{L L''}(B) = sum_{L'} f_{L'}(B) E(L'') G^{L L' L''},
//   f = R_{L'} / R_0, each entry a fixed-order sum over its nonzero terms, several
//   bin tuples per pass over the terms.
// k_edge_solve:  solves sum_L A[L''][L] zeta_L = N_{L''} / R_0 (eq.
//   edge-correction-matrix as written: M transposed) by a blocked LU with partial
//   pivoting and back substitution (row exchanges chosen by the first largest
//   |pivot|, so the result does not depend on thread timing).  B with R_0 = 0 or a
//   zero pivot get NaN and are counted.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "device.h"

namespace encore {

namespace {

constexpr int kEdgeThreads = 1024;   // 16 waves per block: enough loads in flight for the row updates

// One workgroup per (group of G bin tuples, range of L''): f = R_{L'} / R_0 of the G
// bin tuples sits in LDS ([L'][G]), a thread per L walks the terms of entry (L,
// L'') once for all G (so the term lists are read nB / G times, not nB) and writes
// the G matrices' row L'' (A[B][L''][L], coalesced along L).
template <int G>
__global__ void __launch_bounds__(kEdgeThreads) k_edge_matrix(EdgeArgs a, int rows_per_block)
{
    extern __shared__ double f[];   // [nlam][G]
    const int n = a.nlam;
    const int B0 = blockIdx.x * G;
    const int nb = min(G, a.nB - B0);
    for (int i = threadIdx.x; i < n * G; i += kEdgeThreads) {
        const int lp = i / G, g = i - lp * G;
        f[i] = g < nb ? a.rmult[(size_t)lp * a.nB + B0 + g] / a.rmult[B0 + g] : 0.0;
    }
    __syncthreads();
    const int q0 = blockIdx.y * rows_per_block, q1 = min(n, q0 + rows_per_block);
    for (int Lpp = q0; Lpp < q1; ++Lpp)
        for (int L = threadIdx.x; L < n; L += kEdgeThreads) {
            const int64_t e = (int64_t)L * n + Lpp;
            double s[G];
#pragma unroll
            for (int g = 0; g < G; ++g) s[g] = 0.0;
            for (int64_t t = a.row_start[e]; t < a.row_start[e + 1]; ++t) {
                const double v = a.term_val[t];
                const double* fp = &f[(size_t)a.term_lp[t] * G];
#pragma unroll
                for (int g = 0; g < G; ++g) s[g] += v * fp[g];
            }
#pragma unroll
            for (int g = 0; g < G; ++g) {
                if (g >= nb) break;
                a.A[((size_t)(B0 + g) * n + Lpp) * n + L] = s[g];
                if (a.M_out) a.M_out[((size_t)(B0 + g) * n + L) * n + Lpp] = s[g];
            }
        }
}

template <int G>
int launch_edge_matrix(const EdgeArgs& a, hipStream_t stream)
{
    const int gx = (a.nB + G - 1) / G;
    const int gy = std::max(1, std::min(a.nlam, (1024 + gx - 1) / gx));   // ~1024 blocks
    const int rows = (a.nlam + gy - 1) / gy;
    const size_t lds = sizeof(double) * (size_t)a.nlam * G;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_edge_matrix<G>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return (int)e;
    k_edge_matrix<G><<<dim3((unsigned)gx, (unsigned)((a.nlam + rows - 1) / rows)), dim3(kEdgeThreads), lds, stream>>>(a,
                                                                                                               rows);
    return (int)hipGetLastError();
}

// Solve: LU with partial pivoting, blocked right-looking (panels of kLuPanel columns),
// one workgroup per B, the matrix in global memory.  Per panel: (1) the panel's
// columns are eliminated one by one (first largest |pivot| of the column, the row
// exchange applied from the panel's first column on and to the right-hand side, the
// multipliers stored in place, the right-hand side updated); (2) the panel rows'
// part right of the panel becomes U12 = L11^-1 A12 (forward substitution with the
// panel's unit lower triangle); (3) the trailing matrix takes A22 -= L21 U12 in
// 128 x 128 tiles, 4 x 4 per thread, L21 and U12 staged in LDS.  The trailing
// matrix is thus read and written once per panel instead of once per column, which
// bounded the unblocked elimination.  Then back substitution on U.
constexpr int kLuPanel = 32;
constexpr int kLuTile = 128;
constexpr size_t kLuLds = sizeof(double) * ((size_t)kLuTile * (kLuPanel + 1) + (size_t)kLuPanel * kLuTile +
                                            (size_t)kLuPanel * kLuPanel + kEdgeThreads) +
                          sizeof(int) * kEdgeThreads;

__global__ void __launch_bounds__(kEdgeThreads) k_edge_solve(EdgeArgs a)
{
    extern __shared__ double sh[];
    double* Ls = sh;                                        // [kLuTile][kLuPanel + 1]
    double* Us = Ls + kLuTile * (kLuPanel + 1);             // [kLuPanel][kLuTile]
    double* L11 = Us + kLuPanel * kLuTile;                  // [kLuPanel][kLuPanel]
    double* redv = L11 + kLuPanel * kLuPanel;               // [kEdgeThreads]
    int* redi = reinterpret_cast<int*>(redv + kEdgeThreads);
    __shared__ int bad;
    const int tid = threadIdx.x;
    const int B = blockIdx.x;
    const int n = a.nlam;
    double* A = a.A + (size_t)B * n * n;
    double* x = a.rhs + (size_t)B * n;
    const double r0 = a.rmult[B];
    if (tid == 0) bad = !(r0 != 0.0) || !std::isfinite(r0);
    for (int i = tid; i < n; i += kEdgeThreads) x[i] = a.nmult[(size_t)i * a.nB + B] / r0;
    __syncthreads();
    for (int k0 = 0; k0 < n && !bad; k0 += kLuPanel) {
        const int kb = min(kLuPanel, n - k0);
        const int ke = k0 + kb;                             // first column right of the panel
        // (1) the panel's columns
        for (int j = k0; j < ke; ++j) {
            double best = -1.0;
            int bi = n;
            for (int r = j + tid; r < n; r += kEdgeThreads) {
                const double v = fabs(A[(size_t)r * n + j]);
                if (v > best) { best = v; bi = r; }
            }
            redv[tid] = best;
            redi[tid] = bi;
            __syncthreads();
            for (int st = kEdgeThreads / 2; st > 0; st >>= 1) {
                if (tid < st) {
                    const double v2 = redv[tid + st];
                    const int i2 = redi[tid + st];
                    if (v2 > redv[tid] || (v2 == redv[tid] && i2 < redi[tid])) {
                        redv[tid] = v2;
                        redi[tid] = i2;
                    }
                }
                __syncthreads();
            }
            const int p = redi[0];
            const double pv = A[(size_t)p * n + j];
            __syncthreads();
            if (!(pv != 0.0) || !std::isfinite(pv)) {
                if (tid == 0) bad = 1;
                __syncthreads();
                break;
            }
            if (p != j)
                for (int c = k0 + tid; c <= n; c += kEdgeThreads) {
                    double* aj = (c < n) ? &A[(size_t)j * n + c] : &x[j];
                    double* ap = (c < n) ? &A[(size_t)p * n + c] : &x[p];
                    const double v = *aj;
                    *aj = *ap;
                    *ap = v;
                }
            __syncthreads();
            // multipliers of column j, and the rank-1 update of the panel's columns
            // right of j and of the right-hand side; a thread per row
            const double xj = x[j];
            for (int r = j + 1 + tid; r < n; r += kEdgeThreads) {
                double* ar = &A[(size_t)r * n];
                const double l = ar[j] / pv;
                ar[j] = l;
                if (l == 0.0) continue;
                const double* aj = &A[(size_t)j * n];
                for (int c = j + 1; c < ke; ++c) ar[c] -= l * aj[c];
                x[r] -= l * xj;
            }
            __syncthreads();
        }
        if (bad || ke >= n) break;
        // (2) U12 = L11^-1 A12: row i of the panel loses its multipliers times the
        // rows above it (already final), a thread per column
        for (int e = tid; e < kb * kb; e += kEdgeThreads) L11[e] = A[(size_t)(k0 + e / kb) * n + k0 + e % kb];
        __syncthreads();
        for (int i = 1; i < kb; ++i) {
            for (int c = ke + tid; c < n; c += kEdgeThreads) {
                double v = A[(size_t)(k0 + i) * n + c];
                for (int t = 0; t < i; ++t) v -= L11[i * kb + t] * A[(size_t)(k0 + t) * n + c];
                A[(size_t)(k0 + i) * n + c] = v;
            }
            __syncthreads();
        }
        // (3) A22 -= L21 U12 over 128 x 128 tiles; thread (ty, tx) of 32 x 32 owns rows
        // R0 + ty + 32 i and columns C0 + tx + 32 jj (coalesced along tx)
        const int tx = tid & 31, ty = tid >> 5;
        for (int R0 = ke; R0 < n; R0 += kLuTile)
            for (int C0 = ke; C0 < n; C0 += kLuTile) {
                for (int e = tid; e < kLuTile * kLuPanel; e += kEdgeThreads) {
                    const int rr = e / kLuPanel, t = e % kLuPanel;
                    Ls[rr * (kLuPanel + 1) + t] =
                        (R0 + rr < n && t < kb) ? A[(size_t)(R0 + rr) * n + k0 + t] : 0.0;
                    const int t2 = e / kLuTile, cc = e % kLuTile;
                    Us[t2 * kLuTile + cc] = (C0 + cc < n && t2 < kb) ? A[(size_t)(k0 + t2) * n + C0 + cc] : 0.0;
                }
                __syncthreads();
                double acc[4][4];
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int jj = 0; jj < 4; ++jj) acc[i][jj] = 0.0;
                for (int t = 0; t < kb; ++t) {
                    double lv[4], uv[4];
#pragma unroll
                    for (int i = 0; i < 4; ++i) lv[i] = Ls[(ty + 32 * i) * (kLuPanel + 1) + t];
#pragma unroll
                    for (int jj = 0; jj < 4; ++jj) uv[jj] = Us[t * kLuTile + tx + 32 * jj];
#pragma unroll
                    for (int i = 0; i < 4; ++i)
#pragma unroll
                        for (int jj = 0; jj < 4; ++jj) acc[i][jj] = fma(lv[i], uv[jj], acc[i][jj]);
                }
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int r = R0 + ty + 32 * i;
                    if (r >= n) continue;
#pragma unroll
                    for (int jj = 0; jj < 4; ++jj) {
                        const int c = C0 + tx + 32 * jj;
                        if (c < n) A[(size_t)r * n + c] -= acc[i][jj];
                    }
                }
                __syncthreads();
            }
    }
    // back substitution on the upper triangle
    if (!bad) {
        for (int k = n - 1; k >= 0; --k) {
            if (tid == 0) x[k] /= A[(size_t)k * n + k];
            __syncthreads();
            const double xk = x[k];
            for (int r = tid; r < k; r += kEdgeThreads) x[r] -= A[(size_t)r * n + k] * xk;
            __syncthreads();
        }
    }
    __syncthreads();
    // outputs: the kept multiplets in output order
    for (int i = tid; i < a.nout; i += kEdgeThreads)
        a.zeta[(size_t)i * a.nB + B] = bad ? NAN : x[a.keep[i]];
    if (tid == 0 && bad) atomicAdd(a.nbad, 1u);
}

}  // namespace

int launch_edge(const EdgeArgs& a, hipStream_t stream)
{
    if (a.nB == 0 || a.nlam == 0) return (int)hipSuccess;
    if (a.nlam > kEdgeMaxMultiplets) return (int)hipErrorInvalidValue;
    // eight bin tuples per block while their f tables fit the LDS, else four
    hipError_t e = (hipError_t)(a.nlam * 8 * sizeof(double) <= 150 * 1024 ? launch_edge_matrix<8>(a, stream)
                                                                         : launch_edge_matrix<4>(a, stream));
    if (e != hipSuccess) return (int)e;
    static bool attr_set = false;
    if (!attr_set) {
        e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_edge_solve),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLuLds);
        if (e != hipSuccess) return (int)e;
        attr_set = true;
    }
    k_edge_solve<<<dim3((unsigned)a.nB), dim3(kEdgeThreads), kLuLds, stream>>>(a);
    return (int)hipGetLastError();
}

}  // namespace encore
