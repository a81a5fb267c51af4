// Edge correction on the device (Section 3.2, eqs. edge-correction-matrix and
// edge-corrected-NPCF), one workgroup per radial-bin tuple B, FP64 throughout.
//
// k_edge_matrix: A[B][L''][L] = M_{L L''}(B) = sum_{L'} f_{L'}(B) E(L'') G^{L L' L''},
//   f = R_{L'} / R_0, each entry a fixed-order sum over its nonzero terms.
// k_edge_solve:  solves sum_L A[L''][L] zeta_L = N_{L''} / R_0 (eq.
//   edge-correction-matrix as written: M transposed) by Gaussian elimination with
//   partial pivoting and back substitution (row exchanges chosen by the first
//   largest |pivot|, so the result does not depend on thread timing).  B with
//   R_0 = 0 or a zero pivot get NaN and are counted.
#include <hip/hip_runtime.h>

#include <cmath>

#include "device.h"

namespace encore {

namespace {

constexpr int kEdgeThreads = 1024;   // 16 waves per block: enough loads in flight for the row updates

__global__ void __launch_bounds__(kEdgeThreads) k_edge_matrix(EdgeArgs a)
{
    extern __shared__ double f[];   // [nlam]
    const int B = blockIdx.x;
    const int n = a.nlam;
    const double r0 = a.rmult[B];
    for (int i = threadIdx.x; i < n; i += kEdgeThreads)
        f[i] = a.rmult[(size_t)i * a.nB + B] / r0;
    __syncthreads();
    double* A = a.A + (size_t)B * n * n;
    for (int L = 0; L < n; ++L)
        for (int Lpp = threadIdx.x; Lpp < n; Lpp += kEdgeThreads) {
            const int64_t e = (int64_t)L * n + Lpp;
            double s = 0.0;
            for (int64_t t = a.row_start[e]; t < a.row_start[e + 1]; ++t) s += a.term_val[t] * f[a.term_lp[t]];
            A[(size_t)Lpp * n + L] = s;
            if (a.M_out) a.M_out[(size_t)B * n * n + e] = s;
        }
}

__global__ void __launch_bounds__(kEdgeThreads) k_edge_solve(EdgeArgs a)
{
    extern __shared__ double sh[];   // factor column [n], then reduction scratch
    double* fac = sh;
    double* redv = sh + a.nlam;
    int* redi = reinterpret_cast<int*>(redv + kEdgeThreads);
    __shared__ int bad;
    const int B = blockIdx.x;
    const int n = a.nlam;
    double* A = a.A + (size_t)B * n * n;
    double* x = a.rhs + (size_t)B * n;
    const double r0 = a.rmult[B];
    if (threadIdx.x == 0) bad = !(r0 != 0.0) || !std::isfinite(r0);
    for (int i = threadIdx.x; i < n; i += kEdgeThreads) x[i] = a.nmult[(size_t)i * a.nB + B] / r0;
    __syncthreads();
    for (int k = 0; k < n && !bad; ++k) {
        // pivot: largest |A[r][k]|, r >= k, first such r
        double best = -1.0;
        int bi = n;
        for (int r = k + threadIdx.x; r < n; r += kEdgeThreads) {
            const double v = fabs(A[(size_t)r * n + k]);
            if (v > best) { best = v; bi = r; }
        }
        redv[threadIdx.x] = best;
        redi[threadIdx.x] = bi;
        __syncthreads();
        for (int s = kEdgeThreads / 2; s > 0; s >>= 1) {
            if (threadIdx.x < s) {
                const double v2 = redv[threadIdx.x + s];
                const int i2 = redi[threadIdx.x + s];
                if (v2 > redv[threadIdx.x] || (v2 == redv[threadIdx.x] && i2 < redi[threadIdx.x])) {
                    redv[threadIdx.x] = v2;
                    redi[threadIdx.x] = i2;
                }
            }
            __syncthreads();
        }
        const int p = redi[0];
        const double pv = A[(size_t)p * n + k];
        __syncthreads();
        if (!(pv != 0.0) || !std::isfinite(pv)) {
            if (threadIdx.x == 0) bad = 1;
            __syncthreads();
            break;
        }
        // exchange rows p and k (columns k.. and the right-hand side)
        if (p != k)
            for (int j = k + threadIdx.x; j <= n; j += kEdgeThreads) {
                double* ak = (j < n) ? &A[(size_t)k * n + j] : &x[k];
                double* ap = (j < n) ? &A[(size_t)p * n + j] : &x[p];
                const double vk = *ak;
                *ak = *ap;
                *ap = vk;
            }
        __syncthreads();
        for (int r = k + 1 + threadIdx.x; r < n; r += kEdgeThreads) fac[r] = A[(size_t)r * n + k] / pv;
        __syncthreads();
        // eliminate column k below the pivot: a wave per row, lanes along the row
        for (int r = k + 1 + threadIdx.x / kWave; r < n; r += kEdgeThreads / kWave) {
            const double fr = fac[r];
            if (fr == 0.0) continue;
            double* ar = &A[(size_t)r * n];
            const double* ak = &A[(size_t)k * n];
#pragma unroll 4
            for (int j = k + 1 + (threadIdx.x & (kWave - 1)); j < n; j += kWave) ar[j] -= fr * ak[j];
            if ((threadIdx.x & (kWave - 1)) == 0) x[r] -= fr * x[k];
        }
        __syncthreads();
    }
    // back substitution on the upper triangle
    if (!bad) {
        for (int k = n - 1; k >= 0; --k) {
            if (threadIdx.x == 0) x[k] /= A[(size_t)k * n + k];
            __syncthreads();
            const double xk = x[k];
            for (int r = threadIdx.x; r < k; r += kEdgeThreads) x[r] -= A[(size_t)r * n + k] * xk;
            __syncthreads();
        }
    }
    __syncthreads();
    // outputs: the kept multiplets in output order
    for (int i = threadIdx.x; i < a.nout; i += kEdgeThreads)
        a.zeta[(size_t)i * a.nB + B] = bad ? NAN : x[a.keep[i]];
    if (threadIdx.x == 0 && bad) atomicAdd(a.nbad, 1u);
}

}  // namespace

int launch_edge(const EdgeArgs& a, hipStream_t stream)
{
    if (a.nB == 0 || a.nlam == 0) return (int)hipSuccess;
    if (a.nlam > kEdgeMaxMultiplets) return (int)hipErrorInvalidValue;
    const size_t lds_m = sizeof(double) * (size_t)a.nlam;
    k_edge_matrix<<<dim3((unsigned)a.nB), dim3(kEdgeThreads), lds_m, stream>>>(a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return (int)e;
    const size_t lds_s = sizeof(double) * (size_t)(a.nlam + kEdgeThreads) + sizeof(int) * kEdgeThreads;
    k_edge_solve<<<dim3((unsigned)a.nB), dim3(kEdgeThreads), lds_s, stream>>>(a);
    return (int)hipGetLastError();
}

}  // namespace encore
