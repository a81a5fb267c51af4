// Coupling step (eq. NPCF-mult-discrete-binned-estimator with the Appendix B half
// sum), reassociated so that the sum over primaries comes first:
//
//   T[t][B]  = sum_i w_i Q_t[ prod_k a~^{b_k}_{l_k m_k}(i) ]          (k_couple)
//   Z[L][B]  = sum_{terms (L, t)} 2 S(m_{N-1}) E(L) C^L_M  T[t][B]      (k_contract)
//
// t runs over the distinct (l_k, m_k)_k tuples with m_{N-1} >= 0 that carry a
// nonzero coupling; Q_t is Re for parity-even and Im for parity-odd tuples.  The
// identity is exact in real arithmetic (the coupling does not depend on i).
// a~ for m < 0 comes from a~_{l,-m} = (-1)^m conj(a~_{l,m}) (Appendix B).
//
// k_couple: one thread per (t, B) output, FP64 accumulator; the block stages a tile
// of primaries' coefficients in LDS and every thread walks the tile.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device.h"

namespace encore {

namespace {

constexpr int kBlock = 256;
constexpr int kMaxK = 5;

template <typename T> struct C2;
template <> struct C2<float> { using type = float2; };
template <> struct C2<double> { using type = double2; };

template <typename T, int NK>
__global__ void __launch_bounds__(kBlock) k_couple(CoupleArgs a, int ptile)
{
    using V = typename C2<T>::type;
    extern __shared__ __align__(16) unsigned char smem[];
    V* tile = reinterpret_cast<V*>(smem);
    const int per = a.nbins * a.nlm;                       // complex values per primary
    double* wtile = reinterpret_cast<double*>(smem + sizeof(V) * (size_t)ptile * per);

    const int64_t gid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const bool valid = gid < (int64_t)a.ntuple * a.nB;
    const int t = valid ? (int)(gid / a.nB) : 0;
    const int b = valid ? (int)(gid - (int64_t)t * a.nB) : 0;
    const int split = blockIdx.y;
    const int p_lo = a.split_lo[split];
    const int p_hi = a.split_hi[split];

    int off[NK];
    T cs[NK];
    int flags = 0;
#pragma unroll
    for (int k = 0; k < NK; ++k) { off[k] = 0; cs[k] = (T)1; }
    if (valid) {
        flags = a.tuple_flags[t];
#pragma unroll
        for (int k = 0; k < NK; ++k) {
            off[k] = a.btab[b * a.nk + k] * a.nlm + a.tuple_off[t * a.nk + k];
            cs[k] = ((flags >> k) & 1) ? (T)-1 : (T)1;
        }
    }
    const bool take_im = (flags >> 16) & 1;
    double acc = 0.0;

    for (int p0 = p_lo; p0 < p_hi; p0 += ptile) {
        const int np = min(ptile, p_hi - p0);
        __syncthreads();
        const V* src = reinterpret_cast<const V*>(a.alm) + (size_t)p0 * per;
        for (int q = threadIdx.x; q < np * per; q += kBlock) tile[q] = src[q];
        for (int q = threadIdx.x; q < np; q += kBlock) wtile[q] = a.wprim[p0 + q];
        __syncthreads();
        if (valid) {
            for (int pp = 0; pp < np; ++pp) {
                const V* ap = tile + pp * per;
                V v = ap[off[0]];
                T pr = v.x, pi = cs[0] * v.y;
#pragma unroll
                for (int k = 1; k < NK; ++k) {
                    const V u = ap[off[k]];
                    const T ur = u.x, ui = cs[k] * u.y;
                    const T nr = pr * ur - pi * ui;
                    const T ni = pr * ui + pi * ur;
                    pr = nr; pi = ni;
                }
                const T q = take_im ? pi : pr;
                acc += wtile[pp] * (double)q;
            }
        }
    }
    if (valid) {
        if ((flags >> 8) & 1) acc = -acc;
        a.T[((size_t)split * a.ntuple + t) * a.nB + b] = acc;
    }
}

// 4PCF with 10 radial bins: one block per (b1, 256 tuples, primary split).
// For each primary each thread loads a~^{b1} of its first factor once, the
// second-factor a~^{b2} and third-factor a~^{b3} rows once each, forms
// P = w a1 a2 once per b2 and adds Q[P a3] for every b3 > b2.  Accumulation: FP32
// over a tile of primaries, then FP64 registers (the FP64 path: FP64 throughout).
constexpr int kNB4 = 10;
__host__ __device__ constexpr int pair_count(int b1) { return (kNB4 - 1 - b1) * (kNB4 - 2 - b1) / 2; }

template <typename T, int B1>
__global__ void __launch_bounds__(kBlock) k_couple4(CoupleArgs a, int ptile)
{
    using V = typename C2<T>::type;
    constexpr int NA = pair_count(B1);
    constexpr int NR = kNB4 - B1;                         // bins b1..9 staged
    extern __shared__ __align__(16) unsigned char smem[];
    V* tile = reinterpret_cast<V*>(smem);
    const int per = NR * a.nlm;                           // staged complex values per primary
    double* wtile = reinterpret_cast<double*>(smem + sizeof(V) * (size_t)ptile * per);

    const int t = blockIdx.x * kBlock + threadIdx.x;
    const bool valid = t < a.ntuple;
    const int split = blockIdx.y;
    const int p_lo = a.split_lo[split];
    const int p_hi = a.split_hi[split];

    int lm0 = 0, lm1 = 0, lm2 = 0, flags = 0;
    if (valid) {
        lm0 = a.tuple_off[t * 3 + 0];
        lm1 = a.tuple_off[t * 3 + 1];
        lm2 = a.tuple_off[t * 3 + 2];
        flags = a.tuple_flags[t];
    }
    const T c0 = (flags & 1) ? (T)-1 : (T)1;
    const T c1 = (flags & 2) ? (T)-1 : (T)1;
    const T c2 = (flags & 4) ? (T)-1 : (T)1;
    const bool take_im = (flags >> 16) & 1;

    double acc[NA];
    T part[NA];
#pragma unroll
    for (int q = 0; q < NA; ++q) { acc[q] = 0.0; part[q] = (T)0; }

    for (int p0 = p_lo; p0 < p_hi; p0 += ptile) {
        const int np = min(ptile, p_hi - p0);
        __syncthreads();
        // stage bins B1..9 of each primary of the tile
        const V* src = reinterpret_cast<const V*>(a.alm);
        const int full = a.nbins * a.nlm;
        for (int q = threadIdx.x; q < np * per; q += kBlock) {
            const int pp = q / per, r = q - pp * per;
            tile[q] = src[(size_t)(p0 + pp) * full + B1 * a.nlm + r];
        }
        for (int q = threadIdx.x; q < np; q += kBlock) wtile[q] = a.wprim[p0 + q];
        __syncthreads();
        if (valid) {
            for (int pp = 0; pp < np; ++pp) {
                const V* ap = tile + pp * per;
                const T w = (T)wtile[pp];
                const V v0 = ap[lm0];
                const T a1r = w * v0.x, a1i = w * (c0 * v0.y);
                T u3r[NR], u3i[NR];
#pragma unroll
                for (int b = 2; b < NR; ++b) {
                    const V u = ap[b * a.nlm + lm2];
                    u3r[b] = u.x; u3i[b] = c2 * u.y;
                }
                int q = 0;
#pragma unroll
                for (int b2 = 1; b2 < NR - 1; ++b2) {
                    const V u = ap[b2 * a.nlm + lm1];
                    const T ur = u.x, ui = c1 * u.y;
                    T pr = a1r * ur - a1i * ui;
                    T pi = a1r * ui + a1i * ur;
                    if (take_im) { const T tmp = pr; pr = pi; pi = -tmp; }   // Im(z) = Re(-i z)
#pragma unroll
                    for (int b3 = b2 + 1; b3 < NR; ++b3) {
                        part[q] += pr * u3r[b3] - pi * u3i[b3];
                        ++q;
                    }
                }
            }
        }
#pragma unroll
        for (int q = 0; q < NA; ++q) { acc[q] += (double)part[q]; part[q] = (T)0; }
    }
    if (valid) {
        const double sgn = ((flags >> 8) & 1) ? -1.0 : 1.0;
        // B index of (B1, b2, b3): tuples with first bin < B1 come first
        int bidx = 0;
        for (int b = 0; b < B1; ++b) bidx += pair_count(b);
        double* dst = a.T + ((size_t)split * a.ntuple + t) * a.nB + bidx;
#pragma unroll
        for (int q = 0; q < NA; ++q) dst[q] = sgn * acc[q];
    }
}

__global__ void __launch_bounds__(kBlock) k_contract(ContractArgs a)
{
    const int64_t gid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (gid >= (int64_t)a.nlam * a.nB) return;
    const int l = (int)(gid / a.nB);
    const int b = (int)(gid - (int64_t)l * a.nB);
    double z = 0.0;
    for (int q = a.term_start[l]; q < a.term_start[l + 1]; ++q) {
        const int t = a.term_tuple[q];
        double s = 0.0;
        if (a.tmap) {
            const int32_t mv = a.tmap[(size_t)t * a.nB + b];
            s = a.T[mv & 0x7fffffff];
            if (mv < 0) s = -s;
        } else {
            for (int sp = 0; sp < a.nsplit; ++sp) s += a.T[((size_t)sp * a.ntuple + t) * a.nB + b];
        }
        z += a.term_coef[q] * s;
    }
    if (a.bscale) z *= a.bscale[b];
    a.zeta[gid] = z;
}

}  // namespace

int couple_split_rows(int nk, int nbins, int64_t ntuple, int64_t nB, int64_t nrows)
{
    int64_t ns;
    if (nk == 3 && nbins == kNB4) {
        // one block per (b1, 256 tuples, split): aim at ~1024 blocks per launch
        const int64_t tblocks = (ntuple + kBlock - 1) / kBlock;
        ns = (1024 + tblocks - 1) / std::max<int64_t>(tblocks, 1);
    } else {
        ns = (int64_t)(1 << 20) / std::max<int64_t>(ntuple * nB, 1);
    }
    ns = std::max<int64_t>(1, std::min<int64_t>(ns, 1024));
    int64_t rows = (nrows + ns - 1) / ns;
    return (int)std::max<int64_t>(64, rows);
}

__global__ void k_reduce(ReduceArgs a)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int r = blockIdx.y;
    if (i >= a.per) return;
    // left fold from the running total, split by split in row order: the same
    // association however the job's splits were distributed over slices
    double* dst = a.dst[r] + i;
    double s = *dst;
    for (int y = a.red_lo[r]; y < a.red_hi[r]; ++y) s += a.T[(size_t)y * a.per + i];
    *dst = s;
}

int launch_reduce(const ReduceArgs& a, hipStream_t stream)
{
    if (a.nred == 0 || a.per == 0) return (int)hipSuccess;
    k_reduce<<<dim3((unsigned)((a.per + kBlock - 1) / kBlock), (unsigned)a.nred), kBlock, 0, stream>>>(a);
    return (int)hipGetLastError();
}

int couple_ptile(int nbins, int nlm, int precision)
{
    const int per = nbins * nlm * (precision == 0 ? 16 : 8) + 8;
    int pt = 32768 / per;
    return pt < 1 ? 1 : (pt > 64 ? 64 : pt);
}

template <typename T, int B1>
void launch4(const CoupleArgs& a, int ptile, hipStream_t stream)
{
    const int nblk = (a.ntuple + kBlock - 1) / kBlock;
    const size_t lds = (size_t)ptile * (kNB4 - B1) * a.nlm * sizeof(typename C2<T>::type) + 8 * (size_t)ptile;
    k_couple4<T, B1><<<dim3((unsigned)nblk, (unsigned)a.nsplit), kBlock, lds, stream>>>(a, ptile);
}

template <typename T>
void launch4_all(const CoupleArgs& a, int ptile, hipStream_t stream)
{
    launch4<T, 0>(a, ptile, stream);
    launch4<T, 1>(a, ptile, stream);
    launch4<T, 2>(a, ptile, stream);
    launch4<T, 3>(a, ptile, stream);
    launch4<T, 4>(a, ptile, stream);
    launch4<T, 5>(a, ptile, stream);
    launch4<T, 6>(a, ptile, stream);
    launch4<T, 7>(a, ptile, stream);
    // bins 8 and 9 cannot be the first bin of a triple: their rows of T are absent
}

int launch_couple(const CoupleArgs& a, int precision, hipStream_t stream)
{
    if (a.nk > kMaxK) return (int)hipErrorInvalidValue;
    if (a.nsplit == 0 || a.ntuple == 0) return (int)hipSuccess;
    if (a.nk == 3 && a.nbins == kNB4) {
        const int ptile = std::max(1, std::min(64, 32768 / (kNB4 * a.nlm * (precision == 0 ? 16 : 8) + 8)));
        if (precision == 0) launch4_all<double>(a, ptile, stream);
        else launch4_all<float>(a, ptile, stream);
        return (int)hipGetLastError();
    }
    const int64_t nthreads = (int64_t)a.ntuple * a.nB;
    const int64_t nblk = (nthreads + kBlock - 1) / kBlock;
    if (nblk == 0) return (int)hipSuccess;
    const int ptile = couple_ptile(a.nbins, a.nlm, precision);
    const size_t lds = (size_t)ptile * a.nbins * a.nlm * (precision == 0 ? 16 : 8) + 8 * (size_t)ptile;
    dim3 grid((unsigned)nblk, (unsigned)a.nsplit);
#define ENCORE_COUPLE_CASE(NKV)                                                      \
    case NKV:                                                                        \
        if (precision == 0)                                                          \
            k_couple<double, NKV><<<grid, kBlock, lds, stream>>>(a, ptile);          \
        else                                                                         \
            k_couple<float, NKV><<<grid, kBlock, lds, stream>>>(a, ptile);           \
        break;
    switch (a.nk) {
        ENCORE_COUPLE_CASE(2)
        ENCORE_COUPLE_CASE(3)
        ENCORE_COUPLE_CASE(4)
        ENCORE_COUPLE_CASE(5)
    default: return (int)hipErrorInvalidValue;
    }
#undef ENCORE_COUPLE_CASE
    return (int)hipGetLastError();
}

int launch_contract(const ContractArgs& a, hipStream_t stream)
{
    const int64_t n = (int64_t)a.nlam * a.nB;
    if (n == 0) return (int)hipSuccess;
    k_contract<<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, stream>>>(a);
    return (int)hipGetLastError();
}

}  // namespace encore
