// Split-BF16 MFMA coupling on gfx950 (the reassociated contraction of eq.
// NPCF-mult-discrete-binned-estimator, Appendix B half sum).  The host plan
// (mfma_plan.cpp) lists wave jobs of up to four 16 x 16 output tiles:
//
//   D[tile][i][j] = sum_{primaries p} sum_{c in re, im} A[row_i][(p, c)] B[(p, c)][col_j]
//
// with A the (Re P, -Im P) or (Im P, Re P) parts of the row's product P of
// harmonic coefficients and B the (Re, Im) parts of w_p a~ of the column's last
// factor.  Both operands are split into bf16 hi + lo (hi = RNE(x), lo =
// RNE(x - hi)) and each tile takes three MFMAs per K block: hi*hi + hi*lo +
// lo*hi, accumulated in FP32 by the matrix cores and flushed into FP64
// registers every kFlushSteps K blocks; the dropped lo*lo term and the two
// representation errors are each below 2^-18 of |A B|.
//
// A block of 16 waves works on one split of primaries; every K block (16
// primaries) is staged once in LDS for all its waves: an FP32 plane of the
// coefficients (the row factors) and two packed bf16x2 planes (hi, lo) of
// w_p a~ (the columns), double buffered so that the global loads of the next K
// block overlap the MFMAs of this one.
#include <hip/hip_runtime.h>

#include "device.h"

namespace encore {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

constexpr int kMfWaves = 16;
constexpr int kMfThreads = kMfWaves * kWave;
constexpr int kStageP = 16;          // primaries per K block (K = 32 = 16 x (re, im))
constexpr int kAStride = 18;         // float2 per entry of the FP32 plane (16 + 2 pad)
constexpr int kBStride = 20;         // bf16x2 words per entry of a bf16 plane (16 + 4 pad)
constexpr int kStageBytesPerEntry = kAStride * 8 + 2 * kBStride * 4;
// staging: each thread moves (entry, pair of primaries) items; consecutive threads
// take consecutive entries, so the global reads are coalesced along a primary's
// row and the 16-byte LDS writes of 16 consecutive lanes land in 16 distinct bank
// slots (the entry stride is 9 slots of 16 bytes)
constexpr int kMaxStagePairs = (kStageP / 2 * kMfmaMaxEntries + kMfThreads - 1) / kMfThreads;
constexpr int kFlushSteps = 16;      // FP32 MFMA accumulation over 16 K blocks (256 primaries)

__device__ __forceinline__ unsigned pack_bf16(float x0, float x1)
{
    const bf16x2 h = {(__bf16)x0, (__bf16)x1};
    return __builtin_bit_cast(unsigned, h);
}
// float value of the low / high bf16 of a packed pair
__device__ __forceinline__ float bf16_lo(unsigned u) { return __uint_as_float(u << 16); }
__device__ __forceinline__ float bf16_hi(unsigned u) { return __uint_as_float(u & 0xffff0000u); }

// hi and lo bf16 pairs of (x0, x1)
__device__ __forceinline__ void split2(float x0, float x1, unsigned& hi, unsigned& lo)
{
    hi = pack_bf16(x0, x1);
    lo = pack_bf16(x0 - bf16_lo(hi), x1 - bf16_hi(hi));
}

__device__ __forceinline__ f32x4 mfma(u32x4 a, u32x4 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                   __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}

// ODD: some rows take the Im part (all-parity multiplets); otherwise every row
// takes the Re part and no per-row select is needed.
template <int KF, int RT, int NC, bool ODD>
__global__ void __launch_bounds__(kMfThreads) k_couple_mfma(MfmaArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int stage_bytes = a.nent * kStageBytesPerEntry;

    // blocks of one split run on one XCD (block b is placed on XCD b % 8), so the
    // split's coefficients are shared through that XCD's L2
    const int nbj = (a.njobs + kMfWaves - 1) / kMfWaves;
    const int li = blockIdx.x >> 3;
    const int split = (blockIdx.x & 7) + 8 * (li / nbj);
    const int bj = li % nbj;
    if (split >= a.nsplit) return;          // uniform over the block, before any barrier

    const int wid = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
    const int g = lane >> 4, c16 = lane & 15;
    const int job = bj * kMfWaves + wid;
    const bool active = job < a.njobs;      // wave-uniform

    int row_base = 0, col_base = 0, tile_base = 0, nrt = 0;
    if (active) {
        row_base = a.jobs[job * kMfmaJobWidth + 0];
        col_base = a.jobs[job * kMfmaJobWidth + 1];
        tile_base = a.jobs[job * kMfmaJobWidth + 2];
        nrt = a.jobs[job * kMfmaJobWidth + 3];
    }
    nrt = __builtin_amdgcn_readfirstlane(nrt);
    // this lane's row of each row tile: byte offsets of its factor entries in the
    // FP32 plane (entries are below kMfmaMaxEntries, offsets fit 16 bits, two per
    // word) and flags (conjugate bits 0..3, bit 4 = Im part), 5 flag bits per row
    // tile; padded rows and columns read entry 0, their outputs are never mapped
    constexpr int KW = (KF + 1) / 2;
    unsigned roff[RT][KW], rfl = 0;
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
        const int r = row_base + rt * 16 + c16;
#pragma unroll
        for (int k = 0; k < KW; ++k) roff[rt][k] = 0;
#pragma unroll
        for (int k = 0; k < KF; ++k) {
            const unsigned e = active ? (unsigned)a.rows[r * (KF + 1) + k] : 0u;
            roff[rt][k / 2] |= (e * kAStride * 8 + 32 * g) << (16 * (k & 1));
        }
        const unsigned f = active ? (unsigned)a.rows[r * (KF + 1) + KF] : 0u;
        rfl |= ((f & 15u) | (((f >> 8) & 1u) << 4)) << (5 * rt);
    }
    int coff[NC];
#pragma unroll
    for (int ct = 0; ct < NC; ++ct) {
        const int c = active ? a.cols[col_base + ct * 16 + c16] : 0;
        coff[ct] = (c < 0 ? 0 : c) * kBStride + 4 * g;
    }

    f32x4 acc[RT][NC];
    double acc64[RT][NC][4];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int ct = 0; ct < NC; ++ct) {
            acc[rt][ct] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int r = 0; r < 4; ++r) acc64[rt][ct][r] = 0.0;
        }

    const int p_lo = a.split_lo[split], p_hi = a.split_hi[split];
    const int nstep = (p_hi - p_lo + kStageP - 1) / kStageP;

    const int npair = kStageP / 2 * a.nent;   // (entry, primary pair) items per K block
    float4 sv[kMaxStagePairs];
    float2 sw[kMaxStagePairs];
    auto gload = [&](int st) {
        const int p0 = p_lo + st * kStageP;
#pragma unroll
        for (int q = 0; q < kMaxStagePairs; ++q) {
            const int idx = threadIdx.x + q * kMfThreads;
            sv[q] = make_float4(0.f, 0.f, 0.f, 0.f);
            sw[q] = make_float2(0.f, 0.f);
            if (idx < npair) {
                const int pp = idx / a.nent, e = idx - pp * a.nent;
                const int p = p0 + 2 * pp;
                if (p < p_hi) {
                    const float2 v = a.alm[(size_t)p * a.nent + e];
                    sv[q].x = v.x; sv[q].y = v.y;
                    sw[q].x = (float)a.wprim[p];
                }
                if (p + 1 < p_hi) {
                    const float2 v = a.alm[(size_t)(p + 1) * a.nent + e];
                    sv[q].z = v.x; sv[q].w = v.y;
                    sw[q].y = (float)a.wprim[p + 1];
                }
            }
        }
    };
    auto lstore = [&](unsigned char* buf) {
        float2* A = reinterpret_cast<float2*>(buf);
        unsigned* Bh = reinterpret_cast<unsigned*>(buf + (size_t)a.nent * kAStride * 8);
        unsigned* Bl = Bh + (size_t)a.nent * kBStride;
#pragma unroll
        for (int q = 0; q < kMaxStagePairs; ++q) {
            const int idx = threadIdx.x + q * kMfThreads;
            if (idx < npair) {
                const int pp = idx / a.nent, e = idx - pp * a.nent;
                *reinterpret_cast<float4*>(A + e * kAStride + 2 * pp) = sv[q];
                unsigned h0, l0, h1, l1;
                split2(sw[q].x * sv[q].x, sw[q].x * sv[q].y, h0, l0);
                split2(sw[q].y * sv[q].z, sw[q].y * sv[q].w, h1, l1);
                *reinterpret_cast<uint2*>(Bh + e * kBStride + 2 * pp) = make_uint2(h0, h1);
                *reinterpret_cast<uint2*>(Bl + e * kBStride + 2 * pp) = make_uint2(l0, l1);
            }
        }
    };

    if (nstep > 0) {
        gload(0);
        lstore(smem);
    }
    __syncthreads();
    for (int st = 0; st < nstep; ++st) {
        unsigned char* buf = smem + (size_t)(st & 1) * stage_bytes;
        if (st + 1 < nstep) gload(st + 1);
        if (active) {
            const float2* A = reinterpret_cast<const float2*>(buf);
            const unsigned* Bh = reinterpret_cast<const unsigned*>(buf + (size_t)a.nent * kAStride * 8);
            const unsigned* Bl = Bh + (size_t)a.nent * kBStride;
            u32x4 bh[NC], bl[NC];
#pragma unroll
            for (int ct = 0; ct < NC; ++ct) {
                bh[ct] = *reinterpret_cast<const u32x4*>(Bh + coff[ct]);
                bl[ct] = *reinterpret_cast<const u32x4*>(Bl + coff[ct]);
            }
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) {
                if (rt < nrt) {
                    // this lane's 4 primaries (4g .. 4g+3) of the row product
                    float pr[4], pi[4];
                    const unsigned fl = rfl >> (5 * rt);
                    {
                        const float2* src = reinterpret_cast<const float2*>(
                            reinterpret_cast<const unsigned char*>(A) + (roff[rt][0] & 0xffffu));
                        const float4 v0 = *reinterpret_cast<const float4*>(src);
                        const float4 v1 = *reinterpret_cast<const float4*>(src + 2);
                        const float s = (fl & 1u) ? -1.f : 1.f;
                        pr[0] = v0.x; pi[0] = s * v0.y; pr[1] = v0.z; pi[1] = s * v0.w;
                        pr[2] = v1.x; pi[2] = s * v1.y; pr[3] = v1.z; pi[3] = s * v1.w;
                    }
#pragma unroll
                    for (int k = 1; k < KF; ++k) {
                        const float2* src = reinterpret_cast<const float2*>(
                            reinterpret_cast<const unsigned char*>(A) + ((roff[rt][k / 2] >> (16 * (k & 1))) & 0xffffu));
                        const float4 v0 = *reinterpret_cast<const float4*>(src);
                        const float4 v1 = *reinterpret_cast<const float4*>(src + 2);
                        const float s = ((fl >> k) & 1u) ? -1.f : 1.f;
                        const float ur[4] = {v0.x, v0.z, v1.x, v1.z};
                        const float ui[4] = {s * v0.y, s * v0.w, s * v1.y, s * v1.w};
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const float nr = pr[q] * ur[q] - pi[q] * ui[q];
                            const float ni = pr[q] * ui[q] + pi[q] * ur[q];
                            pr[q] = nr; pi[q] = ni;
                        }
                    }
                    const bool im = ODD && ((fl >> 4) & 1u);
                    u32x4 ah, al;
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const float x0 = ODD ? (im ? pi[q] : pr[q]) : pr[q];
                        const float x1 = ODD ? (im ? pr[q] : -pi[q]) : -pi[q];
                        unsigned h, l;
                        split2(x0, x1, h, l);
                        ah[q] = h;
                        al[q] = l;
                    }
#pragma unroll
                    for (int ct = 0; ct < NC; ++ct) {
                        acc[rt][ct] = mfma(ah, bh[ct], acc[rt][ct]);
                        acc[rt][ct] = mfma(ah, bl[ct], acc[rt][ct]);
                        acc[rt][ct] = mfma(al, bh[ct], acc[rt][ct]);
                    }
                }
            }
            if ((st + 1) % kFlushSteps == 0 || st + 1 == nstep) {
#pragma unroll
                for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                    for (int ct = 0; ct < NC; ++ct) {
#pragma unroll
                        for (int r = 0; r < 4; ++r) acc64[rt][ct][r] += (double)acc[rt][ct][r];
                        acc[rt][ct] = f32x4{0.f, 0.f, 0.f, 0.f};
                    }
            }
        }
        if (st + 1 < nstep) lstore(smem + (size_t)((st + 1) & 1) * stage_bytes);
        __syncthreads();
    }
    if (!active) return;
    // output tile layout of the 16x16 MFMA: lane holds column c16, rows 4g .. 4g+3
    double* D = a.D + (size_t)split * a.dense;
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int ct = 0; ct < NC; ++ct) {
            double* t = D + (size_t)(tile_base + rt * NC + ct) * 256;
#pragma unroll
            for (int r = 0; r < 4; ++r) t[(4 * g + r) * 16 + c16] = acc64[rt][ct][r];
        }
}

template <int KF, int RT, int NC, bool ODD>
int launch_shape(const MfmaArgs& a, hipStream_t stream)
{
    const int nbj = (a.njobs + kMfWaves - 1) / kMfWaves;
    const int64_t groups = (a.nsplit + 7) / 8;
    const int64_t blocks = groups * 8 * nbj;
    if (blocks > INT32_MAX) return (int)hipErrorInvalidValue;
    const size_t lds = 2 * (size_t)a.nent * kStageBytesPerEntry;
    auto fn = k_couple_mfma<KF, RT, NC, ODD>;
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           2 * kMfmaMaxEntries * kStageBytesPerEntry);
        if (e != hipSuccess) return (int)e;
        attr_set = true;
    }
    fn<<<dim3((unsigned)blocks), dim3(kMfThreads), lds, stream>>>(a);
    return (int)hipGetLastError();
}

template <int KF, bool ODD>
int launch_kf(const MfmaArgs& a, int shape, hipStream_t stream)
{
    switch (shape) {
    case 0: return launch_shape<KF, 4, 1, ODD>(a, stream);
    case 1: return launch_shape<KF, 2, 2, ODD>(a, stream);
    case 2: return launch_shape<KF, 1, 3, ODD>(a, stream);
    case 3: return launch_shape<KF, 1, 4, ODD>(a, stream);
    }
    return (int)hipErrorInvalidValue;
}

}  // namespace

int mfma_stage_bytes(int nent) { return 2 * nent * kStageBytesPerEntry; }

int launch_couple_mfma(const MfmaArgs& a, int KF, int shape, hipStream_t stream)
{
    if (a.njobs == 0 || a.nsplit == 0) return (int)hipSuccess;
    if (a.nent < 1 || a.nent > kMfmaMaxEntries) return (int)hipErrorInvalidValue;
    switch (KF * 2 + (a.any_odd ? 1 : 0)) {
    case 2: return launch_kf<1, false>(a, shape, stream);
    case 3: return launch_kf<1, true>(a, shape, stream);
    case 4: return launch_kf<2, false>(a, shape, stream);
    case 5: return launch_kf<2, true>(a, shape, stream);
    case 6: return launch_kf<3, false>(a, shape, stream);
    case 7: return launch_kf<3, true>(a, shape, stream);
    case 8: return launch_kf<4, false>(a, shape, stream);
    case 9: return launch_kf<4, true>(a, shape, stream);
    }
    return (int)hipErrorInvalidValue;
}

}  // namespace encore
