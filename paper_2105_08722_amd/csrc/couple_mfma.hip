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
// A block of 16 waves works on one split of primaries.  The coefficients come in
// the blocked layout (16 primaries per block, 144 bytes per entry, weights in the
// padding); each K block is copied as it is from global memory to LDS by direct
// global-to-LDS loads, kStages - 1 K blocks ahead of the one in use, so the loads
// never pass through registers and their latency hides behind three K blocks of
// MFMAs.  Each wave forms its operands from the LDS copy: the row products (A) and
// w_p a~ of its columns (B), both split into bf16 hi + lo.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>
#include <vector>

#include "device.h"

namespace encore {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

constexpr int kMfWaves = 16;
constexpr int kMfThreads = kMfWaves * kWave;
constexpr int kStages = 4;           // K blocks resident in LDS (3 in flight while one is read)
constexpr int kEntBytes = kBlkEntFloats * 4;   // 144 bytes per entry of a block
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

// Block -> (split, job group) of a coupling launch of nsplit x nper blocks.  Splits
// in whole groups of 8 run one per XCD (block b is placed on XCD b % 8), so that the
// blocks of a split share its coefficients through that XCD's L2; the splits past
// the last whole group spread their blocks over all XCDs, so that a slice with
// fewer than 8 splits still fills the chip.
__device__ __forceinline__ void split_of_block(int nsplit, int nper, int& split, int& job)
{
    const int full = nsplit & ~7;
    const long long b = blockIdx.x, nfull = (long long)full * nper;
    if (b < nfull) {
        const int li = (int)(b >> 3);
        split = (int)(b & 7) + 8 * (li / nper);
        job = li % nper;
    } else {
        const long long r = b - nfull;
        split = full + (int)(r / nper);
        job = (int)(r % nper);
    }
}

// ODD: some rows take the Im part (all-parity multiplets); otherwise every row
// takes the Re part and no per-row select is needed.  GL: the K blocks are read
// where they lie in global memory (through the L2) instead of being staged in LDS,
// for blocks too large for the stages (more than kMfmaMaxEntries coefficients per
// primary).
template <int KF, int RT, int NC, bool ODD, bool GL>
__global__ void __launch_bounds__(kMfThreads) k_couple_mfma(MfmaArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int blk_b = a.ent_blk * kEntBytes;      // bytes of one K block
    const int units = (blk_b + 1023) >> 10;       // 1 KiB copy units (64 lanes x 16 bytes)
    const int stage_b = units << 10;

    const int nbj = (a.njobs + kMfWaves - 1) / kMfWaves;
    int split, bj;
    split_of_block(a.nsplit, nbj, split, bj);

    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);   // uniform per wave
    const int lane = threadIdx.x & (kWave - 1);
    const int g = lane >> 4, c16 = lane & 15;
    const int job = bj * kMfWaves + wid;
    const bool active = job < a.njobs;      // wave-uniform

    int row_base = 0, col_base = 0, tile_base = 0;
    if (active) {
        row_base = a.jobs[job * kMfmaJobWidth + 0];
        col_base = a.jobs[job * kMfmaJobWidth + 1];
        tile_base = a.jobs[job * kMfmaJobWidth + 2];
    }
    // this lane's row of each row tile: byte offsets of its factor entries in a K
    // block (staged blocks have at most kMfmaMaxEntries entries, so the offsets fit
    // 16 bits, two per word; GL keeps them whole) and flags (conjugate bits 0..3,
    // bit 4 = Im part), 5 flag bits per row tile; padded rows and columns read entry
    // 0, their outputs are never mapped
    constexpr int KW = GL ? KF : (KF + 1) / 2;
    unsigned roff[RT][KW], rfl = 0;
    auto row_off = [&](int rt, int k) -> unsigned {
        if constexpr (GL) return roff[rt][k];
        else return (roff[rt][k / 2] >> (16 * (k & 1))) & 0xffffu;
    };
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
        const int r = row_base + rt * 16 + c16;
#pragma unroll
        for (int k = 0; k < KW; ++k) roff[rt][k] = 0;
#pragma unroll
        for (int k = 0; k < KF; ++k) {
            const unsigned e = active ? (unsigned)a.rows[r * (KF + 1) + k] : 0u;
            if constexpr (GL) roff[rt][k] = e * kEntBytes + 32 * g;
            else roff[rt][k / 2] |= (e * kEntBytes + 32 * g) << (16 * (k & 1));
        }
        const unsigned f = active ? (unsigned)a.rows[r * (KF + 1) + KF] : 0u;
        rfl |= ((f & 15u) | (((f >> 8) & 1u) << 4)) << (5 * rt);
    }
    int coff[NC];
#pragma unroll
    for (int ct = 0; ct < NC; ++ct) {
        const int c = active ? a.cols[col_base + ct * 16 + c16] : 0;
        coff[ct] = (c < 0 ? 0 : c) * kEntBytes + 32 * g;
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

    // K blocks [kb0, kb1) cover the split's primaries [p_lo, p_hi); primaries of a
    // shared boundary block outside the split get weight 0 (their coefficients
    // are finite: other rows, or the zero padding of the last block)
    const int p_lo = a.split_lo[split], p_hi = a.split_hi[split];
    const int kb0 = p_lo / kBlkRows, kb1 = (p_hi + kBlkRows - 1) / kBlkRows;
    const int nstep = p_hi > p_lo ? kb1 - kb0 : 0;

    // Copies: wave wid moves units wid, wid + 16, ... of a K block; a wave issues
    // the same number of copies (ncp) for every K block, so "at most
    // (kStages - 2) * ncp copies of this wave outstanding" means the copies of the
    // K block kStages - 2 blocks back have landed.  Past the last K block the last
    // one is copied again (into a stage nobody reads), which keeps that count.
    const int ncp = units > wid ? (units - wid + kMfWaves - 1) / kMfWaves : 0;
    const unsigned char* gsrc = reinterpret_cast<const unsigned char*>(a.alm);
    auto copy_block = [&](int st) {
        const int kb = kb0 + (st < nstep ? st : nstep - 1);
        const unsigned char* src = gsrc + (size_t)kb * blk_b + lane * 16;
        unsigned char* dst = smem + (size_t)(st % kStages) * stage_b;
        for (int i = 0; i < ncp; ++i) {
            const int u = wid + kMfWaves * i;
            // LDS address = M0 + 16 * lane.  Issued as inline assembly: the compiler
            // cannot tell the stages of one LDS array apart and would otherwise
            // wait for every copy in flight before each LDS read; the waits are
            // explicit below (wait_copies and the end of the kernel).
            const unsigned m0 = (unsigned)(size_t)(dst + (u << 10));
            asm volatile("s_mov_b32 m0, %0\n\tglobal_load_lds_dwordx4 %1, off"
                         :
                         : "s"(m0), "v"(src + (u << 10))
                         : "memory", "m0");
        }
    };
    auto wait_copies = [&]() {
        // vmcnt <= (kStages - 2) * ncp; ncp <= 3 for blocks of <= 256 entries
        static_assert(kStages == 4, "copy wait counts assume 4 stages");
        switch (ncp) {
        case 0: asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); break;
        case 1: asm volatile("s_waitcnt vmcnt(2)" ::: "memory"); break;
        case 2: asm volatile("s_waitcnt vmcnt(4)" ::: "memory"); break;
        default: asm volatile("s_waitcnt vmcnt(6)" ::: "memory"); break;
        }
    };

    if (!GL && nstep > 0)
        for (int st = 0; st < kStages - 1; ++st) copy_block(st);
    for (int st = 0; st < nstep; ++st) {
        // this wave's copies of K block st have landed; after the barrier every
        // wave's have, and every wave has finished K block st - 1, whose stage the
        // next copy overwrites
        if constexpr (!GL) {
            wait_copies();
            asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
            copy_block(st + kStages - 1);
        }
        if (active) {
            const unsigned char* stg = GL ? gsrc + (size_t)(kb0 + st) * blk_b
                                          : smem + (size_t)(st % kStages) * stage_b;
            // weights of this lane's primaries 4g .. 4g+3 (padding of entry g)
            float4 w4 = *reinterpret_cast<const float4*>(stg + g * kEntBytes + 128);
            const int pb = (kb0 + st) * kBlkRows;
            if (pb < p_lo || pb + kBlkRows > p_hi) {
                const int p = pb + 4 * g;
                w4.x = (p + 0 >= p_lo && p + 0 < p_hi) ? w4.x : 0.f;
                w4.y = (p + 1 >= p_lo && p + 1 < p_hi) ? w4.y : 0.f;
                w4.z = (p + 2 >= p_lo && p + 2 < p_hi) ? w4.z : 0.f;
                w4.w = (p + 3 >= p_lo && p + 3 < p_hi) ? w4.w : 0.f;
            }
            // B operands: w a~ of the column entries, split into bf16 hi + lo
            u32x4 bh[NC], bl[NC];
#pragma unroll
            for (int ct = 0; ct < NC; ++ct) {
                const float4 v0 = *reinterpret_cast<const float4*>(stg + coff[ct]);
                const float4 v1 = *reinterpret_cast<const float4*>(stg + coff[ct] + 16);
                unsigned h, l;
                split2(w4.x * v0.x, w4.x * v0.y, h, l); bh[ct][0] = h; bl[ct][0] = l;
                split2(w4.y * v0.z, w4.y * v0.w, h, l); bh[ct][1] = h; bl[ct][1] = l;
                split2(w4.z * v1.x, w4.z * v1.y, h, l); bh[ct][2] = h; bl[ct][2] = l;
                split2(w4.w * v1.z, w4.w * v1.w, h, l); bh[ct][3] = h; bl[ct][3] = l;
            }
            const unsigned char* A = stg;
            // every row tile is formed, the job's invalid ones too (their rows are
            // padding that reads entry 0 and their tiles are never mapped): without a
            // branch per tile the compiler interleaves the tiles' LDS reads, VALU and
            // MFMAs
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) {
                // this lane's 4 primaries (4g .. 4g+3) of the row product
                float pr[4], pi[4];
                const unsigned fl = rfl >> (5 * rt);
                {
                    const float2* src = reinterpret_cast<const float2*>(A + row_off(rt, 0));
                    const float4 v0 = *reinterpret_cast<const float4*>(src);
                    const float4 v1 = *reinterpret_cast<const float4*>(src + 2);
                    const float s = (fl & 1u) ? -1.f : 1.f;
                    pr[0] = v0.x; pi[0] = s * v0.y; pr[1] = v0.z; pi[1] = s * v0.w;
                    pr[2] = v1.x; pi[2] = s * v1.y; pr[3] = v1.z; pi[3] = s * v1.w;
                }
#pragma unroll
                for (int k = 1; k < KF; ++k) {
                    const float2* src = reinterpret_cast<const float2*>(A + row_off(rt, k));
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
    }
    // no copy may still be writing LDS when the block ends
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
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
    const int64_t blocks = (int64_t)a.nsplit * nbj;
    if (blocks > INT32_MAX) return (int)hipErrorInvalidValue;
    if (a.nent > kMfmaMaxEntries) {
        k_couple_mfma<KF, RT, NC, ODD, true><<<dim3((unsigned)blocks), dim3(kMfThreads), 0, stream>>>(a);
        return (int)hipGetLastError();
    }
    const size_t stage_b = (blk_bytes(a.nent) + 1023) / 1024 * 1024;
    const size_t lds = kStages * stage_b;
    auto fn = k_couple_mfma<KF, RT, NC, ODD, false>;
    static bool attr_set = false;
    if (!attr_set) {
        const size_t max_lds = kStages * ((blk_bytes(kMfmaMaxEntries) + 1023) / 1024 * 1024);
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)max_lds);
        if (e != hipSuccess) return (int)e;
        attr_set = true;
    }
    fn<<<dim3((unsigned)blocks), dim3(kMfThreads), lds, stream>>>(a);
    return (int)hipGetLastError();
}

// ---------------------------------------------------------------- macro-tiled GEMM
// One workgroup per (split, macro tile) of the GEMM plan (mfma_plan.h).  Wave k
// forms operand tile k of the macro tile (its row tiles first: products of the
// first KL factors, Re or Im part; then its column tiles: w times the products of
// the other KR factors), split into bf16 hi + lo and stored in LDS in the MFMA lane
// order; wave w computes one 2 x 2 block of output tiles (three MFMAs each) from
// the shared operands, reading each of its two row and two column operand tiles
// once per K block.  The two are pipelined over two operand buffers: in one step a
// wave issues the MFMAs of K block st and forms its operand of K block st + 1, so
// one barrier per K block separates them.
constexpr int kGmWaves = kGemmMaxOps;
constexpr int kGmThreads = kGmWaves * kWave;
constexpr int kOpBytes = 2 * kWave * 16;           // one operand tile: hi and lo, 16 bytes per lane each
constexpr int kGmOpnd = kGemmMaxOps * kOpBytes;    // one operand buffer

// The product of NF factors for this lane's 4 primaries (4g .. 4g+3) from a staged K
// block, conjugating the factors flagged in fl.
template <int NF>
__device__ __forceinline__ void gemm_product(const unsigned char* stg, const int (&off)[NF], unsigned fl, float (&pr)[4],
                                             float (&pi)[4])
{
    {
        const float4 v0 = *reinterpret_cast<const float4*>(stg + off[0]);
        const float4 v1 = *reinterpret_cast<const float4*>(stg + off[0] + 16);
        const float s = (fl & 1u) ? -1.f : 1.f;
        pr[0] = v0.x; pi[0] = s * v0.y; pr[1] = v0.z; pi[1] = s * v0.w;
        pr[2] = v1.x; pi[2] = s * v1.y; pr[3] = v1.z; pi[3] = s * v1.w;
    }
#pragma unroll
    for (int k = 1; k < NF; ++k) {
        const float4 v0 = *reinterpret_cast<const float4*>(stg + off[k]);
        const float4 v1 = *reinterpret_cast<const float4*>(stg + off[k] + 16);
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
}

// GL: K blocks read in global memory, not staged (as for k_couple_mfma).
template <int KL, int KR, bool ODD, int ST, bool GL>
__global__ void __launch_bounds__(kGmThreads) k_couple_gemm(MfmaArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int blk_b = a.ent_blk * kEntBytes;      // bytes of one K block
    const int units = (blk_b + 1023) >> 10;       // 1 KiB copy units (64 lanes x 16 bytes)
    const int stage_b = units << 10;
    unsigned char* opnd = smem + (GL ? 0 : (size_t)ST * stage_b);   // two operand buffers of kGmOpnd bytes

    int split, mac;
    split_of_block(a.nsplit, a.njobs, split, mac);

    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int lane = threadIdx.x & (kWave - 1);
    const int g = lane >> 4, c16 = lane & 15;
    const int32_t* M = a.jobs + (size_t)mac * kGemmMacroWidth;
    const int row_start = M[0], col_start = M[1], MR = M[2], MC = M[3], tile_base = M[4];

    // formation role: operand tile wid (row tile wid, or column tile wid - MR).
    // Padding rows and columns read real entries; their outputs are never mapped.
    const bool forms = wid < MR + MC;
    const bool is_col = wid >= MR;
    int roff[KL], coff[KR];
    unsigned fl = 0;
#pragma unroll
    for (int k = 0; k < KL; ++k) roff[k] = 32 * g;
#pragma unroll
    for (int k = 0; k < KR; ++k) coff[k] = 32 * g;
    if (forms) {
        if (is_col) {
            const int32_t* c = a.cols + (size_t)(col_start + 16 * (wid - MR) + c16) * (KR + 1);
#pragma unroll
            for (int k = 0; k < KR; ++k) coff[k] = c[k] * kEntBytes + 32 * g;
            fl = (unsigned)c[KR];
        } else {
            const int32_t* r = a.rows + (size_t)(row_start + 16 * wid + c16) * (KL + 1);
#pragma unroll
            for (int k = 0; k < KL; ++k) roff[k] = r[k] * kEntBytes + 32 * g;
            fl = (unsigned)r[KL];
        }
    }
    // output role: the 2 x 2 block (bi, bj) of output tiles, rows tr0, tr0 + 1 and
    // columns tc0, tc0 + 1 of the macro tile, those inside it (wave-uniform)
    const int nbc = (MC + 1) / 2;
    const int bi = wid / nbc, bj = wid - bi * nbc;
    const int tr0 = 2 * bi, tc0 = 2 * bj;
    const int nr = bi < (MR + 1) / 2 ? min(2, MR - tr0) : 0;   // 0: no block for this wave
    const int nc = min(2, MC - tc0);
    // operand slots of the block's rows and columns; a row or column outside the
    // macro tile (and every operand of a wave without a block) reads a real operand
    // tile, and the tiles it feeds are never written
    const int r0 = nr > 0 ? tr0 : 0, c0 = nr > 0 ? tc0 : 0;
    const int aslot[2] = {r0 * kOpBytes + lane * 16, (nr == 2 ? r0 + 1 : r0) * kOpBytes + lane * 16};
    const int bslot[2] = {(MR + c0) * kOpBytes + lane * 16, (MR + (nc == 2 ? c0 + 1 : c0)) * kOpBytes + lane * 16};

    f32x4 acc[2][2];
    double acc64[2][2][4];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int r = 0; r < 4; ++r) acc64[i][j][r] = 0.0;
        }

    const int p_lo = a.split_lo[split], p_hi = a.split_hi[split];
    const int kb0 = p_lo / kBlkRows, kb1 = (p_hi + kBlkRows - 1) / kBlkRows;
    const int nstep = p_hi > p_lo ? kb1 - kb0 : 0;

    // Copies as in k_couple_mfma: wave wid moves units wid, wid + 16, ..., the same
    // number (ncp <= 3) for every K block.  K block st sits in stage st % ST; past
    // the last block the last one is copied again (into a stage nobody reads), which
    // keeps the count of copies per block.
    const int ncp = units > wid ? (units - wid + kGmWaves - 1) / kGmWaves : 0;
    const unsigned char* gsrc = reinterpret_cast<const unsigned char*>(a.alm);
    auto copy_block = [&](int st) {
        const int kb = kb0 + (st < nstep ? st : nstep - 1);
        const unsigned char* src = gsrc + (size_t)kb * blk_b + lane * 16;
        unsigned char* dst = smem + (size_t)(st % ST) * stage_b;
        for (int i = 0; i < ncp; ++i) {
            const int u = wid + kGmWaves * i;
            const unsigned m0 = (unsigned)(size_t)(dst + (u << 10));
            asm volatile("s_mov_b32 m0, %0\n\tglobal_load_lds_dwordx4 %1, off"
                         :
                         : "s"(m0), "v"(src + (u << 10))
                         : "memory", "m0");
        }
    };
    // this wave's copies of all but the last `behind` K blocks issued have landed
    auto wait_copies = [&](int behind) {
        switch (behind * ncp) {
        case 0: asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); break;
        case 1: asm volatile("s_waitcnt vmcnt(1)" ::: "memory"); break;
        case 2: asm volatile("s_waitcnt vmcnt(2)" ::: "memory"); break;
        case 3: asm volatile("s_waitcnt vmcnt(3)" ::: "memory"); break;
        case 4: asm volatile("s_waitcnt vmcnt(4)" ::: "memory"); break;
        case 5: asm volatile("s_waitcnt vmcnt(5)" ::: "memory"); break;
        default: asm volatile("s_waitcnt vmcnt(6)" ::: "memory"); break;
        }
    };
    static_assert(ST == 2 || ST == 3, "copy wait counts assume 2 or 3 stages");

    // forms this wave's operand of K block st (staged) into operand buffer st & 1;
    // EDGE: the split's first or last K block, whose primaries outside the split get
    // weight 0 (a block inside the split needs no such check, and its code is then
    // one basic block with the MFMAs of the step)
    auto form = [&](int st, auto edge) {
        constexpr bool EDGE = decltype(edge)::value;
        const unsigned char* stg = GL ? gsrc + (size_t)(kb0 + st) * blk_b : smem + (size_t)(st % ST) * stage_b;
        float pr[4], pi[4];
        u32x4 hi, lo;
        if (is_col) {
            gemm_product<KR>(stg, coff, fl, pr, pi);
            // weights of this lane's primaries 4g .. 4g+3 (padding of entry g); 0
            // for primaries of a boundary block outside the split
            float4 w4 = *reinterpret_cast<const float4*>(stg + g * kEntBytes + 128);
            const int pb = (kb0 + st) * kBlkRows;
            if (EDGE && (pb < p_lo || pb + kBlkRows > p_hi)) {
                const int p = pb + 4 * g;
                w4.x = (p + 0 >= p_lo && p + 0 < p_hi) ? w4.x : 0.f;
                w4.y = (p + 1 >= p_lo && p + 1 < p_hi) ? w4.y : 0.f;
                w4.z = (p + 2 >= p_lo && p + 2 < p_hi) ? w4.z : 0.f;
                w4.w = (p + 3 >= p_lo && p + 3 < p_hi) ? w4.w : 0.f;
            }
            const float ww[4] = {w4.x, w4.y, w4.z, w4.w};
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                unsigned h, l;
                split2(ww[q] * pr[q], ww[q] * pi[q], h, l);
                hi[q] = h;
                lo[q] = l;
            }
        } else {
            gemm_product<KL>(stg, roff, fl, pr, pi);
            const bool im = ODD && ((fl >> 8) & 1u);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const float x0 = ODD ? (im ? pi[q] : pr[q]) : pr[q];
                const float x1 = ODD ? (im ? pr[q] : -pi[q]) : -pi[q];
                unsigned h, l;
                split2(x0, x1, h, l);
                hi[q] = h;
                lo[q] = l;
            }
        }
        unsigned char* o = opnd + (size_t)(st & 1) * kGmOpnd + (size_t)wid * kOpBytes + lane * 16;
        *reinterpret_cast<u32x4*>(o) = hi;
        *reinterpret_cast<u32x4*>(o + kWave * 16) = lo;
    };

    if (nstep > 0) {
        if constexpr (!GL) {
            for (int st = 0; st < ST; ++st) copy_block(st);
            wait_copies(ST - 1);
            asm volatile("s_barrier" ::: "memory");
        }
        if (forms) form(0, std::true_type{});
    }
    for (int st = 0; st < nstep; ++st) {
        // After the barrier: every wave's operands of K block st are in buffer st & 1,
        // K block st + 1 is staged, and every wave is done with step st - 1 (its
        // MFMA reads of buffer (st + 1) & 1 and its reads of K block st's stage,
        // which the next copy overwrites).
        if constexpr (!GL) wait_copies(ST - 2);
        asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
        if constexpr (!GL) copy_block(st + ST);
        const unsigned char* ob = opnd + (size_t)(st & 1) * kGmOpnd;
        // the block's row and column operands, each read once, and the MFMAs of its
        // tiles inside the macro tile
        auto products = [&]() {
            if (nr == 0) return;                          // wave-uniform
            u32x4 ah[2], al[2], bh[2], bl[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                ah[i] = *reinterpret_cast<const u32x4*>(ob + aslot[i]);
                al[i] = *reinterpret_cast<const u32x4*>(ob + aslot[i] + kWave * 16);
                bh[i] = *reinterpret_cast<const u32x4*>(ob + bslot[i]);
                bl[i] = *reinterpret_cast<const u32x4*>(ob + bslot[i] + kWave * 16);
            }
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    if (i >= nr || j >= nc) continue;
                    acc[i][j] = mfma(ah[i], bh[j], acc[i][j]);
                    acc[i][j] = mfma(ah[i], bl[j], acc[i][j]);
                    acc[i][j] = mfma(al[i], bh[j], acc[i][j]);
                }
        };
        auto next = [&]() {
            if (!forms || st + 1 >= nstep) return;
            if (st + 2 < nstep) form(st + 1, std::false_type{});   // inside the split
            else form(st + 1, std::true_type{});                  // the split's last K block
        };
        // (half the waves taking the forming first, so that one SIMD's matrix core
        // and VALU would overlap after the barrier, measured slower: 100 ms against
        // 86 ms for the 6PCF at lmax 3 over 200k primaries)
        products();
        next();
        if ((st + 1) % kFlushSteps == 0 || st + 1 == nstep) {
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) acc64[i][j][r] += (double)acc[i][j][r];
                    acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
                }
        }
    }
    // no copy may still be writing LDS when the block ends
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    // output tile layout of the 16x16 MFMA: lane holds column c16, rows 4g .. 4g+3
    double* D = a.D + (size_t)split * a.dense + (size_t)tile_base * 256;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            if (i >= nr || j >= nc) continue;              // never written: outside the macro tile
            double* t = D + (size_t)((tr0 + i) * MC + tc0 + j) * 256;
#pragma unroll
            for (int r = 0; r < 4; ++r) t[(4 * g + r) * 16 + c16] = acc64[i][j][r];
        }
}

template <int KL, int KR, bool ODD>
int launch_gemm_shape(const MfmaArgs& a, hipStream_t stream)
{
    const int64_t blocks = (int64_t)a.nsplit * a.njobs;
    if (blocks > INT32_MAX) return (int)hipErrorInvalidValue;
    const size_t stage_b = (blk_bytes(a.nent) + 1023) / 1024 * 1024;
    const size_t opnd_b = 2 * (size_t)kGmOpnd;
    // three stages while they fit next to the two operand buffers in the 160 KiB of
    // LDS, else two (blocks of <= kMfmaMaxEntries entries: 37 KiB); larger blocks
    // are read in global memory
    const bool gl = a.nent > kMfmaMaxEntries;
    const bool three = !gl && 3 * stage_b + opnd_b <= (size_t)160 * 1024;
    if (!gl && !three && 2 * stage_b + opnd_b > (size_t)160 * 1024) return (int)hipErrorInvalidValue;
    const void* fn = gl      ? reinterpret_cast<const void*>(&k_couple_gemm<KL, KR, ODD, 2, true>)
                     : three ? reinterpret_cast<const void*>(&k_couple_gemm<KL, KR, ODD, 3, false>)
                             : reinterpret_cast<const void*>(&k_couple_gemm<KL, KR, ODD, 2, false>);
    const size_t lds = (gl ? 0 : (three ? 3 : 2) * stage_b) + opnd_b;
    static thread_local std::vector<const void*> raised;
    if (std::find(raised.begin(), raised.end(), fn) == raised.end()) {
        const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return (int)e;
        raised.push_back(fn);
    }
    MfmaArgs args = a;
    void* kargs[] = {&args};
    return (int)hipLaunchKernel(fn, dim3((unsigned)blocks), dim3(kGmThreads), kargs, lds, stream);
}

// One workgroup per 16-row block: the block's rows are read along the entries
// (coalesced), transposed through LDS in chunks of kToBlkChunk entries and written
// as one contiguous block.
constexpr int kToBlkThreads = 256;
constexpr int kToBlkChunk = 256;
__global__ void __launch_bounds__(kToBlkThreads) k_to_blocked(const float2* __restrict__ alm,
                                                              const double* __restrict__ wprim,
                                                              const GatherSeg* __restrict__ segs, int nseg,
                                                              int nrows, int nent, int ent_blk, float* out)
{
    __shared__ float2 tile[kBlkRows][kToBlkChunk + 1];
    __shared__ int valid[kBlkRows];
    const int r0 = blockIdx.x * kBlkRows;
    if (threadIdx.x < kBlkRows) {
        // the row belongs to the segment with the last row0 <= row (binary search)
        const int row = r0 + threadIdx.x;
        int ok = 0;
        if (row < nrows) {
            int lo = 0, hi = nseg - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (segs[mid].row0 <= row) lo = mid; else hi = mid - 1;
            }
            ok = row - segs[lo].row0 < segs[lo].nprim;
        }
        valid[threadIdx.x] = ok;
    }
    __syncthreads();
    float* ob = out + (size_t)blockIdx.x * ent_blk * kBlkEntFloats;
    for (int e0 = 0; e0 < ent_blk; e0 += kToBlkChunk) {
        const int ne = min(kToBlkChunk, ent_blk - e0);
        for (int i = threadIdx.x; i < kBlkRows * ne; i += kToBlkThreads) {
            const int r = i / ne, e = i - r * ne;
            tile[r][e] = (valid[r] && e0 + e < nent) ? alm[(size_t)(r0 + r) * nent + e0 + e] : make_float2(0.f, 0.f);
        }
        __syncthreads();
        for (int i = threadIdx.x; i < ne * kBlkEntFloats; i += kToBlkThreads) {
            const int e = i / kBlkEntFloats, f = i - e * kBlkEntFloats;
            float v = 0.f;
            if (f < 2 * kBlkRows) {
                const float2 c = tile[f >> 1][e];
                v = (f & 1) ? c.y : c.x;
            } else if (e0 + e < kBlkRows / 4) {
                const int r = 4 * (e0 + e) + (f - 2 * kBlkRows);
                v = valid[r] ? (float)wprim[r0 + r] : 0.f;
            }
            ob[(size_t)e0 * kBlkEntFloats + i] = v;
        }
        __syncthreads();
    }
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

int launch_to_blocked(const float2* alm, const double* wprim, const GatherSeg* segs, int nseg, int nrows,
                      int nent, float* out, hipStream_t stream)
{
    if (nrows <= 0) return (int)hipSuccess;
    if (nent < 1 || nent > kMfmaMaxAllEntries || nseg < 1) return (int)hipErrorInvalidValue;
    const int nblk = (nrows + kBlkRows - 1) / kBlkRows;
    k_to_blocked<<<dim3((unsigned)nblk), dim3(kToBlkThreads), 0, stream>>>(alm, wprim, segs, nseg, nrows, nent,
                                                                           blk_entries(nent), out);
    return (int)hipGetLastError();
}

int launch_couple_gemm(const MfmaArgs& a, int KL, int KR, hipStream_t stream)
{
    if (a.njobs == 0 || a.nsplit == 0) return (int)hipSuccess;
    if (a.nent < 1 || a.nent > kMfmaMaxAllEntries || a.ent_blk != blk_entries(a.nent))
        return (int)hipErrorInvalidValue;
    const bool odd = a.any_odd != 0;
    switch (KL * 10 + KR) {
    case 22: return odd ? launch_gemm_shape<2, 2, true>(a, stream) : launch_gemm_shape<2, 2, false>(a, stream);
    case 23: return odd ? launch_gemm_shape<2, 3, true>(a, stream) : launch_gemm_shape<2, 3, false>(a, stream);
    case 32: return odd ? launch_gemm_shape<3, 2, true>(a, stream) : launch_gemm_shape<3, 2, false>(a, stream);
    }
    return (int)hipErrorInvalidValue;
}

int launch_couple_mfma(const MfmaArgs& a, int KF, int shape, hipStream_t stream)
{
    if (a.njobs == 0 || a.nsplit == 0) return (int)hipSuccess;
    if (a.nent < 1 || a.nent > kMfmaMaxAllEntries || a.ent_blk != blk_entries(a.nent))
        return (int)hipErrorInvalidValue;
    switch (KF * 2 + (a.any_odd ? 1 : 0)) {
    case 2: return launch_kf<1, false>(a, shape, stream);
    case 3: return launch_kf<1, true>(a, shape, stream);
    case 4: return launch_kf<2, false>(a, shape, stream);
    case 5: return launch_kf<2, true>(a, shape, stream);
    }
    return (int)hipErrorInvalidValue;
}

}  // namespace encore
