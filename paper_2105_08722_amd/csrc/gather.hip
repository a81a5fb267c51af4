// Harmonic-coefficient gather on gfx950 (eq. binned-discrete-alm, without 1/v_b):
//
//   a~^b_lm(i) = sum_{j != i} w_j Y_lm((r_j - s_i)^) Theta^b(|r_j - s_i|)
//
// One wavefront owns one work item = (primary, group of radial bins, range of m).
//
//  1. Row set-up, lane-parallel: every lane takes one (y, z) row of cells that can
//     hold a secondary of the group's shell [R_in, R_out) and clips the row's x
//     extent to the shell's chord (minus the inner hole where the whole row is
//     inside R_in), splitting at periodic images.  Because particles are sorted by
//     cell with x fastest, each clipped piece is one contiguous particle range;
//     pieces without a periodic image come first.
//  2. Candidate test, 64 candidates per step: separation in FP64 exactly as the
//     definition orders it (x_j - x_i, then the periodic image), r^2 =
//     (dx*dx + dy*dy) + dz*dz without contraction, bin by comparing r^2 with the
//     squared edges.  Accepted pairs are pushed into one LDS ring per bin (slots
//     from lane-mask ballots and mbcnt ranks, no atomics).
//  3. Drain: whenever a ring holds 64 pairs, all 64 lanes pop one pair each, form
//     Y_lm by the monic Legendre recurrence in z times (x + i y)^m and add w Y into
//     per-lane register accumulators of that bin (the bin is wave-uniform, so the
//     register index is static).
//  4. Reduce the 64 lanes' accumulators (FP32: cross-lane swaps and row
//     rotations, then staged in LDS; FP64: through LDS), scale by the recurrence
//     normalisation kappa_lm and write the complex coefficients.
//
// Primaries are read from the segment's primary array (the catalog's own points,
// or another grid's), candidates from its cell-sorted points; lanes past the last
// candidate take the grid's NaN sentinel points, which no bin accepts.
//
// Y_lm = N_lm(z) (x + i y)^m for a unit vector (Condon-Shortley phase inside N_lm);
// N_lm = kappa_lm R_lm with R_mm = 1, R_{m+1,m} = z, R_lm = z R_{l-1,m} - gamma_lm R_{l-2,m}.
#include <hip/hip_runtime.h>
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <type_traits>
#include <utility>
#include <vector>

#include "device.h"

namespace encore {

namespace {

constexpr int kCap = 128;          // ring capacity per bin (pairs)
constexpr int kRowsPerBatch = 64;  // rows set up per lane-parallel pass
constexpr int kSegPerRow = 6;      // <= 2 x-ranges x 3 periodic images
constexpr int kSegCap = kRowsPerBatch * kSegPerRow;
// Waves of a block are independent (no block barriers); they take the same bin
// group of kWavesPerBlock consecutive rows, so nearly the same candidate stream
// runs on one compute unit and its vector L1 serves the repeats.
constexpr int kWavesPerBlock = 4;
constexpr int kRedCh = 16;         // accumulator values per pass of the lane reduction

__host__ __device__ constexpr int nlm_of(int L) { return (L + 1) * (L + 2) / 2; }
__host__ __device__ constexpr int lm_index(int l, int m) { return l * (l + 1) / 2 + m; }
__host__ __device__ constexpr int m_of_lm(int lm)
{
    int l = 0;
    while (lm_index(l + 1, 0) <= lm) ++l;
    return lm - lm_index(l, 0);
}

template <typename T> struct Entry;
template <> struct Entry<float> { using type = float4; };
template <> struct Entry<double> { using type = double4; };

template <typename T> __device__ __forceinline__ T rsqrt_t(T v);
template <> __device__ __forceinline__ float rsqrt_t<float>(float v) { return __builtin_amdgcn_rsqf(v); }
template <> __device__ __forceinline__ double rsqrt_t<double>(double v) { return 1.0 / sqrt(v); }

// LDS of one wave: the per-bin rings plus one dump entry per lane (reused as the
// reduction scratch, whose values are FP64 for the FP64 accumulators of the FP64
// and the FP32 paths) and the piece descriptors of one row batch.
template <typename T, int NBG, bool COMP>
__host__ __device__ constexpr int ring_bytes()
{
    constexpr int red = kRedCh * 65 * ((COMP || sizeof(T) == 8) ? 8 : 4);
    constexpr int ring = (NBG * kCap + kWave) * (int)sizeof(typename Entry<T>::type);
    return ring > red ? ring : red;
}
template <typename T, int NBG, bool COMP>
__host__ __device__ constexpr int wave_lds_bytes()
{
    // ring | seg_dl[kSegCap] seg_flat[kSegCap + 1]
    return ring_bytes<T, NBG, COMP>() + 4 * (2 * kSegCap + 4);
}

// Square root by Newton's iteration, for the compile-time tables below.
constexpr double ce_sqrt(double x)
{
    if (!(x > 0.0)) return 0.0;
    double r = x < 1.0 ? 1.0 : x;
    for (int i = 0; i < 200; ++i) {
        const double n = 0.5 * (r + x / r);
        if (n == r) break;
        r = n;
    }
    return r;
}

// Recurrence coefficients of the normalised associated Legendre functions,
// R_lm = z R_{l-1,m} - gamma_lm R_{l-2,m} (l >= m + 2), with
// gamma_lm = b_lm kappa_{l-2,m} / kappa_{l-1,m} (kappa, a and b as in gather_tables):
// the ratio is 1 / sqrt(2m + 3) for l = m + 2 and 1 / a_{l-1,m} above.  Zero for l < m + 2.
template <int L>
struct GammaTable {
    double v[nlm_of(L)];
    constexpr GammaTable() : v{}
    {
        for (int m = 0; m <= L; ++m)
            for (int l = m + 2; l <= L; ++l) {
                const double l1 = l - 1;
                const double bl = ce_sqrt((l1 * l1 - (double)m * m) / (4.0 * l1 * l1 - 1.0));
                const double den = (l == m + 2) ? ce_sqrt(2.0 * m + 3.0)
                                                : ce_sqrt((4.0 * l1 * l1 - 1.0) / (l1 * l1 - (double)m * m));
                v[lm_index(l, m)] = bl / den;
            }
    }
};
template <int L> struct Gamma { static constexpr GammaTable<L> t{}; };

// Final scales kappa_lm of the recurrence (the values gather_tables computes):
// kappa_mm = (-1)^m c_m, c_0 = 1/sqrt(4 pi), c_m = c_{m-1} sqrt((2m+1)/(2m)),
// kappa_{m+1,m} = sqrt(2m+3) kappa_mm, kappa_lm = a_lm kappa_{l-1,m} (l >= m+2).
template <int L>
struct KappaTable {
    double v[nlm_of(L)];
    constexpr KappaTable() : v{}
    {
        double c = 1.0 / ce_sqrt(4.0 * 3.14159265358979323846);
        for (int m = 0; m <= L; ++m) {
            if (m > 0) c *= ce_sqrt((2.0 * m + 1.0) / (2.0 * m));
            const double kmm = (m % 2) ? -c : c;
            v[lm_index(m, m)] = kmm;
            if (m + 1 <= L) v[lm_index(m + 1, m)] = ce_sqrt(2.0 * m + 3.0) * kmm;
            for (int l = m + 2; l <= L; ++l)
                v[lm_index(l, m)] = ce_sqrt((4.0 * l * l - 1.0) / ((double)l * l - (double)m * m)) *
                                    v[lm_index(l - 1, m)];
        }
    }
};
template <int L> struct Kappa { static constexpr KappaTable<L> t{}; };

// Accumulator type: T, or with COMP (T = float) FP64: the terms w Y_lm are formed in
// FP32 and each is added exactly into an FP64 sum, so a lane's sum of many pairs
// keeps no rounding of its own beyond the terms' (the data-minus-randoms terms cancel
// inside each coefficient, and FP32 sums would lose that difference).
template <typename T, bool COMP>
using AccT = typename std::conditional<COMP, double, T>::type;

// Add w*Y_lm for m in [M0, M1] of one pair into acc (layout [lm][re, im]).
template <typename T, int L, int M0, int M1, bool COMP>
__device__ __forceinline__ void accum_pair(T dx, T dy, T dz, T w, AccT<T, COMP> (&acc)[nlm_of(L)][2])
{
    const T r2 = dx * dx + dy * dy + dz * dz;
    const T inv = rsqrt_t<T>(r2);
    const T x = dx * inv, y = dy * inv, z = dz * inv;
    const T zw = z * w;
    T ur = (T)1, ui = (T)0;
#pragma unroll
    for (int m = 1; m <= M0; ++m) {   // (x + i y)^M0
        const T nr = ur * x - ui * y;
        const T ni = ur * y + ui * x;
        ur = nr; ui = ni;
    }
#pragma unroll
    for (int m = M0; m <= M1; ++m) {
        if (m > M0) {
            if (m == 1) { ur = x; ui = y; }
            else {
                const T nr = ur * x - ui * y;
                const T ni = ur * y + ui * x;
                ur = nr; ui = ni;
            }
        }
        T r0 = w, r1 = zw;
        if constexpr (COMP) {
            // each recurrence value and (x + i y)^m widened once, one FP64 FMA per term
            const double urd = ur, uid = ui;
            auto put = [&](int l, T rn) {
                const double rd = rn;
                if (m == 0) {
                    acc[lm_index(l, 0)][0] += rd;
                } else {
                    acc[lm_index(l, m)][0] = fma(rd, urd, acc[lm_index(l, m)][0]);
                    acc[lm_index(l, m)][1] = fma(rd, uid, acc[lm_index(l, m)][1]);
                }
            };
            put(m, r0);
            if (m + 1 <= L) put(m + 1, r1);
#pragma unroll
            for (int l = m + 2; l <= L; ++l) {
                const T rn = z * r1 - (T)Gamma<L>::t.v[lm_index(l, m)] * r0;
                put(l, rn);
                r0 = r1; r1 = rn;
            }
        } else {
            if (m == 0) {
                acc[lm_index(0, 0)][0] += r0;
                if (L >= 1) acc[lm_index(1, 0)][0] += r1;
            } else {
                acc[lm_index(m, m)][0] += r0 * ur;
                acc[lm_index(m, m)][1] += r0 * ui;
                if (m + 1 <= L) {
                    acc[lm_index(m + 1, m)][0] += r1 * ur;
                    acc[lm_index(m + 1, m)][1] += r1 * ui;
                }
            }
#pragma unroll
            for (int l = m + 2; l <= L; ++l) {
                const T rn = z * r1 - (T)Gamma<L>::t.v[lm_index(l, m)] * r0;
                if (m == 0) {
                    acc[lm_index(l, 0)][0] += rn;
                } else {
                    acc[lm_index(l, m)][0] += rn * ur;
                    acc[lm_index(l, m)][1] += rn * ui;
                }
                r0 = r1; r1 = rn;
            }
        }
    }
}

// Separation and squared distance exactly as the definition orders the FP64
// operations: (x_j - x_i) + image shift, then (dx*dx + dy*dy) + dz*dz, with no
// fused multiply-add anywhere (the bin decision must match the definition bit for
// bit).  The image shift is exactly +-L or 0.
__device__ __forceinline__ double sep(double xj, double xi, double shift)
{
#pragma clang fp contract(off)
    return (xj - xi) + shift;
}
__device__ __forceinline__ double diff(double xj, double xi)
{
#pragma clang fp contract(off)
    return xj - xi;
}
__device__ __forceinline__ double dist2(double dx, double dy, double dz)
{
#pragma clang fp contract(off)
    return (dx * dx + dy * dy) + dz * dz;
}

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// wave-uniform copies (the value must already be uniform)
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ double uni(double v)
{
    const unsigned long long u = __double_as_longlong(v);
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)u);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(u >> 32));
    return __longlong_as_double(((unsigned long long)hi << 32) | lo);
}

template <typename PT>
__device__ __forceinline__ PT* uni(PT* v)
{
    const unsigned long long u = (unsigned long long)v;
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)u);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(u >> 32));
    return (PT*)(((unsigned long long)hi << 32) | lo);
}

// Catalog and cell-table pointers come from a descriptor in memory, so the
// compiler cannot tell their address space and would emit flat loads; flat loads
// count against the LDS wait counter too, which would make every LDS wait in the
// candidate loop also wait for the next chunk's prefetch.  Loads through these
// pointers are global loads.
template <typename T> using gptr = const __attribute__((address_space(1))) T*;
template <typename T> __device__ __forceinline__ gptr<T> as_global(const T* p) { return (gptr<T>)p; }
__device__ __forceinline__ double4 load_point(gptr<double4> p, int j)
{
    const gptr<double> d = (gptr<double>)p + 4 * (int64_t)j;
    return make_double4(d[0], d[1], d[2], d[3]);
}

// a segment descriptor with every field made wave-uniform (SGPRs)
__device__ __forceinline__ GatherSeg load_seg(const GatherSeg* segs, int s)
{
    GatherSeg g = segs[s];
    g.P = uni(g.P);
    g.cell_start = uni(g.cell_start);
    g.prim = uni(g.prim);
    g.ncx = uni(g.ncx); g.ncy = uni(g.ncy); g.ncz = uni(g.ncz); g.periodic = uni(g.periodic);
    g.ox = uni(g.ox); g.oy = uni(g.oy); g.oz = uni(g.oz);
    g.csx = uni(g.csx); g.csy = uni(g.csy); g.csz = uni(g.csz);
    g.Lx = uni(g.Lx); g.Ly = uni(g.Ly); g.Lz = uni(g.Lz);
    g.Pq = uni(g.Pq);
    g.row0 = uni(g.row0); g.nprim = uni(g.nprim); g.nP = uni(g.nP);
    g.icsx = uni(g.icsx); g.icsy = uni(g.icsy); g.icsz = uni(g.icsz);
    g.cull_pad = uni(g.cull_pad); g.frame_eps = uni(g.frame_eps);
    return g;
}

// Exclusive wave scan by DPP: shifts by 1, 2, 4, 8 inside each row of 16 lanes
// (lanes without a source add 0), then row 0's total into rows 1 and 3 and the
// total of rows 0-1 into rows 2 and 3 (row broadcasts of lanes 15 and 31).
__device__ __forceinline__ int wave_excl_scan(int v, int* total)
{
    int incl = v;
    incl += __builtin_amdgcn_update_dpp(0, incl, 0x111, 0xf, 0xf, false);   // row_shr:1
    incl += __builtin_amdgcn_update_dpp(0, incl, 0x112, 0xf, 0xf, false);   // row_shr:2
    incl += __builtin_amdgcn_update_dpp(0, incl, 0x114, 0xf, 0xf, false);   // row_shr:4
    incl += __builtin_amdgcn_update_dpp(0, incl, 0x118, 0xf, 0xf, false);   // row_shr:8
    incl += __builtin_amdgcn_update_dpp(0, incl, 0x142, 0xa, 0xf, false);   // row_bcast:15
    incl += __builtin_amdgcn_update_dpp(0, incl, 0x143, 0xc, 0xf, false);   // row_bcast:31
    *total = __builtin_amdgcn_readlane(incl, kWave - 1);
    return incl - v;
}

constexpr int kCodeShift = 26;               // segment start | (image code << 26)
constexpr int kStartMask = (1 << kCodeShift) - 1;
constexpr int kCenterCode = 1 | (1 << 2) | (1 << 4);   // no periodic image on any axis

// Uniform inputs of the row set-up in precision R: primary position relative to
// the grid origin, cell sizes and their reciprocals, the culling sphere radius and
// inner-hole radius (widened / shrunk by the margin eps), the row range.
template <typename R>
struct RowFrame {
    R px, py, pz, csx, csy, csz, icsx, eps, Rc2, R2in;
    int ky0, kz0, nyr;
    float inv_nyr;
};

template <typename R>
__device__ __forceinline__ RowFrame<R> make_frame(const GatherSeg& g, double xi, double yi, double zi,
                                                 double Rin, double Rout, int ky0, int kz0, int nyr)
{
    RowFrame<R> f;
    const double eps = g.frame_eps;
    f.px = (R)(xi - g.ox); f.py = (R)(yi - g.oy); f.pz = (R)(zi - g.oz);
    f.csx = (R)g.csx; f.csy = (R)g.csy; f.csz = (R)g.csz;
    f.icsx = (R)g.icsx;
    f.eps = (R)eps;
    const double rc = Rout + eps;
    f.Rc2 = (R)(rc * rc);
    const double rin = fmax(0.0, Rin - eps);
    f.R2in = (R)(rin * rin);
    f.ky0 = ky0; f.kz0 = kz0; f.nyr = nyr;
    f.inv_nyr = __builtin_amdgcn_rcpf((float)max(nyr, 1));
    return f;
}

// One cell row (lane's row r of the primary's row range): its x extent clipped to
// the culling sphere's chord, minus the inner hole where the whole row is inside
// it.  Row, cell and image indices stay within one period of the grid because the
// largest separation is at most half the box.
struct RowGeom {
    int rowbase, code_yz;
    int lo[2], hi[2];   // unwrapped x cell ranges, left and right of the hole (lo > hi: none)
};

template <typename R>
__device__ __forceinline__ RowGeom row_geom(const RowFrame<R>& f, const GatherSeg& g, int r)
{
    RowGeom rg;
    rg.lo[0] = rg.lo[1] = 1;
    rg.hi[0] = rg.hi[1] = 0;
    rg.rowbase = 0;
    rg.code_yz = 0;
    // r / nyr: with inv_nyr within 1 ulp of 1 / nyr the float product stays within
    // 2^-22 relative of (r + 0.5) / nyr, whose distance from an integer is at least
    // 0.5 / nyr, so its floor is exact for r + 0.5 < 2^21
    const int rz = r < (1 << 20) ? (int)(((float)r + 0.5f) * f.inv_nyr) : r / f.nyr;
    const int ky = f.ky0 + (r - rz * f.nyr), kz = f.kz0 + rz;
    int wy = ky, wz = kz, sy = 0, sz = 0;
    if (g.periodic) {
        sy = ky < 0 ? -1 : (ky >= g.ncy ? 1 : 0);
        sz = kz < 0 ? -1 : (kz >= g.ncz ? 1 : 0);
        wy = ky - sy * g.ncy;
        wz = kz - sz * g.ncz;
    }
    const R ylo = (R)ky * f.csy - f.eps, yhi = (R)(ky + 1) * f.csy + f.eps;
    const R zlo = (R)kz * f.csz - f.eps, zhi = (R)(kz + 1) * f.csz + f.eps;
    const R dymin = fmax((R)0, fmax(ylo - f.py, f.py - yhi));
    const R dzmin = fmax((R)0, fmax(zlo - f.pz, f.pz - zhi));
    const R rho2 = dymin * dymin + dzmin * dzmin;
    if (!(rho2 < f.Rc2)) return rg;
    const R h = sqrt(f.Rc2 - rho2) + f.eps;
    int kx0 = (int)floor((f.px - h) * f.icsx), kx1 = (int)floor((f.px + h) * f.icsx);
    if (!g.periodic) { kx0 = max(kx0, 0); kx1 = min(kx1, g.ncx - 1); }
    const R dymax = fmax(fabs(ylo - f.py), fabs(yhi - f.py));
    const R dzmax = fmax(fabs(zlo - f.pz), fabs(zhi - f.pz));
    const R rhomax2 = dymax * dymax + dzmax * dzmax;
    int kin0 = 1, kin1 = 0;
    if (f.R2in > (R)0 && rhomax2 < f.R2in) {
        const R hin = sqrt(f.R2in - rhomax2) - f.eps;
        if (hin > (R)0) {
            kin0 = (int)ceil((f.px - hin) * f.icsx);
            kin1 = (int)floor((f.px + hin) * f.icsx) - 1;
        }
    }
    rg.rowbase = (wz * g.ncy + wy) * g.ncx;
    rg.code_yz = ((sy + 1) << 2) | ((sz + 1) << 4);
    if (kin0 <= kin1) {
        rg.lo[0] = kx0; rg.hi[0] = min(kx1, kin0 - 1);
        rg.lo[1] = max(kx0, kin1 + 1); rg.hi[1] = kx1;
    } else {
        rg.lo[0] = kx0; rg.hi[0] = kx1;
    }
    return rg;
}

// periodic image range (-1, 0, +1) of the cells [lo, hi]
__device__ __forceinline__ void image_range(const GatherSeg& g, int lo, int hi, int& sxa, int& sxb)
{
    sxa = 0; sxb = 0;
    if (g.periodic) {
        sxa = lo < 0 ? -1 : (lo >= g.ncx ? 1 : 0);
        sxb = hi < 0 ? -1 : (hi >= g.ncx ? 1 : 0);
    }
}

// Pieces of a row: one per x range and periodic image (<= kSegPerRow), empty ones
// included, split into centre pieces (no periodic image on any axis) and image
// pieces.  Counted (nc, ni), then written to two slot ranges, so that a batch's
// flat positions hold all centre pieces first: entry of the first candidate
// (start | image code) and length.  Because particles are sorted by cell with x
// fastest, each piece is one contiguous particle range.
__device__ __forceinline__ void row_pieces_split(const RowGeom& rg, const GatherSeg& g, int& nc, int& ni)
{
    nc = 0;
    ni = 0;
    const bool yz_centre = rg.code_yz == ((1 << 2) | (1 << 4));
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        if (rg.lo[q] > rg.hi[q]) continue;
        int sxa, sxb;
        image_range(g, rg.lo[q], rg.hi[q], sxa, sxb);
        const int c = (yz_centre && sxa <= 0 && sxb >= 0) ? 1 : 0;
        nc += c;
        ni += sxb - sxa + 1 - c;
    }
}
__device__ __forceinline__ void emit_pieces_split(const RowGeom& rg, const GatherSeg& g, gptr<int32_t> gcs,
                                                  int sc, int si, unsigned* ent, int* len, int& nlc, int& nli)
{
    nlc = 0;
    nli = 0;
    const bool yz_centre = rg.code_yz == ((1 << 2) | (1 << 4));
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        if (rg.lo[q] > rg.hi[q]) continue;
        int sxa, sxb;
        image_range(g, rg.lo[q], rg.hi[q], sxa, sxb);
        for (int sx = sxa; sx <= sxb; ++sx) {
            const int plo = max(rg.lo[q], sx * g.ncx) - sx * g.ncx;
            const int phi = min(rg.hi[q], sx * g.ncx + g.ncx - 1) - sx * g.ncx;
            const int st = gcs[rg.rowbase + plo];
            const int en = gcs[rg.rowbase + phi + 1];
            const bool centre = yz_centre && sx == 0;
            const int k = centre ? sc++ : si++;
            ent[k] = (unsigned)st | ((unsigned)((sx + 1) | rg.code_yz) << kCodeShift);
            len[k] = en - st;
            if (centre) nlc += en - st; else nli += en - st;
        }
    }
}

// waves per SIMD the kernel is compiled for, from its accumulator registers
template <typename T, int L, int NBG, int M0, int M1, bool COMP>
__host__ __device__ constexpr int gather_wpe()
{
    constexpr int acc = NBG * ((L + 1) * (L + 1)) * (int)(sizeof(T) / 4) * (COMP ? 2 : 1);
    return acc <= 72 ? 4 : 2;
}

// PERS: persistent grid (work items pulled from queues); otherwise one item per wave.
// COMP (T = float only): FP32 terms summed in FP64 accumulators, reduced in FP64.
template <typename T, int L, int NBG, int M0, int M1, bool PERS, bool COMP>
__global__ void __launch_bounds__(kWave * kWavesPerBlock, (gather_wpe<T, L, NBG, M0, M1, COMP>())) k_gather(GatherArgs a)
{
    static_assert(!COMP || std::is_same_v<T, float>, "FP64 accumulation of FP32 terms is for FP32");
    using E = typename Entry<T>::type;
    using RT = typename std::conditional<COMP, double, T>::type;   // lane reduction type
    constexpr int NLM = nlm_of(L);
    constexpr int CH = kRedCh;
    extern __shared__ __align__(16) unsigned char smem[];

    const int lane = threadIdx.x & (kWave - 1);
    const int wib = threadIdx.x / kWave;
    unsigned char* base = smem + wib * wave_lds_bytes<T, NBG, COMP>();
    E* ring = reinterpret_cast<E*>(base);
    RT* scratch = reinterpret_cast<RT*>(base);
    unsigned* seg_dl = reinterpret_cast<unsigned*>(base + ring_bytes<T, NBG, COMP>());
    int* seg_flat = reinterpret_cast<int*>(seg_dl + kSegCap);


    // Item j -> quad j / kWavesPerBlock = (row block, bin group), row = block *
    // kWavesPerBlock + j % kWavesPerBlock.  Rows are cell-sorted primaries, so the
    // waves of one quad scan almost the same cells.  A static grid gives each XCD
    // (block b runs on XCD b % 8) a contiguous run of quads, so neighbouring
    // primaries share that XCD's L2; the persistent grid pulls items from 8
    // contiguous queues the same way.
    const int64_t nquads = ((int64_t)a.nrows + kWavesPerBlock - 1) / kWavesPerBlock * a.ngroups;
    const int64_t nitems = nquads * kWavesPerBlock;
    const int home = blockIdx.x & 7;
    auto pop = [&]() -> int64_t {
        for (int t = 0; t < 8; ++t) {
            const int qi = (home + t) & 7;
            const int64_t lo = nitems * qi / 8, hi = nitems * (qi + 1) / 8;
            unsigned got = 0;
            if (lane == 0) got = atomicAdd(&a.queues[qi], 1u);
            got = __builtin_amdgcn_readfirstlane(got);
            if (lo + (int64_t)got < hi) return lo + (int64_t)got;
        }
        return -1;
    };
    // One work item.  The persistent kernel calls it in a loop, the static kernel
    // once: there nothing is hoisted out of an item loop, which keeps values that
    // only the end of the item needs out of the registers of its hot loop.
    auto work = [&](const int64_t item) __attribute__((always_inline)) {
    const int64_t quad = item / kWavesPerBlock;
    // 32-bit division when the quads fit (always, below 2^31 work items)
    const int64_t rblk = quad <= INT32_MAX ? (int64_t)((unsigned)quad / (unsigned)a.ngroups) : quad / a.ngroups;
    const int grp = uni((int)(quad - rblk * a.ngroups));
    const int row = uni((int)(rblk * kWavesPerBlock + (item - quad * kWavesPerBlock)));
    if (row >= a.nrows) return;   // ragged last row block
    // segment (catalog) of this row: binary search over the segments' first rows
    int slo = 0, shi = a.nseg - 1;
    while (slo < shi) {
        const int mid = (slo + shi + 1) >> 1;
        if (uni(a.segs[mid].row0) <= row) slo = mid; else shi = mid - 1;
    }
    const GatherSeg g = load_seg(a.segs, uni(slo));
    if (row - g.row0 >= g.nprim) return;   // a row between jobs (see prepare_slice): no primary
    const gptr<double4> gP = as_global(g.P);
    const gptr<int32_t> gcs = as_global(g.cell_start);
    const int ip = uni(g.prim[row - g.row0]);
    const double4 Pi = g.Pq[ip];
    const double xi = uni(Pi.x), yi = uni(Pi.y), zi = uni(Pi.z);
    const int b_lo = grp * NBG;
    const int b_hi = min(b_lo + NBG, a.nbins);
    const double R2in = uni(a.e2[b_lo]), R2out = uni(a.e2[b_hi]);
    // interior squared edges of the group (+inf past the last bin of the group)
    double e2k[NBG];
#pragma unroll
    for (int q = 1; q < NBG; ++q) e2k[q] = uni((b_lo + q < b_hi) ? a.e2[min(b_lo + q, kMaxBins)] : INFINITY);
    // periodic images: shift per axis for image codes 0, 1, 2 (-L, 0, +L)
    const double Lx = g.Lx, Ly = g.Ly, Lz = g.Lz;
    // culling uses slightly enlarged cells and radius; the bin test below is exact
    const double Rin = uni(a.e1[b_lo]), Rout = uni(a.e1[b_hi]);
    const double Rc = Rout + g.cull_pad;

    int head[NBG], tail[NBG];
#pragma unroll
    for (int k = 0; k < NBG; ++k) { head[k] = 0; tail[k] = 0; }
    using A = AccT<T, COMP>;
    A acc[NBG][NLM][2];
#pragma unroll
    for (int k = 0; k < NBG; ++k)
#pragma unroll
        for (int q = 0; q < NLM; ++q) { acc[k][q][0] = (A)0; acc[k][q][1] = (A)0; }

    // row range (unwrapped cell indices)
    // (reciprocal multiplies: the pad of Rc is far above their rounding)
    int ky0 = (int)floor((yi - Rc - g.oy) * g.icsy), ky1 = (int)floor((yi + Rc - g.oy) * g.icsy);
    int kz0 = (int)floor((zi - Rc - g.oz) * g.icsz), kz1 = (int)floor((zi + Rc - g.oz) * g.icsz);
    if (!g.periodic) {
        ky0 = max(ky0, 0); ky1 = min(ky1, g.ncy - 1);
        kz0 = max(kz0, 0); kz1 = min(kz1, g.ncz - 1);
    }
    const int nyr = ky1 - ky0 + 1, nzr = kz1 - kz0 + 1;
    const int nrows = (nyr > 0 && nzr > 0) ? nyr * nzr : 0;
    // Row set-up frame.  Rows only cull candidates (every candidate is binned
    // exactly in FP64 below), so the set-up runs in FP32 with a margin, in cell
    // units, far above the FP32 rounding of coordinates relative to the grid origin
    // (about n * 2^-23 cells for a grid n cells long).
    const RowFrame<float> rf = make_frame<float>(g, xi, yi, zi, Rin, Rout, ky0, kz0, nyr);

    for (int rb = 0; rb < nrows; rb += kRowsPerBatch) {
        // ---- 1. lane-parallel row set-up: lane r counts its row's pieces, which
        //         are written straight to their slots in (lane, piece) order; then
        //         each lane turns its lengths into flat positions and its entries
        //         into deltas (entry minus flat position: a candidate's entry is its
        //         flat position plus its piece's delta; start + length < 2^26 never
        //         carries into the image code)
        const int r = rb + lane;
        RowGeom rg;
        rg.lo[0] = rg.lo[1] = 1;
        rg.hi[0] = rg.hi[1] = 0;
        rg.rowbase = rg.code_yz = 0;
        if (r < nrows) rg = row_geom<float>(rf, g, r);
        // centre pieces first, image pieces after them: a chunk wholly below
        // total_c has no image (one scalar compare instead of a per-lane test)
        int nc, ni;
        row_pieces_split(rg, g, nc, ni);
        int ntot = 0;   // both counts in one scan (at most 64 * kSegPerRow each)
        const int sb = wave_excl_scan(nc | (ni << 16), &ntot);
        const int nseg_c = ntot & 0xffff;
        const int nseg = nseg_c + (ntot >> 16);
        const int sbase_c = sb & 0xffff, sbase_i = nseg_c + (sb >> 16);
        wave_sync();                        // the previous batch's descriptors are consumed
        int nlc, nli;
        emit_pieces_split(rg, g, gcs, sbase_c, sbase_i, seg_dl, seg_flat, nlc, nli);
        int total_c = 0, total_i = 0;
        int fc = wave_excl_scan(nlc, &total_c);
        int fi = wave_excl_scan(nli, &total_i) + total_c;
        const int total = total_c + total_i;
        for (int q = 0; q < nc; ++q) {      // the lane's own slots only
            const int sl = sbase_c + q, ln = seg_flat[sl];
            seg_flat[sl] = fc;
            seg_dl[sl] -= (unsigned)fc;
            fc += ln;
        }
        for (int q = 0; q < ni; ++q) {
            const int sl = sbase_i + q, ln = seg_flat[sl];
            seg_flat[sl] = fi;
            seg_dl[sl] -= (unsigned)fi;
            fi += ln;
        }
        wave_sync();

        // ---- 2./3. candidates, 64 per chunk: lane l of the chunk at flat position p0
        //      takes candidate p0 + l, whose entry (particle index | image code) is
        //      p0 + l plus the delta of the last piece starting at or before it.
        //      One more piece starts at the batch's end and maps the positions past
        //      it onto the grid's NaN sentinels (every bin compare is false), so no
        //      lane needs a select of its own.  Piece descriptors are held 64 at a time in VGPRs
        //      (lane l: piece gbase + l) and read with readlane.
        const unsigned fill_entry = (unsigned)g.nP | ((unsigned)kCenterCode << kCodeShift);
        const unsigned fill_delta = fill_entry - (unsigned)total;
        int gbase = 0;
        unsigned dl_v = 0;
        int fs_v = 0;
        auto reload = [&](int base) {
            gbase = base;
            // the window start as an opaque scalar: the LDS address is formed here,
            // on a reload, and not carried along the walk as a vector induction
            int b = base;
            asm("" : "+s"(b));
            const int sl = b + lane;
            dl_v = sl < nseg ? seg_dl[sl] : (sl == nseg ? fill_delta : 0u);
            fs_v = sl < nseg ? seg_flat[sl] : (sl == nseg ? total : INT_MAX);
        };
        // descriptor of piece t (uniform); piece nseg is the sentinel piece, past
        // it the start is INT_MAX.  The walk only moves forward, so a piece below
        // the window is never asked for.
        auto desc = [&](int t, unsigned& dl, int& fs) {
            if (t >= gbase + kWave) reload(t);
            dl = (unsigned)__builtin_amdgcn_readlane((int)dl_v, t - gbase);
            fs = __builtin_amdgcn_readlane(fs_v, t - gbase);
        };
        reload(0);
        // walk state: piece sg holds the next chunk's first position; (dnext, fnext)
        // describe piece sg + 1
        int sg = 0;
        unsigned dcur = 0u, dnext = 0u;
        int fnext = INT_MAX;
        {
            int f0;
            desc(0, dcur, f0);   // with no pieces: the sentinel piece at 0
            desc(1, dnext, fnext);
        }
        // entries of the chunk at p0 (uniform, increasing from call to call).
        // A chunk past the batch's end stays on the sentinel piece; the prefetch
        // fetches a chunk only when the one before it starts inside the batch,
        // so its lanes stay within 2 * kWave - 1 of the end (kSentinels records).
        auto fetch = [&](int p0) -> unsigned {
            while (fnext <= p0) {
                ++sg;
                dcur = dnext;
                desc(sg + 1, dnext, fnext);
            }
            if (fnext >= p0 + kWave) return (unsigned)lane + ((unsigned)p0 + dcur);
            // pieces starting inside the chunk; the walk ends on the last of them,
            // which holds the next chunk's first position
            const unsigned pl = (unsigned)(p0 + lane);
            unsigned me = pl + dcur;
            do {
                if (lane >= fnext - p0) me = pl + dnext;
                ++sg;
                dcur = dnext;
                desc(sg + 1, dnext, fnext);
            } while (fnext < p0 + kWave);
            return me;
        };
        {
            // one chunk of 64 candidates: exact FP64 bin, ring push, drains
            auto chunk = [&](const unsigned me, const int p0, const double4& q) {
                // x_j - x_i, then the periodic image (+/- L; chunks below the image
                // pieces skip the shift, which would add exactly 0)
                double dx = diff(q.x, xi), dy = diff(q.y, yi), dz = diff(q.z, zi);
                if (p0 + kWave > total_c) {
                    const int code = (int)(me >> kCodeShift);
                    dx = sep(dx, 0.0, (double)((code & 3) - 1) * Lx);
                    dy = sep(dy, 0.0, (double)(((code >> 2) & 3) - 1) * Ly);
                    dz = sep(dz, 0.0, (double)(((code >> 4) & 3) - 1) * Lz);
                }
                const double r2 = dist2(dx, dy, dz);
                bool ok;
                int k = 0;
                int slot;
                if constexpr (NBG == 2) {
                    // three compares give the lane masks: inside the shell, and past
                    // the interior edge (bin 1); each bin's lanes are ranked by one
                    // mbcnt of that bin's mask, offset by the bin's tail
                    const bool c_in = r2 >= R2in, c_out = r2 < R2out, c_k = r2 >= e2k[1];
                    ok = c_in && c_out;
                    const unsigned long long okm =
                        __builtin_amdgcn_ballot_w64(c_in) & __builtin_amdgcn_ballot_w64(c_out);
                    const unsigned long long km = __builtin_amdgcn_ballot_w64(c_k);
                    const unsigned long long m1 = okm & km, m0 = okm & ~km;
                    const unsigned r0 = __builtin_amdgcn_mbcnt_hi((unsigned)(m0 >> 32),
                                                                  __builtin_amdgcn_mbcnt_lo((unsigned)m0, 0u)) +
                                        (unsigned)tail[0];
                    const unsigned r1 = __builtin_amdgcn_mbcnt_hi((unsigned)(m1 >> 32),
                                                                  __builtin_amdgcn_mbcnt_lo((unsigned)m1, 0u)) +
                                        (unsigned)tail[1];
                    // select by the lane mask itself (both ranks are computed anyway; a
                    // conditional would be turned into two divergent branches)
                    const unsigned s0 = r0 & (kCap - 1), s1 = (r1 & (kCap - 1)) | (unsigned)kCap;
                    unsigned sl;
                    asm("v_cndmask_b32_e64 %0, %1, %2, %3" : "=v"(sl) : "v"(s0), "v"(s1), "s"(km));
                    // rejected lanes write their own dump entry: the ring push then
                    // needs no exec-mask branch
                    slot = ok ? (int)sl : NBG * kCap + lane;
                    tail[0] += __popcll(m0);
                    tail[1] += __popcll(m1);
                } else {
                    ok = (r2 >= R2in) && (r2 < R2out);
#pragma unroll
                    for (int q2 = 1; q2 < NBG; ++q2) k += (r2 >= e2k[q2]) ? 1 : 0;
                    // ring slots: one ballot per bit of the bin index; the lanes of
                    // the same bin are those agreeing on every bit
                    constexpr int NBITS = (NBG <= 1) ? 0 : (NBG <= 4) ? 2 : (NBG <= 8) ? 3 : 4;
                    const unsigned long long okm = __builtin_amdgcn_ballot_w64(ok);
                    unsigned long long bm[NBITS > 0 ? NBITS : 1];
                    unsigned long long same = okm;
#pragma unroll
                    for (int bb = 0; bb < NBITS; ++bb) {
                        bm[bb] = __builtin_amdgcn_ballot_w64(ok && ((k >> bb) & 1));
                        same &= ((k >> bb) & 1) ? bm[bb] : ~bm[bb];
                    }
                    const int rank = __builtin_amdgcn_mbcnt_hi((unsigned)(same >> 32),
                                                               __builtin_amdgcn_mbcnt_lo((unsigned)same, 0u));
                    int tk = tail[0];
#pragma unroll
                    for (int q2 = 1; q2 < NBG; ++q2) tk = (k == q2) ? tail[q2] : tk;
#pragma unroll
                    for (int q2 = 0; q2 < NBG; ++q2) {
                        unsigned long long mq = okm;
#pragma unroll
                        for (int bb = 0; bb < NBITS; ++bb) mq &= ((q2 >> bb) & 1) ? bm[bb] : ~bm[bb];
                        tail[q2] += __popcll(mq);
                    }
                    slot = k * kCap + ((tk + rank) & (kCap - 1));
                }
                {
                    E ev;
                    ev.x = (T)dx; ev.y = (T)dy; ev.z = (T)dz; ev.w = (T)q.w;
                    if constexpr (NBG == 2) ring[slot] = ev;
                    else if (ok) ring[slot] = ev;
                }
                [&]<int... K>(std::integer_sequence<int, K...>) {
                    ([&] {
                        if (tail[K] - head[K] >= kWave) {
                            wave_sync();
                            const E e = ring[K * kCap + ((head[K] + lane) & (kCap - 1))];
                            accum_pair<T, L, M0, M1, COMP>(e.x, e.y, e.z, e.w, acc[K]);
                            head[K] += kWave;
                        }
                    }(), ...);
                }(std::make_integer_sequence<int, NBG>{});
            };
            // two chunks per iteration, alternating prefetch registers; the
            // prefetch is unconditional (past the last chunk it loads the sentinel)
            // so that waiting for a chunk's loads never waits for the next's
            unsigned me_a = fetch(0);
            double4 q_a = load_point(gP, (int)(me_a & kStartMask));
            for (int c0 = 0; c0 < total; c0 += 2 * kWave) {
                const unsigned me_b = fetch(c0 + kWave);
                const double4 q_b = load_point(gP, (int)(me_b & kStartMask));
                chunk(me_a, c0, q_a);
                if (c0 + kWave >= total) break;
                me_a = fetch(c0 + 2 * kWave);
                q_a = load_point(gP, (int)(me_a & kStartMask));
                chunk(me_b, c0 + kWave, q_b);
            }
        }
        wave_sync();
    }

    if (a.npairs && lane == 0) {
        unsigned long long tot = 0;
#pragma unroll
        for (int k = 0; k < NBG; ++k) tot += (unsigned long long)tail[k];
        atomicAdd(a.npairs, tot);
    }

    // ---- flush partial rings (missing lanes add zero-weight pairs)
    wave_sync();
    [&]<int... K>(std::integer_sequence<int, K...>) {
        ([&] {
            const int rem = tail[K] - head[K];
            if (rem > 0) {
                E e = ring[K * kCap + ((head[K] + lane) & (kCap - 1))];
                if (lane >= rem) { e.x = (T)1; e.y = (T)0; e.z = (T)0; e.w = (T)0; }
                accum_pair<T, L, M0, M1, COMP>(e.x, e.y, e.z, e.w, acc[K]);
            }
        }(), ...);
    }(std::make_integer_sequence<int, NBG>{});
    wave_sync();

    // ---- 4. reduce the 64 lanes' accumulators and write
    constexpr int NV = NBG * NLM * 2;
    A* accf = &acc[0][0][0];
    const int nvalid = (b_hi - b_lo) * NLM * 2;
    T* out = reinterpret_cast<T*>(a.alm) + ((size_t)row * a.nbins + b_lo) * NLM * 2;
    if (grp == 0 && lane == 0) a.wprim[row] = Pi.w;
    if constexpr (std::is_same_v<T, float> && !COMP) {
        // Reduce-scatter across lanes, two values per step: a 32-lane swap packs
        // values 2p and 2p+1 into one register (lanes 0-31 and 32-63) summed over
        // lanes i, i+32; a 16-row swap packs four values (one per row of 16 lanes)
        // summed over 4 lanes; four rotate-adds inside each row finish the sums.
        // Row r of c[q] then holds value 4q + {0, 2, 1, 3}[r].
        constexpr int NV4 = (NV + 3) / 4 * 4;
        unsigned v[NV4];
#pragma unroll
        for (int q = 0; q < NV4; ++q) v[q] = q < NV ? __float_as_uint(accf[q]) : 0u;
        unsigned b[NV4 / 2];
#pragma unroll
        for (int p2 = 0; p2 < NV4 / 2; ++p2) {
            const auto r = __builtin_amdgcn_permlane32_swap(v[2 * p2], v[2 * p2 + 1], false, false);
            b[p2] = __float_as_uint(__uint_as_float(r[0]) + __uint_as_float(r[1]));
        }
        float c[NV4 / 4];
#pragma unroll
        for (int q = 0; q < NV4 / 4; ++q) {
            const auto r = __builtin_amdgcn_permlane16_swap(b[2 * q], b[2 * q + 1], false, false);
            float x = __uint_as_float(r[0]) + __uint_as_float(r[1]);
            x += __uint_as_float(__builtin_amdgcn_update_dpp(0u, __float_as_uint(x), 0x128, 0xf, 0xf, false));
            x += __uint_as_float(__builtin_amdgcn_update_dpp(0u, __float_as_uint(x), 0x124, 0xf, 0xf, false));
            x += __uint_as_float(__builtin_amdgcn_update_dpp(0u, __float_as_uint(x), 0x122, 0xf, 0xf, false));
            x += __uint_as_float(__builtin_amdgcn_update_dpp(0u, __float_as_uint(x), 0x121, 0xf, 0xf, false));
            c[q] = x;
        }
        const int rrow = lane >> 4;
        const int sub = (rrow == 1) ? 2 : (rrow == 2 ? 1 : rrow);
        if constexpr (M0 == 0 && M1 == L) {
            // Every coefficient is written: stage the sums in LDS (the rings are
            // free after the flush) in value order, then lane l scales values
            // 4l .. 4l+3 (coefficients 2l and 2l+1 mod NLM) and stores them with
            // two 8-byte stores (an item's row is 8 NLM bytes long, so out is
            // 8-byte aligned; nvalid is even).
            static_assert(NV4 / 4 <= kWave && NV4 * 4 <= ring_bytes<T, NBG, COMP>(), "staged values fit");
            float* st = reinterpret_cast<float*>(base);
            if ((lane & 15) == 0) {
#pragma unroll
                for (int q = 0; q < NV4 / 4; ++q) st[4 * q + sub] = c[q];
            }
            wave_sync();
            if (lane < NV4 / 4) {
                const int v0 = 4 * lane;
                const float4 x = *reinterpret_cast<const float4*>(st + v0);
                const double kA = Kappa<L>::t.v[(2 * lane) % NLM], kB = Kappa<L>::t.v[(2 * lane + 1) % NLM];
                if (v0 + 1 < nvalid)
                    *reinterpret_cast<float2*>(out + v0) =
                        make_float2((T)((double)x.x * kA), (T)((double)x.y * kA));
                if (v0 + 3 < nvalid)
                    *reinterpret_cast<float2*>(out + v0 + 2) =
                        make_float2((T)((double)x.z * kB), (T)((double)x.w * kB));
            }
            wave_sync();
        } else if ((lane & 15) == 0) {
            // value 4q + sub is coefficient 2q + (sub >> 1) (mod NLM), part sub & 1;
            // both candidates and their m are compile-time constants
            const bool hi = (sub >> 1) != 0;
#pragma unroll
            for (int q = 0; q < NV4 / 4; ++q) {
                const int vi = 4 * q + sub;
                const int lmA = (2 * q) % NLM, lmB = (2 * q + 1) % NLM;
                const bool inA = m_of_lm(lmA) >= M0 && m_of_lm(lmA) <= M1;
                const bool inB = m_of_lm(lmB) >= M0 && m_of_lm(lmB) <= M1;
                const double ks = hi ? Kappa<L>::t.v[lmB] : Kappa<L>::t.v[lmA];
                if (vi < nvalid && (hi ? inB : inA)) out[vi] = (T)((double)c[q] * ks);
            }
        }
        wave_sync();
    } else {
        // FP64 accumulators (the FP64 path, and the FP32 path's FP64 sums): through
        // LDS, 8 interleaved FP64 partial sums per value
#pragma unroll
        for (int v0 = 0; v0 < NV; v0 += CH) {
#pragma unroll
            for (int c = 0; c < CH; ++c)
                if (v0 + c < NV) {
                    scratch[c * 65 + lane] = accf[v0 + c];
                }
            wave_sync();
            const int v = v0 + lane;
            if (lane < CH && v < nvalid) {
                const int lm = (v >> 1) % NLM;
                int l = 0;   // degree of coefficient lm: the count of t <= L with t(t+1)/2 <= lm
#pragma unroll
                for (int t = 1; t <= L; ++t) l += (lm >= t * (t + 1) / 2) ? 1 : 0;
                const int m = lm - l * (l + 1) / 2;
                if (m >= M0 && m <= M1) {
                    double s8[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) s8[u] = 0.0;
#pragma unroll
                    for (int l2 = 0; l2 < kWave; ++l2) s8[l2 & 7] += (double)scratch[lane * 65 + l2];
                    const double s = ((s8[0] + s8[1]) + (s8[2] + s8[3])) + ((s8[4] + s8[5]) + (s8[6] + s8[7]));
                    out[v] = (T)(s * Kappa<L>::t.v[lm]);
                }
            }
            wave_sync();
        }
    }
    wave_sync();
    };
    if constexpr (PERS) {
        for (int64_t item = pop(); item >= 0 && item < nitems; item = pop()) work(item);
    } else {
        const int nblk = gridDim.x;
        const int bid = (blockIdx.x % 8) * (nblk / 8) + blockIdx.x / 8;
        const int64_t item = (int64_t)bid * kWavesPerBlock + wib;
        if (item < nitems) work(item);
    }
}


// --------------------------------------------------------------- configurations
struct KernelCfg {
    int nbg;
    int nm;                 // number of m groups
    int m0[2], m1[2];
    const void* fn[2];      // static grid
    const void* fnp[2];     // persistent grid
    int lds;                // bytes per block
};

template <typename T, int L, int NBG, int M0, int M1, bool PERS, bool COMP>
const void* kfn() { return reinterpret_cast<const void*>(&k_gather<T, L, NBG, M0, M1, PERS, COMP>); }

template <typename T, int L, int NBG, bool COMP = false>
KernelCfg cfg1()
{
    KernelCfg c{};
    c.nbg = NBG; c.nm = 1; c.m0[0] = 0; c.m1[0] = L;
    c.fn[0] = kfn<T, L, NBG, 0, L, false, COMP>(); c.fnp[0] = kfn<T, L, NBG, 0, L, true, COMP>();
    c.lds = kWavesPerBlock * wave_lds_bytes<T, NBG, COMP>();
    return c;
}
template <typename T, int L, int NBG, int MS, bool COMP = false>
KernelCfg cfg2()
{
    KernelCfg c{};
    c.nbg = NBG; c.nm = 2;
    c.m0[0] = 0; c.m1[0] = MS - 1;
    c.fn[0] = kfn<T, L, NBG, 0, MS - 1, false, COMP>(); c.fnp[0] = kfn<T, L, NBG, 0, MS - 1, true, COMP>();
    c.m0[1] = MS; c.m1[1] = L;
    c.fn[1] = kfn<T, L, NBG, MS, L, false, COMP>(); c.fnp[1] = kfn<T, L, NBG, MS, L, true, COMP>();
    c.lds = kWavesPerBlock * wave_lds_bytes<T, NBG, COMP>();
    return c;
}

// Bins per work item: fewer bins per item means more passes over the candidates
// but fewer accumulator registers, hence more resident waves to hide the LDS and
// L2 latency of the candidate stream.  Several values are compiled for the common
// cases; encore_autotune picks one per job shape (ENCORE_GATHER_NBG overrides).
int nbg_env()
{
    static int v = [] {
        const char* s = getenv("ENCORE_GATHER_NBG");
        return s ? atoi(s) : 0;
    }();
    return v;
}

// The compiled variant with `nbg` bins per item, or the default (first) one.
// precision: 0 FP64, 1 FP32, 2 FP32 terms with FP64 accumulators (as many registers
// per value as FP64, so the same bins per item and m split).
KernelCfg config(int lmax, int precision, int nbg)
{
    if (nbg_env() > 0) nbg = nbg_env();
    if (precision == 2) {
        switch (lmax) {
        case 0: return cfg1<float, 0, 8, true>();
        case 1: return cfg1<float, 1, 8, true>();
        case 2: return cfg1<float, 2, 8, true>();
        case 3: return nbg == 2 ? cfg1<float, 3, 2, true>() : cfg1<float, 3, 5, true>();
        case 4: return nbg == 2 ? cfg1<float, 4, 2, true>() : cfg1<float, 4, 3, true>();
        case 5: return nbg == 1 ? cfg1<float, 5, 1, true>() : cfg1<float, 5, 2, true>();
        case 6: return cfg1<float, 6, 1, true>();
        case 7: return cfg1<float, 7, 1, true>();
        case 8: return cfg1<float, 8, 1, true>();
        case 9: return cfg2<float, 9, 1, 5, true>();
        case 10: return cfg2<float, 10, 1, 4, true>();
        }
    } else if (precision == 1) {
        switch (lmax) {
        case 0: return cfg1<float, 0, 16>();
        case 1: return cfg1<float, 1, 16>();
        case 2: return nbg == 10 ? cfg1<float, 2, 10>() : cfg1<float, 2, 6>();
        case 3: return nbg == 5 ? cfg1<float, 3, 5>() : (nbg == 2 ? cfg1<float, 3, 2>() : cfg1<float, 3, 4>());
        case 4: return nbg == 5 ? cfg1<float, 4, 5>() : (nbg == 2 ? cfg1<float, 4, 2>() : cfg1<float, 4, 3>());
        case 5: return nbg == 3 ? cfg1<float, 5, 3>() : cfg1<float, 5, 2>();
        case 6: return nbg == 1 ? cfg1<float, 6, 1>() : cfg1<float, 6, 2>();
        case 7: return cfg1<float, 7, 1>();
        case 8: return cfg1<float, 8, 1>();
        case 9: return cfg1<float, 9, 1>();
        case 10: return cfg1<float, 10, 1>();
        }
    } else {
        switch (lmax) {
        case 0: return cfg1<double, 0, 8>();
        case 1: return cfg1<double, 1, 8>();
        case 2: return cfg1<double, 2, 8>();
        case 3: return nbg == 2 ? cfg1<double, 3, 2>() : cfg1<double, 3, 5>();
        case 4: return nbg == 2 ? cfg1<double, 4, 2>() : cfg1<double, 4, 3>();
        case 5: return cfg1<double, 5, 2>();
        case 6: return cfg1<double, 6, 1>();
        case 7: return cfg1<double, 7, 1>();
        case 8: return cfg1<double, 8, 1>();
        case 9: return cfg2<double, 9, 1, 5>();
        case 10: return cfg2<double, 10, 1, 4>();
        }
    }
    return KernelCfg{};
}

}  // namespace

int gather_group_bins(int lmax, int precision, int nbg) { return config(lmax, precision, nbg).nbg; }

std::vector<int> gather_nbg_options(int lmax, int precision)
{
    static const std::vector<int> f32[11] = {{16}, {16}, {6, 10}, {4, 2, 5}, {3, 2, 5}, {2, 3},
                                             {2, 1}, {1}, {1}, {1}, {1}};
    static const std::vector<int> f64[11] = {{8}, {8}, {8}, {5, 2}, {3, 2}, {2}, {1}, {1}, {1}, {1}, {1}};
    static const std::vector<int> f32c[11] = {{8}, {8}, {8}, {5, 2}, {3, 2}, {2, 1}, {1}, {1}, {1}, {1}, {1}};
    if (lmax < 0 || lmax > 10) return {};
    return precision == 1 ? f32[lmax] : (precision == 2 ? f32c[lmax] : f64[lmax]);
}

void gather_tables(int lmax, double* kappa)
{
    // kappa_mm = (-1)^m c_m, c_0 = 1/sqrt(4 pi), c_m = c_{m-1} sqrt((2m+1)/(2m));
    // kappa_{m+1,m} = sqrt(2m+3) kappa_mm; kappa_lm = a_lm kappa_{l-1,m} (l >= m+2),
    // a_lm = sqrt((4l^2-1)/(l^2-m^2)); the recurrence coefficients gamma_lm use
    // b_lm = sqrt(((l-1)^2-m^2)/(4(l-1)^2-1)) (GammaTable).
    double c = 1.0 / std::sqrt(4.0 * M_PI);
    for (int m = 0; m <= lmax; ++m) {
        if (m > 0) c *= std::sqrt((2.0 * m + 1.0) / (2.0 * m));
        const double kmm = (m % 2) ? -c : c;
        kappa[lm_index(m, m)] = kmm;
        if (m + 1 <= lmax) kappa[lm_index(m + 1, m)] = std::sqrt(2.0 * m + 3.0) * kmm;
        for (int l = m + 2; l <= lmax; ++l) {
            const double al = std::sqrt((4.0 * l * l - 1.0) / ((double)l * l - (double)m * m));
            kappa[lm_index(l, m)] = al * kappa[lm_index(l - 1, m)];
        }
    }
}

int launch_gather(const GatherArgs& a0, int lmax, int precision, int nbg, bool persistent, hipStream_t stream)
{
    const KernelCfg c = config(lmax, precision, nbg);
    if (!c.fn[0]) return (int)hipErrorInvalidValue;
    GatherArgs a = a0;
    a.group_bins = c.nbg;
    a.ngroups = (a.nbins + c.nbg - 1) / c.nbg;
    if (!persistent) a.queues = nullptr;
    if (persistent && !a.queues) return (int)hipErrorInvalidValue;
    const int64_t quads = ((int64_t)a.nrows + kWavesPerBlock - 1) / kWavesPerBlock * a.ngroups;
    if (quads == 0) return (int)hipSuccess;
    for (int g = 0; g < c.nm; ++g) {
        const void* fn = persistent ? c.fnp[g] : c.fn[g];
        int64_t blocks;
        if (persistent) {
            // one block per resident block slot
            int dev = 0, per_cu = 0;
            hipDeviceProp_t prop;
            hipError_t e = hipGetDevice(&dev);
            if (e == hipSuccess) e = hipGetDeviceProperties(&prop, dev);
            if (e == hipSuccess)
                e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kWave * kWavesPerBlock,
                                                                 (size_t)c.lds);
            if (e != hipSuccess) return (int)e;
            blocks = std::max(1, per_cu) * (int64_t)prop.multiProcessorCount;
            blocks = std::min<int64_t>(blocks, quads);
            const int rc = launch_fill_u32(a.queues, 8, 0u, stream);
            if (rc != 0) return rc;
        } else {
            blocks = quads;
        }
        blocks = (blocks + 7) / 8 * 8;
        if (blocks > INT32_MAX) return (int)hipErrorInvalidValue;
        if (c.lds > 65536) {   // blocks above 64 KiB of LDS need the limit raised once
            static thread_local std::vector<const void*> raised;
            if (std::find(raised.begin(), raised.end(), fn) == raised.end()) {
                const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, c.lds);
                if (e != hipSuccess) return (int)e;
                raised.push_back(fn);
            }
        }
        void* args[] = {&a};
        hipError_t e = hipLaunchKernel(fn, dim3((unsigned)blocks), dim3(kWave * kWavesPerBlock),
                                       args, (size_t)c.lds, stream);
        if (e != hipSuccess) return (int)e;
    }
    return (int)hipSuccess;
}

namespace {
// One block per row: the row of primary prim[r] gets cache row prim[r] (its
// cached data part; complex entries, 2 * T each) added.
template <typename T>
__global__ void __launch_bounds__(256) k_add_cached(T* __restrict__ alm, int row0, const int32_t* __restrict__ prim,
                                                   const T* __restrict__ cache, int row_cplx)
{
    const int r = blockIdx.x;
    const int src = prim[r];
    using V = typename std::conditional<sizeof(T) == 8, double2, float2>::type;
    V* dst = reinterpret_cast<V*>(alm) + (int64_t)(row0 + r) * row_cplx;
    const V* cs = reinterpret_cast<const V*>(cache) + (int64_t)src * row_cplx;
    for (int c = threadIdx.x; c < row_cplx; c += 256) {
        V v = dst[c];
        const V u = cs[c];
        v.x += u.x;
        v.y += u.y;
        dst[c] = v;
    }
}
}  // namespace

int launch_add_cached(void* alm, int precision, int row0, int nrows, const int32_t* prim, const void* cache,
                      int row_cplx, hipStream_t stream)
{
    if (nrows <= 0) return (int)hipSuccess;
    if (precision == 0)
        k_add_cached<double><<<dim3((unsigned)nrows), dim3(256), 0, stream>>>(
            static_cast<double*>(alm), row0, prim, static_cast<const double*>(cache), row_cplx);
    else
        k_add_cached<float><<<dim3((unsigned)nrows), dim3(256), 0, stream>>>(
            static_cast<float*>(alm), row0, prim, static_cast<const float*>(cache), row_cplx);
    return (int)hipGetLastError();
}

}  // namespace encore
