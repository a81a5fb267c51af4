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
//     cell with x fastest, each clipped piece is one contiguous particle range.
//  2. Candidate test, 64 candidates per step: separation in FP64 exactly as the
//     definition orders it (x_j - x_i, then the periodic image), r^2 =
//     (dx*dx + dy*dy) + dz*dz without contraction, bin by comparing r^2 with the
//     squared edges.  Accepted pairs are pushed into one LDS ring per bin
//     (slot from an LDS atomic).
//  3. Drain: whenever a ring holds 64 pairs, all 64 lanes pop one pair each, form
//     Y_lm by the monic Legendre recurrence in z times (x + i y)^m and add w Y into
//     per-lane register accumulators of that bin (the bin is wave-uniform, so the
//     register index is static).
//  4. Reduce the 64 lanes' accumulators through LDS (FP64 sums), scale by the
//     recurrence normalisation kappa_lm and write the complex coefficients.
//
// Y_lm = N_lm(z) (x + i y)^m for a unit vector (Condon-Shortley phase inside N_lm);
// N_lm = kappa_lm R_lm with R_mm = 1, R_{m+1,m} = z, R_lm = z R_{l-1,m} - gamma_lm R_{l-2,m}.
#include <hip/hip_runtime.h>
#include <cmath>
#include <utility>

#include "device.h"

namespace encore {

namespace {

constexpr int kCap = 128;          // ring capacity per bin (pairs)
constexpr int kRowsPerBatch = 64;  // rows set up per lane-parallel pass
constexpr int kSegPerRow = 6;      // <= 2 x-ranges x 3 periodic images
constexpr int kSegCap = kRowsPerBatch * kSegPerRow;
constexpr int kWavesPerBlock = 1;  // waves are independent; no block barriers

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
template <> __device__ __forceinline__ float rsqrt_t<float>(float v) { return rsqrtf(v); }
template <> __device__ __forceinline__ double rsqrt_t<double>(double v) { return 1.0 / sqrt(v); }

template <typename T, int NBG>
__host__ __device__ constexpr int wave_lds_bytes()
{
    // ring storage (reused as the reduction scratch) + tails + segment lists
    return ((NBG * kCap * (int)sizeof(typename Entry<T>::type) > 32 * 65 * (int)sizeof(T))
                ? NBG * kCap * (int)sizeof(typename Entry<T>::type)
                : 32 * 65 * (int)sizeof(T)) +
           16 * 4 + 3 * kSegCap * 4 + kWave * 4;
}

// Add w*Y_lm for m in [M0, M1] of one pair into acc (layout [lm][re, im]).
template <typename T, int L, int M0, int M1>
__device__ __forceinline__ void accum_pair(T dx, T dy, T dz, T w, T (&acc)[nlm_of(L)][2],
                                           const T (&gam)[nlm_of(L)])
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
            const T nr = ur * x - ui * y;
            const T ni = ur * y + ui * x;
            ur = nr; ui = ni;
        }
        T r0 = w, r1 = zw;
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
            const T rn = z * r1 - gam[lm_index(l, m)] * r0;
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

__device__ __forceinline__ double dmul(double a, double b) { return __dmul_rn(a, b); }
__device__ __forceinline__ double dadd(double a, double b) { return __dadd_rn(a, b); }

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

template <typename T, int L, int NBG, int M0, int M1>
__global__ void __launch_bounds__(kWave * kWavesPerBlock, 2) k_gather(GatherArgs a)
{
    using E = typename Entry<T>::type;
    constexpr int NLM = nlm_of(L);
    constexpr int CH = 32;
    extern __shared__ __align__(16) unsigned char smem[];

    const int lane = threadIdx.x & (kWave - 1);
    const int wib = threadIdx.x / kWave;
    // XCD-aware block order: the grid is a multiple of 8 blocks and block b runs on
    // XCD b % 8; give each XCD a contiguous run of work items so that neighbouring
    // primaries (same cells) share that XCD's L2.
    const int nblk = gridDim.x;
    const int bid = (blockIdx.x % 8) * (nblk / 8) + blockIdx.x / 8;
    const int item = bid * kWavesPerBlock + wib;
    const int p = item / a.ngroups;
    const int grp = item - p * a.ngroups;
    if (p >= a.nprim) return;

    unsigned char* base = smem + wib * wave_lds_bytes<T, NBG>();
    constexpr int ring_bytes = (NBG * kCap * (int)sizeof(E) > CH * 65 * (int)sizeof(T))
                                   ? NBG * kCap * (int)sizeof(E) : CH * 65 * (int)sizeof(T);
    E* ring = reinterpret_cast<E*>(base);
    T* scratch = reinterpret_cast<T*>(base);
    int* tails = reinterpret_cast<int*>(base + ring_bytes);
    int* seg_start = tails + 16;
    int* seg_end = seg_start + kSegCap;
    int* seg_code = seg_end + kSegCap;
    int* seg_count = seg_code + kSegCap;

    // recurrence coefficients -> registers (uniform)
    T gam[NLM];
#pragma unroll
    for (int q = 0; q < NLM; ++q) gam[q] = (T)a.gamma[q];

    const int ip = a.prim[p];
    const double4 Pi = a.P[ip];
    const double xi = Pi.x, yi = Pi.y, zi = Pi.z;
    const int b_lo = grp * NBG;
    const int b_hi = min(b_lo + NBG, a.nbins);
    const double R2in = a.e2[b_lo], R2out = a.e2[b_hi];
    // culling uses slightly enlarged cells and radius; the bin test below is exact
    const double eps = 1e-7 * fmin(a.csx, fmin(a.csy, a.csz));
    const double Rc = sqrt(R2out) + eps;
    const double Rc2 = Rc * Rc;
    const double Rin = sqrt(R2in);

    if (lane < 16) tails[lane] = 0;
    int head[NBG];
#pragma unroll
    for (int k = 0; k < NBG; ++k) head[k] = 0;
    T acc[NBG][NLM][2];
#pragma unroll
    for (int k = 0; k < NBG; ++k)
#pragma unroll
        for (int q = 0; q < NLM; ++q) { acc[k][q][0] = (T)0; acc[k][q][1] = (T)0; }
    wave_sync();

    auto drain = [&](auto kc, int hd) {
        constexpr int k = decltype(kc)::value;
        const E e = ring[k * kCap + ((hd + lane) & (kCap - 1))];
        accum_pair<T, L, M0, M1>(e.x, e.y, e.z, e.w, acc[k], gam);
    };

    // row range (unwrapped cell indices)
    int ky0 = (int)floor((yi - Rc - a.oy) / a.csy), ky1 = (int)floor((yi + Rc - a.oy) / a.csy);
    int kz0 = (int)floor((zi - Rc - a.oz) / a.csz), kz1 = (int)floor((zi + Rc - a.oz) / a.csz);
    if (!a.periodic) {
        ky0 = max(ky0, 0); ky1 = min(ky1, a.ncy - 1);
        kz0 = max(kz0, 0); kz1 = min(kz1, a.ncz - 1);
    }
    const int nyr = ky1 - ky0 + 1, nzr = kz1 - kz0 + 1;
    const int nrows = (nyr > 0 && nzr > 0) ? nyr * nzr : 0;

    for (int rb = 0; rb < nrows; rb += kRowsPerBatch) {
        // ---- 1. lane-parallel row set-up: lane r writes its <= kSegPerRow pieces to
        //         slots [lane * kSegPerRow, ...) and its count to seg_count[lane]
        {
            int ns = 0;
            const int r = rb + lane;
            if (r < nrows) {
                const int ky = ky0 + r % nyr, kz = kz0 + r / nyr;
                int wy = ky, wz = kz, sy = 0, sz = 0;
                if (a.periodic) {
                    wy = ((ky % a.ncy) + a.ncy) % a.ncy; sy = (ky - wy) / a.ncy;
                    wz = ((kz % a.ncz) + a.ncz) % a.ncz; sz = (kz - wz) / a.ncz;
                }
                const double ylo = a.oy + ky * a.csy - eps, yhi = a.oy + (ky + 1) * a.csy + eps;
                const double zlo = a.oz + kz * a.csz - eps, zhi = a.oz + (kz + 1) * a.csz + eps;
                const double dymin = fmax(0.0, fmax(ylo - yi, yi - yhi));
                const double dzmin = fmax(0.0, fmax(zlo - zi, zi - zhi));
                const double rho2 = dymin * dymin + dzmin * dzmin;
                if (rho2 < Rc2) {
                    const double h = sqrt(Rc2 - rho2) + eps;
                    int kx0 = (int)floor((xi - h - a.ox) / a.csx), kx1 = (int)floor((xi + h - a.ox) / a.csx);
                    if (!a.periodic) { kx0 = max(kx0, 0); kx1 = min(kx1, a.ncx - 1); }
                    const double dymax = fmax(fabs(ylo - yi), fabs(yhi - yi));
                    const double dzmax = fmax(fabs(zlo - zi), fabs(zhi - zi));
                    const double rhomax2 = dymax * dymax + dzmax * dzmax;
                    int kin0 = 1, kin1 = 0;
                    if (Rin > 0.0 && rhomax2 < R2in) {
                        const double hin = sqrt(R2in - rhomax2) - eps;
                        if (hin > 0.0) {
                            kin0 = (int)ceil((xi - hin - a.ox) / a.csx);
                            kin1 = (int)floor((xi + hin - a.ox) / a.csx) - 1;
                        }
                    }
                    const int rowbase = (wz * a.ncy + wy) * a.ncx;
                    const int code_yz = ((sy + 1) << 2) | ((sz + 1) << 4);
                    // at most two x ranges: left of and right of the inner hole
                    for (int q = 0; q < 2; ++q) {
                        int lo, hi;
                        if (kin0 <= kin1) {
                            lo = (q == 0) ? kx0 : max(kx0, kin1 + 1);
                            hi = (q == 0) ? min(kx1, kin0 - 1) : kx1;
                        } else {
                            if (q == 1) break;
                            lo = kx0; hi = kx1;
                        }
                        if (lo > hi) continue;
                        int sxa = 0, sxb = 0;
                        if (a.periodic) {
                            sxa = (lo >= 0) ? lo / a.ncx : -((-lo + a.ncx - 1) / a.ncx);
                            sxb = (hi >= 0) ? hi / a.ncx : -((-hi + a.ncx - 1) / a.ncx);
                        }
                        for (int sx = sxa; sx <= sxb && ns < kSegPerRow; ++sx) {
                            const int plo = max(lo, sx * a.ncx) - sx * a.ncx;
                            const int phi = min(hi, sx * a.ncx + a.ncx - 1) - sx * a.ncx;
                            const int st = a.cell_start[rowbase + plo];
                            const int en = a.cell_start[rowbase + phi + 1];
                            if (en > st) {
                                const int slot = lane * kSegPerRow + ns;
                                seg_start[slot] = st;
                                seg_end[slot] = en;
                                seg_code[slot] = (sx + 1) | code_yz;
                                ++ns;
                            }
                        }
                    }
                }
            }
            seg_count[lane] = ns;
        }
        wave_sync();

        // ---- 2./3. candidates and drains
        const int nlanes = min(kWave, nrows - rb);
        for (int sl = 0; sl < nlanes * kSegPerRow; ++sl) {
            const int owner = sl / kSegPerRow;
            if (sl - owner * kSegPerRow >= __builtin_amdgcn_readfirstlane(seg_count[owner])) continue;
            const int st = __builtin_amdgcn_readfirstlane(seg_start[sl]);
            const int en = __builtin_amdgcn_readfirstlane(seg_end[sl]);
            const int code = __builtin_amdgcn_readfirstlane(seg_code[sl]);
            const double shx = (double)((code & 3) - 1) * a.Lx;
            const double shy = (double)(((code >> 2) & 3) - 1) * a.Ly;
            const double shz = (double)(((code >> 4) & 3) - 1) * a.Lz;
            const bool shifted = (code != 0x15);
            for (int c = st; c < en; c += kWave) {
                const int j = c + lane;
                bool ok = false;
                double dx = 0.0, dy = 0.0, dz = 0.0, wj = 0.0;
                if (j < en) {
                    const double4 q = a.P[j];
                    dx = q.x - xi; dy = q.y - yi; dz = q.z - zi; wj = q.w;
                    if (shifted) { dx = dadd(dx, shx); dy = dadd(dy, shy); dz = dadd(dz, shz); }
                    const double r2 = dadd(dadd(dmul(dx, dx), dmul(dy, dy)), dmul(dz, dz));
                    ok = (r2 >= R2in) && (r2 < R2out);
                    if (ok) {
                        int k = 0;
#pragma unroll
                        for (int q2 = 1; q2 < NBG; ++q2)
                            if (b_lo + q2 < b_hi && r2 >= a.e2[b_lo + q2]) k = q2;
                        const int slot = atomicAdd(&tails[k], 1);
                        E ev;
                        ev.x = (T)dx; ev.y = (T)dy; ev.z = (T)dz; ev.w = (T)wj;
                        ring[k * kCap + (slot & (kCap - 1))] = ev;
                    }
                }
                wave_sync();
                [&]<int... K>(std::integer_sequence<int, K...>) {
                    ([&] {
                        const int t = __builtin_amdgcn_readfirstlane(tails[K]);
                        if (t - head[K] >= kWave) {
                            drain(std::integral_constant<int, K>{}, head[K]);
                            head[K] += kWave;
                        }
                    }(), ...);
                }(std::make_integer_sequence<int, NBG>{});
                wave_sync();
            }
        }
    }

    if (a.npairs && lane == 0) {
        unsigned long long tot = 0;
#pragma unroll
        for (int k = 0; k < NBG; ++k) tot += (unsigned long long)tails[k];
        atomicAdd(a.npairs, tot);
    }

    // ---- flush partial rings (missing lanes add zero-weight pairs)
    [&]<int... K>(std::integer_sequence<int, K...>) {
        ([&] {
            const int t = __builtin_amdgcn_readfirstlane(tails[K]);
            const int rem = t - head[K];
            if (rem > 0) {
                E e = ring[K * kCap + ((head[K] + lane) & (kCap - 1))];
                if (lane >= rem) { e.x = (T)1; e.y = (T)0; e.z = (T)0; e.w = (T)0; }
                accum_pair<T, L, M0, M1>(e.x, e.y, e.z, e.w, acc[K], gam);
            }
        }(), ...);
    }(std::make_integer_sequence<int, NBG>{});
    wave_sync();

    // ---- 4. reduce over lanes through LDS and write
    constexpr int NV = NBG * NLM * 2;
    T* accf = &acc[0][0][0];
    const int nvalid = (b_hi - b_lo) * NLM * 2;
    T* out = reinterpret_cast<T*>(a.alm) + ((size_t)p * a.nbins + b_lo) * NLM * 2;
#pragma unroll
    for (int v0 = 0; v0 < NV; v0 += CH) {
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            if (v0 + c < NV) scratch[c * 65 + lane] = accf[v0 + c];
        }
        wave_sync();
        const int v = v0 + lane;
        if (lane < CH && v < nvalid) {
            const int lm = (v >> 1) % NLM;
            const int m = m_of_lm(lm);
            if (m >= M0 && m <= M1) {
                double s = 0.0;
                for (int l2 = 0; l2 < kWave; ++l2) s += (double)scratch[lane * 65 + l2];
                out[v] = (T)(s * a.kappa[lm]);
            }
        }
        wave_sync();
    }
}

// --------------------------------------------------------------- configurations
struct KernelCfg {
    int nbg;
    int nm;                 // number of m groups
    int m0[2], m1[2];
    const void* fn[2];
    int lds;                // bytes per block
};

template <typename T, int L, int NBG, int M0, int M1>
const void* kfn() { return reinterpret_cast<const void*>(&k_gather<T, L, NBG, M0, M1>); }

template <typename T, int L, int NBG>
KernelCfg cfg1()
{
    KernelCfg c{};
    c.nbg = NBG; c.nm = 1; c.m0[0] = 0; c.m1[0] = L; c.fn[0] = kfn<T, L, NBG, 0, L>();
    c.lds = kWavesPerBlock * wave_lds_bytes<T, NBG>();
    return c;
}
template <typename T, int L, int NBG, int MS>
KernelCfg cfg2()
{
    KernelCfg c{};
    c.nbg = NBG; c.nm = 2;
    c.m0[0] = 0; c.m1[0] = MS - 1; c.fn[0] = kfn<T, L, NBG, 0, MS - 1>();
    c.m0[1] = MS; c.m1[1] = L; c.fn[1] = kfn<T, L, NBG, MS, L>();
    c.lds = kWavesPerBlock * wave_lds_bytes<T, NBG>();
    return c;
}

KernelCfg config(int lmax, int precision)
{
    if (precision == 1) {
        switch (lmax) {
        case 0: return cfg1<float, 0, 16>();
        case 1: return cfg1<float, 1, 16>();
        case 2: return cfg1<float, 2, 16>();
        case 3: return cfg1<float, 3, 10>();
        case 4: return cfg1<float, 4, 5>();
        case 5: return cfg1<float, 5, 5>();
        case 6: return cfg1<float, 6, 3>();
        case 7: return cfg1<float, 7, 2>();
        case 8: return cfg1<float, 8, 2>();
        case 9: return cfg1<float, 9, 1>();
        case 10: return cfg1<float, 10, 1>();
        }
    } else {
        switch (lmax) {
        case 0: return cfg1<double, 0, 8>();
        case 1: return cfg1<double, 1, 8>();
        case 2: return cfg1<double, 2, 8>();
        case 3: return cfg1<double, 3, 5>();
        case 4: return cfg1<double, 4, 3>();
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

int gather_group_bins(int lmax, int precision) { return config(lmax, precision).nbg; }

void gather_tables(int lmax, double* kappa, double* gamma)
{
    // kappa_mm = (-1)^m c_m, c_0 = 1/sqrt(4 pi), c_m = c_{m-1} sqrt((2m+1)/(2m));
    // kappa_{m+1,m} = sqrt(2m+3) kappa_mm; kappa_lm = a_lm kappa_{l-1,m} (l >= m+2),
    // a_lm = sqrt((4l^2-1)/(l^2-m^2)), b_lm = sqrt(((l-1)^2-m^2)/(4(l-1)^2-1)),
    // gamma_lm = b_lm kappa_{l-2,m} / kappa_{l-1,m}.
    double c = 1.0 / std::sqrt(4.0 * M_PI);
    for (int m = 0; m <= lmax; ++m) {
        if (m > 0) c *= std::sqrt((2.0 * m + 1.0) / (2.0 * m));
        const double kmm = (m % 2) ? -c : c;
        kappa[lm_index(m, m)] = kmm;
        gamma[lm_index(m, m)] = 0.0;
        if (m + 1 <= lmax) {
            kappa[lm_index(m + 1, m)] = std::sqrt(2.0 * m + 3.0) * kmm;
            gamma[lm_index(m + 1, m)] = 0.0;
        }
        for (int l = m + 2; l <= lmax; ++l) {
            const double al = std::sqrt((4.0 * l * l - 1.0) / ((double)l * l - (double)m * m));
            const double bl = std::sqrt(((double)(l - 1) * (l - 1) - (double)m * m) /
                                        (4.0 * (l - 1) * (l - 1) - 1.0));
            kappa[lm_index(l, m)] = al * kappa[lm_index(l - 1, m)];
            gamma[lm_index(l, m)] = bl * kappa[lm_index(l - 2, m)] / kappa[lm_index(l - 1, m)];
        }
    }
}

int launch_gather(const GatherArgs& a0, int lmax, int precision, hipStream_t stream)
{
    const KernelCfg c = config(lmax, precision);
    if (!c.fn[0]) return (int)hipErrorInvalidValue;
    GatherArgs a = a0;
    a.group_bins = c.nbg;
    a.ngroups = (a.nbins + c.nbg - 1) / c.nbg;
    const int64_t items = (int64_t)a.nprim * a.ngroups;
    int64_t blocks = (items + kWavesPerBlock - 1) / kWavesPerBlock;
    blocks = (blocks + 7) / 8 * 8;
    if (blocks > INT32_MAX) return (int)hipErrorInvalidValue;
    for (int g = 0; g < c.nm; ++g) {
        void* args[] = {&a};
        hipError_t e = hipLaunchKernel(c.fn[g], dim3((unsigned)blocks), dim3(kWave * kWavesPerBlock),
                                       args, (size_t)c.lds, stream);
        if (e != hipSuccess) return (int)e;
    }
    return (int)hipSuccess;
}

}  // namespace encore
