// Device-resident cell grid (the Cartesian grid of the paper's neighbour search,
// Section 4.1) and the data-minus-randoms weighting (Section 4.2).
//
// Build steps, all on the device:
//   1. validate (finite positions and weights, inside a periodic box)
//   2. FP64 sums of data and random weights; randoms get -w_R sum(w_D)/sum(w_R)
//   3. bounding box (non-periodic) -> grid geometry on the host
//   4. cell index per point, counts (int atomics)
//   5. exclusive scan of the counts -> cell_start
//   6. scatter into cells, then sort each cell by input index (deterministic order)
//   7. gather (x, y, z, w) into the sorted FP64 array, inverse permutation
#include <hip/hip_runtime.h>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "device.h"

namespace encore {

namespace {

constexpr int kBlock = 256;

__global__ void k_validate(const double* __restrict__ pos, const double* __restrict__ w, int64_t n,
                           int periodic, double Lx, double Ly, double Lz, int* __restrict__ flags)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double x = pos[3 * i], y = pos[3 * i + 1], z = pos[3 * i + 2], wi = w[i];
    int f = 0;
    if (!isfinite(x) || !isfinite(y) || !isfinite(z)) f |= 1;
    if (!isfinite(wi)) f |= 2;
    if (periodic && (x < 0.0 || x >= Lx || y < 0.0 || y >= Ly || z < 0.0 || z >= Lz)) f |= 4;
    if (f) atomicOr(flags, f);
}

// Per-block FP64 partial sums of w over [lo, hi) (fixed tree order).
__global__ void k_wsum_partial(const double* __restrict__ w, int64_t lo, int64_t hi,
                               double* __restrict__ partial)
{
    __shared__ double s[kBlock];
    double acc = 0.0;
    for (int64_t i = lo + blockIdx.x * (int64_t)kBlock + threadIdx.x; i < hi;
         i += (int64_t)gridDim.x * kBlock)
        acc += w[i];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int off = kBlock / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = s[0];
}

__global__ void k_sum_final(const double* __restrict__ partial, int np, double* __restrict__ out)
{
    __shared__ double s[kBlock];
    double acc = 0.0;
    for (int i = threadIdx.x; i < np; i += kBlock) acc += partial[i];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int off = kBlock / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = s[0];
}

// w_out = w for data, -w * (sd / sr) for randoms (FP64)
__global__ void k_dmr_weights(const double* __restrict__ w, int64_t n, int64_t n_data,
                              const double* __restrict__ sums, double* __restrict__ w_out)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double wi = w[i];
    w_out[i] = (i < n_data) ? wi : -wi * (sums[0] / sums[1]);
}

__global__ void k_minmax_partial(const double* __restrict__ pos, int64_t n, double* __restrict__ partial)
{
    __shared__ double smin[3][kBlock], smax[3][kBlock];
    double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        for (int a = 0; a < 3; ++a) {
            const double v = pos[3 * i + a];
            mn[a] = fmin(mn[a], v);
            mx[a] = fmax(mx[a], v);
        }
    for (int a = 0; a < 3; ++a) { smin[a][threadIdx.x] = mn[a]; smax[a][threadIdx.x] = mx[a]; }
    __syncthreads();
    for (int off = kBlock / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off)
            for (int a = 0; a < 3; ++a) {
                smin[a][threadIdx.x] = fmin(smin[a][threadIdx.x], smin[a][threadIdx.x + off]);
                smax[a][threadIdx.x] = fmax(smax[a][threadIdx.x], smax[a][threadIdx.x + off]);
            }
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int a = 0; a < 3; ++a) {
            partial[6 * blockIdx.x + a] = smin[a][0];
            partial[6 * blockIdx.x + 3 + a] = smax[a][0];
        }
}

__global__ void k_minmax_final(const double* __restrict__ partial, int np, double* __restrict__ out)
{
    if (threadIdx.x != 0) return;
    double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int b = 0; b < np; ++b)
        for (int a = 0; a < 3; ++a) {
            mn[a] = fmin(mn[a], partial[6 * b + a]);
            mx[a] = fmax(mx[a], partial[6 * b + 3 + a]);
        }
    for (int a = 0; a < 3; ++a) { out[a] = mn[a]; out[3 + a] = mx[a]; }
}

__device__ __forceinline__ int cell_coord(double v, double o, double cs, int nc)
{
    int c = (int)floor((v - o) / cs);
    return c < 0 ? 0 : (c >= nc ? nc - 1 : c);
}

__global__ void k_cell_count(const double* __restrict__ pos, int64_t n, int ncx, int ncy, int ncz,
                             double ox, double oy, double oz, double csx, double csy, double csz,
                             int32_t* __restrict__ cell, int32_t* __restrict__ count)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int cx = cell_coord(pos[3 * i], ox, csx, ncx);
    const int cy = cell_coord(pos[3 * i + 1], oy, csy, ncy);
    const int cz = cell_coord(pos[3 * i + 2], oz, csz, ncz);
    const int c = (cz * ncy + cy) * ncx + cx;
    cell[i] = c;
    atomicAdd(&count[c], 1);
}

// Exclusive scan of count[0..nc) into start[0..nc] with a single block of 1024
// threads: each thread scans a contiguous chunk, then the chunk totals.  Used for
// the tile totals of the cell scan below (at most 2^26 / kScanTile of them).
__global__ void __launch_bounds__(1024) k_scan(const int32_t* __restrict__ count, int nc,
                                               int32_t* __restrict__ start)
{
    __shared__ int32_t tot[1024];
    const int t = threadIdx.x;
    const int chunk = (nc + 1023) / 1024;
    const int lo = t * chunk, hi = min(nc, lo + chunk);
    int32_t s = 0;
    for (int i = lo; i < hi; ++i) s += count[i];
    tot[t] = s;
    __syncthreads();
    // Hillis-Steele inclusive scan of the 1024 totals
    for (int off = 1; off < 1024; off <<= 1) {
        const int32_t v = (t >= off) ? tot[t - off] : 0;
        __syncthreads();
        tot[t] += v;
        __syncthreads();
    }
    int32_t run = (t == 0) ? 0 : tot[t - 1];
    for (int i = lo; i < hi; ++i) {
        start[i] = run;
        run += count[i];
    }
    if (t == 1023) start[nc] = tot[1023];
}

// The cell scan in three passes over tiles of kScanTile cells: tile totals (reads
// coalesced across the block), the single-block scan of the totals, then each
// tile's own scan offset by its total's prefix.
constexpr int kScanTile = 4096;
constexpr int kScanPer = kScanTile / 256;

__global__ void __launch_bounds__(256) k_scan_tiles(const int32_t* __restrict__ count, int nc,
                                                    int32_t* __restrict__ tsum)
{
    __shared__ int32_t red[256];
    const int t = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    int32_t s = 0;
    for (int k = 0; k < kScanPer; ++k) {
        const int64_t i = base + k * 256 + t;
        if (i < nc) s += count[i];
    }
    red[t] = s;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (t < off) red[t] += red[t + off];
        __syncthreads();
    }
    if (t == 0) tsum[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(256) k_scan_apply(const int32_t* __restrict__ count, int nc,
                                                    const int32_t* __restrict__ toff, int32_t* __restrict__ start)
{
    __shared__ int32_t ws[256];
    const int t = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)t * kScanPer;
    int32_t v[kScanPer];
    int32_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        v[k] = (base + k < nc) ? count[base + k] : 0;
        s += v[k];
    }
    // Hillis-Steele inclusive scan of the 256 thread totals
    ws[t] = s;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const int32_t u = (t >= off) ? ws[t - off] : 0;
        __syncthreads();
        ws[t] += u;
        __syncthreads();
    }
    int32_t run = toff[blockIdx.x] + ws[t] - s;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        if (base + k < nc) start[base + k] = run;
        run += v[k];
    }
    // the thread holding the last cell also writes the grand total
    if (base < nc && nc <= base + kScanPer) start[nc] = run;
}

__global__ void k_scatter(const int32_t* __restrict__ cell, int64_t n, const int32_t* __restrict__ start,
                          int32_t* __restrict__ fill, int32_t* __restrict__ perm)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int c = cell[i];
    const int slot = start[c] + atomicAdd(&fill[c], 1);
    perm[slot] = (int32_t)i;
}

// Sort each cell's members by input index (insertion sort; cells are small).
__global__ void k_cell_sort(const int32_t* __restrict__ start, int nc, int32_t* __restrict__ perm)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nc) return;
    const int lo = start[c], hi = start[c + 1];
    for (int i = lo + 1; i < hi; ++i) {
        const int32_t v = perm[i];
        int j = i - 1;
        while (j >= lo && perm[j] > v) { perm[j + 1] = perm[j]; --j; }
        perm[j + 1] = v;
    }
}

__global__ void k_gather_sorted(const double* __restrict__ pos, const double* __restrict__ w,
                                const int32_t* __restrict__ perm, int64_t n,
                                double4* __restrict__ P, int32_t* __restrict__ inv)
{
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= n + kSentinels) return;
    if (k >= n) {   // sentinels past the last point: NaN position, never binned
        P[k] = make_double4(NAN, NAN, NAN, 0.0);
        return;
    }
    const int32_t i = perm[k];
    P[k] = make_double4(pos[3 * (int64_t)i], pos[3 * (int64_t)i + 1], pos[3 * (int64_t)i + 2], w[i]);
    inv[i] = (int32_t)k;
}

inline int nblocks(int64_t n) { return (int)((n + kBlock - 1) / kBlock); }

}  // namespace

__global__ void k_iota(int32_t* out, int64_t n)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) out[i] = (int32_t)i;
}

__global__ void k_map_subset(const int64_t* idx, int64_t k, const int32_t* inv, int64_t n, int32_t* out,
                             int* bad)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= k) return;
    const int64_t v = idx[i];
    if (v < 0 || v >= n) { atomicOr(bad, 1); out[i] = 0; return; }
    out[i] = inv[v];
}

__global__ void k_fill(double* p, int64_t n, double v)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_fill_u32(unsigned* p, int64_t n, unsigned v)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_f2d(const float* s, int64_t n, double* d)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) d[i] = (double)s[i];
}

int launch_iota(int32_t* out, int64_t n, hipStream_t stream)
{
    if (n <= 0) return 0;
    k_iota<<<nblocks(n), kBlock, 0, stream>>>(out, n);
    return (int)hipGetLastError();
}

int launch_map_subset(const int64_t* idx, int64_t k, const int32_t* inv, int64_t n, int32_t* out,
                      int* bad, hipStream_t stream)
{
    if (k <= 0) return 0;
    k_map_subset<<<nblocks(k), kBlock, 0, stream>>>(idx, k, inv, n, out, bad);
    return (int)hipGetLastError();
}

int launch_fill(double* p, int64_t n, double v, hipStream_t stream)
{
    if (n <= 0) return 0;
    k_fill<<<nblocks(n), kBlock, 0, stream>>>(p, n, v);
    return (int)hipGetLastError();
}

int launch_fill_u32(unsigned* p, int64_t n, unsigned v, hipStream_t stream)
{
    if (n <= 0) return 0;
    k_fill_u32<<<nblocks(n), kBlock, 0, stream>>>(p, n, v);
    return (int)hipGetLastError();
}

int launch_to_double(const void* src, int precision, int64_t n, double* dst, hipStream_t stream)
{
    if (n <= 0) return 0;
    if (precision == 0)
        return (int)hipMemcpyAsync(dst, src, sizeof(double) * n, hipMemcpyDeviceToDevice, stream);
    k_f2d<<<nblocks(n), kBlock, 0, stream>>>(static_cast<const float*>(src), n, dst);
    return (int)hipGetLastError();
}

// Split grid S (data then one random part) against the data-only grid D.
__global__ void k_split_check(const double4* __restrict__ PS, const int32_t* __restrict__ invS, int64_t n_data,
                              const double4* __restrict__ PD, const int32_t* __restrict__ invD,
                              int* __restrict__ bad)
{
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j >= n_data) return;
    const double4 q = PS[invS[j]];
    const double4 r = PD[invD[j]];
    if (!(q.x == r.x && q.y == r.y && q.z == r.z && q.w == r.w)) atomicOr(bad, 1);
}

__global__ void k_split_randoms(const double4* __restrict__ PS, const int32_t* __restrict__ invS, int64_t n_data,
                                int64_t n, double* __restrict__ pos, double* __restrict__ w)
{
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j >= n - n_data) return;
    const double4 q = PS[invS[n_data + j]];
    pos[3 * j] = q.x;
    pos[3 * j + 1] = q.y;
    pos[3 * j + 2] = q.z;
    w[j] = q.w;
}

int launch_split_check(const DevGrid& S, const DevGrid& D, int* bad, hipStream_t stream)
{
    if (S.n_data <= 0) return 0;
    k_split_check<<<nblocks(S.n_data), kBlock, 0, stream>>>(S.P, S.inv, S.n_data, D.P, D.inv, bad);
    return (int)hipGetLastError();
}

int launch_split_randoms(const DevGrid& S, double* pos, double* w, hipStream_t stream)
{
    if (S.n <= S.n_data) return 0;
    k_split_randoms<<<nblocks(S.n - S.n_data), kBlock, 0, stream>>>(S.P, S.inv, S.n_data, S.n, pos, w);
    return (int)hipGetLastError();
}

#define HIPCHK(x)                                                                   \
    do {                                                                            \
        hipError_t e_ = (x);                                                        \
        if (e_ != hipSuccess) {                                                     \
            snprintf(errbuf, errlen, "%s: %s", #x, hipGetErrorString(e_));          \
            goto fail;                                                              \
        }                                                                           \
    } while (0)

hipError_t dev_alloc(void** p, size_t bytes, hipMemPool_t pool, hipStream_t s)
{
    return pool ? hipMallocFromPoolAsync(p, bytes, pool, s) : hipMalloc(p, bytes);
}

void dev_free(void* p, hipMemPool_t pool, hipStream_t s)
{
    if (!p) return;
    if (pool) (void)hipFreeAsync(p, s);
    else (void)hipFree(p);
}

void grid_free(DevGrid& g, hipStream_t s)
{
    dev_free(g.P, g.pool, s);
    dev_free(g.perm, g.pool, s);
    dev_free(g.inv, g.pool, s);
    dev_free(g.cell_start, g.pool, s);
    g.P = nullptr; g.perm = nullptr; g.inv = nullptr; g.cell_start = nullptr;
}

// Returns 0 on success, -1 invalid input (errbuf says why), -3 no memory, -4 HIP error.
int grid_build(DevGrid& g, const double* d_pos, const double* d_w, int64_t n, int64_t n_data,
               bool dmr, bool periodic, const double box[3], double r_max, double cell_size,
               double cell_size_x, hipStream_t stream, char* errbuf, size_t errlen, hipMemPool_t pool)
{
    int rc = -4;
    int* d_flags = nullptr;
    double* d_part = nullptr;
    double* d_sums = nullptr;
    double* d_wn = nullptr;
    double* d_mm = nullptr;
    int32_t* d_cell = nullptr;
    int32_t* d_count = nullptr;
    int32_t* d_tsum = nullptr;
    int32_t* d_toff = nullptr;
    int flags = 0;
    double mm[6];
    const int npart = 512;
    int64_t ncell = 0;
    const double* wsrc = d_w;

    g.n = n;
    g.pool = pool;
    g.periodic = periodic ? 1 : 0;
    g.r_max = r_max;
    g.dmr = dmr ? 1 : 0;
    g.n_data = dmr ? n_data : n;
    if (n > kMaxGridPoints) {
        snprintf(errbuf, errlen, "catalog of %lld points exceeds the limit of one grid (%lld)",
                 (long long)n, (long long)kMaxGridPoints);
        return -1;
    }

    HIPCHK(dev_alloc((void**)&d_flags, sizeof(int), pool, stream));
    HIPCHK(hipMemsetAsync(d_flags, 0, sizeof(int), stream));
    k_validate<<<nblocks(n), kBlock, 0, stream>>>(d_pos, d_w, n, g.periodic, periodic ? box[0] : 0.0,
                                                  periodic ? box[1] : 0.0, periodic ? box[2] : 0.0, d_flags);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(&flags, d_flags, sizeof(int), hipMemcpyDeviceToHost, stream));
    HIPCHK(hipStreamSynchronize(stream));
    if (flags) {
        snprintf(errbuf, errlen, "invalid catalog:%s%s%s", (flags & 1) ? " non-finite position" : "",
                 (flags & 2) ? " non-finite weight" : "",
                 (flags & 4) ? " point outside the periodic box [0, L)" : "");
        rc = -1;
        goto fail;
    }

    HIPCHK(dev_alloc((void**)&d_part, sizeof(double) * 6 * npart, pool, stream));
    HIPCHK(dev_alloc((void**)&d_sums, sizeof(double) * 2, pool, stream));
    HIPCHK(dev_alloc((void**)&d_wn, sizeof(double) * n, pool, stream));
    if (dmr) {
        if (n_data < 1 || n_data >= n) {
            snprintf(errbuf, errlen, "ENCORE_DMR needs 1 <= n_data < n");
            rc = -1;
            goto fail;
        }
        k_wsum_partial<<<npart, kBlock, 0, stream>>>(d_w, 0, n_data, d_part);
        k_sum_final<<<1, kBlock, 0, stream>>>(d_part, npart, d_sums);
        k_wsum_partial<<<npart, kBlock, 0, stream>>>(d_w, n_data, n, d_part);
        k_sum_final<<<1, kBlock, 0, stream>>>(d_part, npart, d_sums + 1);
        HIPCHK(hipGetLastError());
        double sums[2];
        HIPCHK(hipMemcpyAsync(sums, d_sums, sizeof(sums), hipMemcpyDeviceToHost, stream));
        HIPCHK(hipStreamSynchronize(stream));
        if (sums[0] == 0.0 || sums[1] == 0.0) {
            snprintf(errbuf, errlen, "ENCORE_DMR: data or random weights sum to zero");
            rc = -1;
            goto fail;
        }
        k_dmr_weights<<<nblocks(n), kBlock, 0, stream>>>(d_w, n, n_data, d_sums, d_wn);
        HIPCHK(hipGetLastError());
        wsrc = d_wn;
    }

    // geometry
    if (periodic) {
        g.Lx = box[0]; g.Ly = box[1]; g.Lz = box[2];
        g.ox = g.oy = g.oz = 0.0;
        auto ncell_axis = [&](double L, double c) {
            int nc = (int)floor(L / c);
            return nc < 1 ? 1 : nc;
        };
        g.ncx = ncell_axis(box[0], cell_size_x);
        g.ncy = ncell_axis(box[1], cell_size);
        g.ncz = ncell_axis(box[2], cell_size);
        g.csx = box[0] / g.ncx; g.csy = box[1] / g.ncy; g.csz = box[2] / g.ncz;
    } else {
        HIPCHK(dev_alloc((void**)&d_mm, sizeof(double) * 6, pool, stream));
        k_minmax_partial<<<npart, kBlock, 0, stream>>>(d_pos, n, d_part);
        k_minmax_final<<<1, 64, 0, stream>>>(d_part, npart, d_mm);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(mm, d_mm, sizeof(mm), hipMemcpyDeviceToHost, stream));
        HIPCHK(hipStreamSynchronize(stream));
        g.Lx = g.Ly = g.Lz = 0.0;
        g.ox = mm[0]; g.oy = mm[1]; g.oz = mm[2];
        g.csx = cell_size_x;
        g.csy = g.csz = cell_size;
        g.ncx = (int)floor((mm[3] - mm[0]) / cell_size_x) + 1;
        g.ncy = (int)floor((mm[4] - mm[1]) / cell_size) + 1;
        g.ncz = (int)floor((mm[5] - mm[2]) / cell_size) + 1;
    }
    ncell = (int64_t)g.ncx * g.ncy * g.ncz;
    if (ncell > (1 << 26)) {
        snprintf(errbuf, errlen, "grid of %lld cells too large (r_max too small for the extent)",
                 (long long)ncell);
        rc = -1;
        goto fail;
    }

    HIPCHK(dev_alloc((void**)&d_cell, sizeof(int32_t) * n, pool, stream));
    HIPCHK(dev_alloc((void**)&d_count, sizeof(int32_t) * ncell, pool, stream));
    HIPCHK(dev_alloc((void**)&g.cell_start, sizeof(int32_t) * (ncell + 1), pool, stream));
    HIPCHK(dev_alloc((void**)&g.perm, sizeof(int32_t) * n, pool, stream));
    HIPCHK(dev_alloc((void**)&g.inv, sizeof(int32_t) * n, pool, stream));
    HIPCHK(dev_alloc((void**)&g.P, sizeof(double4) * (n + kSentinels), pool, stream));
    HIPCHK(hipMemsetAsync(d_count, 0, sizeof(int32_t) * ncell, stream));
    k_cell_count<<<nblocks(n), kBlock, 0, stream>>>(d_pos, n, g.ncx, g.ncy, g.ncz, g.ox, g.oy, g.oz,
                                                    g.csx, g.csy, g.csz, d_cell, d_count);
    {
        const int ntile = (int)((ncell + kScanTile - 1) / kScanTile);
        HIPCHK(dev_alloc((void**)&d_tsum, sizeof(int32_t) * ntile, pool, stream));
        HIPCHK(dev_alloc((void**)&d_toff, sizeof(int32_t) * (ntile + 1), pool, stream));
        k_scan_tiles<<<ntile, 256, 0, stream>>>(d_count, (int)ncell, d_tsum);
        k_scan<<<1, 1024, 0, stream>>>(d_tsum, ntile, d_toff);
        k_scan_apply<<<ntile, 256, 0, stream>>>(d_count, (int)ncell, d_toff, g.cell_start);
    }
    HIPCHK(hipMemsetAsync(d_count, 0, sizeof(int32_t) * ncell, stream));
    k_scatter<<<nblocks(n), kBlock, 0, stream>>>(d_cell, n, g.cell_start, d_count, g.perm);
    k_cell_sort<<<nblocks(ncell), kBlock, 0, stream>>>(g.cell_start, (int)ncell, g.perm);
    k_gather_sorted<<<nblocks(n + kSentinels), kBlock, 0, stream>>>(d_pos, wsrc, g.perm, n, g.P, g.inv);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(stream));
    rc = 0;

fail:
    dev_free(d_flags, pool, stream);
    dev_free(d_part, pool, stream);
    dev_free(d_sums, pool, stream);
    dev_free(d_wn, pool, stream);
    dev_free(d_mm, pool, stream);
    dev_free(d_cell, pool, stream);
    dev_free(d_count, pool, stream);
    dev_free(d_tsum, pool, stream);
    dev_free(d_toff, pool, stream);
    if (rc != 0) grid_free(g, stream);
    return rc;
}

}  // namespace encore
