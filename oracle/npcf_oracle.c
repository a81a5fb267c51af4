/*
 * Plain FP64 CPU oracle for the discrete isotropic NPCF estimator.
 * TEST INFRASTRUCTURE ONLY: called by tests/, by the smoke check and by the
 * cpu_baseline leg of bench.py; never by the product path.
 *
 * What it computes (Section 3.2.1, eqs. NPCF-mult-discrete-binned-estimator and
 * binned-discrete-alm, without the 1/V and 1/v_b normalisations):
 *
 *   a~^b_lm(i) = sum_{j != i} w_j Y_lm( (r_j - s_i)^ ) Theta^b(|r_j - s_i|)
 *   H^B_L(i)   = sum over ALL M with sum m = 0 of C^L_M prod_k a~^{b_k}_{l_k m_k}(i)
 *   Z^B_L      = sum_i w_i H^B_L(i)
 *
 * C^L_M already carries E(L) (eq. basis-coupling); the estimator multiplies by
 * E(L) C^L_M, so the caller passes E*C = E*E*(chain) per term.  The caller builds
 * the term list; this file only runs the loops.
 *
 * Readings of the paper taken here:
 *  - separation direction r_j - s_i (secondary minus primary), eq. binned-discrete-alm;
 *  - periodic boxes use the minimum image d <- d - L*round(d/L) per axis;
 *  - bin b holds edges[b]^2 <= r^2 < edges[b+1]^2, with r^2 = (dx*dx + dy*dy) + dz*dz
 *    evaluated in that order in FP64 (no fused multiply-add: build with
 *    -ffp-contract=off); pairs outside [edges[0], edges[nbins]) are skipped, and
 *    edges[0] > 0 removes the self pair j = i (Algorithm overview: j != i);
 *  - Y_lm is the orthonormal spherical harmonic with Condon-Shortley phase
 *    (Section 2.1), m < 0 from Y_{l,-m} = (-1)^m conj(Y_lm) (Appendix B).
 *
 * Y_lm: normalised associated Legendre functions by the standard three-term
 * recurrence in l at fixed m (DLMF 14.10.3 rescaled to unit norm), times
 * exp(i m phi) from cos/sin of m*phi with phi = atan2(dy, dx).
 *
 * The sum over primaries uses Neumaier-compensated FP64 per thread (OpenMP,
 * static schedule over primaries, as in the paper's CPU implementation section:
 * thread-private sums combined at the end), then a compensated combine in
 * thread order.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define NLM(lmax) (((lmax) + 1) * ((lmax) + 2) / 2)
#define LMI(l, m) ((l) * ((l) + 1) / 2 + (m))
#define ORACLE_LMAX 20

/* Y_lm for 0 <= m <= l <= lmax of the direction (dx, dy, dz) (need not be unit).
 * out[2*LMI(l,m)] = Re, out[2*LMI(l,m)+1] = Im.  Returns -1 for a zero vector. */
int oracle_ylm(int lmax, double dx, double dy, double dz, double* out)
{
    const double r = sqrt(dx * dx + dy * dy + dz * dz);
    if (!(r > 0.0)) return -1;
    const double ct = dz / r;
    const double rho = sqrt(dx * dx + dy * dy);
    const double st = rho / r;
    const double phi = atan2(dy, dx);
    if (lmax < 0 || lmax > ORACLE_LMAX) return -2;
    double P[NLM(ORACLE_LMAX)];
    /* P[LMI(l,m)] = normalised associated Legendre with CS phase, so that
       Y_lm = P_lm(cos theta) exp(i m phi). */
    P[LMI(0, 0)] = sqrt(1.0 / (4.0 * M_PI));
    for (int m = 1; m <= lmax; ++m)
        P[LMI(m, m)] = -sqrt((2.0 * m + 1.0) / (2.0 * m)) * st * P[LMI(m - 1, m - 1)];
    for (int m = 0; m < lmax; ++m)
        P[LMI(m + 1, m)] = sqrt(2.0 * m + 3.0) * ct * P[LMI(m, m)];
    for (int m = 0; m <= lmax; ++m) {
        for (int l = m + 2; l <= lmax; ++l) {
            const double a = sqrt((4.0 * l * l - 1.0) / ((double)l * l - (double)m * m));
            const double b = sqrt(((double)(l - 1) * (l - 1) - (double)m * m) /
                                  (4.0 * (l - 1) * (l - 1) - 1.0));
            P[LMI(l, m)] = a * (ct * P[LMI(l - 1, m)] - b * P[LMI(l - 2, m)]);
        }
    }
    for (int l = 0; l <= lmax; ++l) {
        for (int m = 0; m <= l; ++m) {
            out[2 * LMI(l, m)] = P[LMI(l, m)] * cos(m * phi);
            out[2 * LMI(l, m) + 1] = P[LMI(l, m)] * sin(m * phi);
        }
    }
    return 0;
}

/* Separation from primary i to secondary j, minimum image when box != NULL,
 * and its radial bin (-1 when outside every bin). */
static int pair_bin(const double* pos, int64_t i, int64_t j, const double* box,
                    const double* e2, int nbins, double d[3])
{
    for (int a = 0; a < 3; ++a) {
        double v = pos[3 * j + a] - pos[3 * i + a];
        if (box) v = v - box[a] * round(v / box[a]);
        d[a] = v;
    }
    const double r2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
    if (r2 < e2[0] || r2 >= e2[nbins]) return -1;
    int b = 0;
    while (b + 1 < nbins && r2 >= e2[b + 1]) ++b;
    return b;
}

/* Raw a~ for one primary: alm[(b*NLM + LMI(l,m))*2 + {0,1}]. */
static void primary_alm(const double* pos, const double* w, int64_t n, const double* box,
                        const double* e2, int nbins, int lmax, int64_t i,
                        double* alm, double* ybuf)
{
    const int nlm = NLM(lmax);
    memset(alm, 0, sizeof(double) * 2 * nlm * nbins);
    for (int64_t j = 0; j < n; ++j) {
        if (j == i) continue;
        double d[3];
        const int b = pair_bin(pos, i, j, box, e2, nbins, d);
        if (b < 0) continue;
        if (oracle_ylm(lmax, d[0], d[1], d[2], ybuf) != 0) continue;
        double* ab = alm + (size_t)2 * nlm * b;
        for (int q = 0; q < 2 * nlm; ++q) ab[q] += w[j] * ybuf[q];
    }
}

int oracle_alm(const double* pos, const double* w, int64_t n, const double* box,
               const double* edges, int nbins, int lmax,
               const int64_t* prim, int64_t nprim, double* alm_out, int nthreads)
{
    double* e2 = (double*)malloc(sizeof(double) * (nbins + 1));
    for (int k = 0; k <= nbins; ++k) e2[k] = edges[k] * edges[k];
    const int nlm = NLM(lmax);
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel
    {
        double* ybuf = (double*)malloc(sizeof(double) * 2 * nlm);
#pragma omp for schedule(static)
        for (int64_t p = 0; p < nprim; ++p)
            primary_alm(pos, w, n, box, e2, nbins, lmax, prim[p],
                        alm_out + (size_t)p * 2 * nlm * nbins, ybuf);
        free(ybuf);
    }
    free(e2);
    return 0;
}

/* a~^b_{l,m} for any sign of m, from the stored m >= 0 values. */
static inline void get_a(const double* alm, int nlm, int b, int l, int m, double* re, double* im)
{
    const int am = m < 0 ? -m : m;
    const double* p = alm + (size_t)2 * (nlm * b + LMI(l, am));
    if (m >= 0) { *re = p[0]; *im = p[1]; }
    else {
        const double s = (am & 1) ? -1.0 : 1.0;
        *re = s * p[0]; *im = -s * p[1];
    }
}

static inline void neumaier_add(double* sum, double* comp, double x)
{
    const double t = *sum + x;
    if (fabs(*sum) >= fabs(x)) *comp += (*sum - t) + x;
    else *comp += (x - t) + *sum;
    *sum = t;
}

/* Z^B_L = sum_i w_i H^B_L(i).
 *  nk = N-1; terms: term_lam[t], term_l[t*nk+k], term_m[t*nk+k], term_c[t] (= E*C);
 *  btab[bidx*nk+k] bin tuples.
 *  Outputs (nlam*nB each): z_re, z_im; abs_re/abs_im = sum_i |w_i Re/Im H(i)|. */
int oracle_zeta(const double* pos, const double* w, int64_t n, const double* box,
                const double* edges, int nbins, int lmax, int nk,
                int nlam, int nterm, const int* term_lam, const int* term_l,
                const int* term_m, const double* term_c,
                int nB, const int* btab,
                const int64_t* prim, int64_t nprim,
                double* z_re, double* z_im, double* abs_re, double* abs_im, int nthreads)
{
    double* e2 = (double*)malloc(sizeof(double) * (nbins + 1));
    for (int k = 0; k <= nbins; ++k) e2[k] = edges[k] * edges[k];
    const int nlm = NLM(lmax);
    const size_t nout = (size_t)nlam * nB;
    if (nthreads > 0) omp_set_num_threads(nthreads);
    const int nt = omp_get_max_threads();
    /* per-thread: sum_re, comp_re, sum_im, comp_im, abs_re, abs_im */
    double* acc = (double*)calloc((size_t)nt * 6 * nout, sizeof(double));
#pragma omp parallel
    {
        const int tid = omp_get_thread_num();
        double* my = acc + (size_t)tid * 6 * nout;
        double* alm = (double*)malloc(sizeof(double) * 2 * nlm * nbins);
        double* ybuf = (double*)malloc(sizeof(double) * 2 * nlm);
        double* H = (double*)malloc(sizeof(double) * 2 * nout);
#pragma omp for schedule(static)
        for (int64_t p = 0; p < nprim; ++p) {
            const int64_t i = prim[p];
            primary_alm(pos, w, n, box, e2, nbins, lmax, i, alm, ybuf);
            memset(H, 0, sizeof(double) * 2 * nout);
            for (int bi = 0; bi < nB; ++bi) {
                const int* B = btab + (size_t)bi * nk;
                for (int t = 0; t < nterm; ++t) {
                    double pr = 1.0, pi = 0.0;
                    for (int k = 0; k < nk; ++k) {
                        double ar, ai;
                        get_a(alm, nlm, B[k], term_l[t * nk + k], term_m[t * nk + k], &ar, &ai);
                        const double nr = pr * ar - pi * ai;
                        const double ni = pr * ai + pi * ar;
                        pr = nr; pi = ni;
                    }
                    double* h = H + 2 * ((size_t)term_lam[t] * nB + bi);
                    h[0] += term_c[t] * pr;
                    h[1] += term_c[t] * pi;
                }
            }
            const double wi = w[i];
            for (size_t o = 0; o < nout; ++o) {
                const double xr = wi * H[2 * o], xi = wi * H[2 * o + 1];
                neumaier_add(&my[0 * nout + o], &my[1 * nout + o], xr);
                neumaier_add(&my[2 * nout + o], &my[3 * nout + o], xi);
                my[4 * nout + o] += fabs(xr);
                my[5 * nout + o] += fabs(xi);
            }
        }
        free(alm); free(ybuf); free(H);
    }
    for (size_t o = 0; o < nout; ++o) {
        double sr = 0.0, cr = 0.0, si = 0.0, ci = 0.0, ar = 0.0, ai = 0.0;
        for (int t = 0; t < nt; ++t) {
            const double* my = acc + (size_t)t * 6 * nout;
            neumaier_add(&sr, &cr, my[0 * nout + o]);
            neumaier_add(&sr, &cr, my[1 * nout + o]);
            neumaier_add(&si, &ci, my[2 * nout + o]);
            neumaier_add(&si, &ci, my[3 * nout + o]);
            ar += my[4 * nout + o];
            ai += my[5 * nout + o];
        }
        z_re[o] = sr + cr; z_im[o] = si + ci;
        if (abs_re) abs_re[o] = ar;
        if (abs_im) abs_im[o] = ai;
    }
    free(acc); free(e2);
    return 0;
}
