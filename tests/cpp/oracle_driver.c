/* Runs the C oracle (oracle/npcf_oracle.c, compiled into this program) on inputs
 * written by tests/test_oracle_sanitized.py and writes its outputs, so that the
 * oracle can be built and run under AddressSanitizer + UndefinedBehaviorSanitizer.
 * Input (little-endian): int64 n, nbins, lmax, nk, nlam, nterm, nB, nprim,
 * periodic, nthreads; double pos[n*3], w[n], box[3], edges[nbins+1]; int32
 * t_lam[nterm], t_l[nterm*nk], t_m[nterm*nk]; double t_c[nterm]; int32
 * btab[nB*nk]; int64 prim[nprim].  Output: double z_re, z_im, abs_re, abs_im
 * [nlam*nB] each, then alm [nprim*nbins*nlm*2]. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_alm(const double* pos, const double* w, int64_t n, const double* box, const double* edges, int nbins,
               int lmax, const int64_t* prim, int64_t nprim, double* alm_out, int nthreads);
int oracle_zeta(const double* pos, const double* w, int64_t n, const double* box, const double* edges, int nbins,
                int lmax, int nk, int nlam, int nterm, const int* term_lam, const int* term_l, const int* term_m,
                const double* term_c, int nB, const int* btab, const int64_t* prim, int64_t nprim, double* z_re,
                double* z_im, double* abs_re, double* abs_im, int nthreads);

static void* rd(FILE* f, size_t size, size_t count)
{
    void* p = malloc(size * (count ? count : 1));
    if (!p || fread(p, size, count, f) != count) {
        fprintf(stderr, "short input\n");
        exit(2);
    }
    return p;
}

int main(int argc, char** argv)
{
    if (argc < 3) return 2;
    FILE* f = fopen(argv[1], "rb");
    if (!f) return 2;
    int64_t* h = (int64_t*)rd(f, sizeof(int64_t), 10);
    const int64_t n = h[0], nbins = h[1], lmax = h[2], nk = h[3], nlam = h[4], nterm = h[5], nB = h[6],
                  nprim = h[7], periodic = h[8], nthreads = h[9];
    double* pos = (double*)rd(f, sizeof(double), (size_t)n * 3);
    double* w = (double*)rd(f, sizeof(double), (size_t)n);
    double* box = (double*)rd(f, sizeof(double), 3);
    double* edges = (double*)rd(f, sizeof(double), (size_t)nbins + 1);
    int* t_lam = (int*)rd(f, sizeof(int), (size_t)nterm);
    int* t_l = (int*)rd(f, sizeof(int), (size_t)(nterm * nk));
    int* t_m = (int*)rd(f, sizeof(int), (size_t)(nterm * nk));
    double* t_c = (double*)rd(f, sizeof(double), (size_t)nterm);
    int* btab = (int*)rd(f, sizeof(int), (size_t)(nB * nk));
    int64_t* prim = (int64_t*)rd(f, sizeof(int64_t), (size_t)nprim);
    fclose(f);
    const size_t nout = (size_t)(nlam * nB);
    const size_t nalm = (size_t)nprim * nbins * ((lmax + 1) * (lmax + 2) / 2) * 2;
    double* z = (double*)calloc(4 * nout + 1, sizeof(double));
    double* alm = (double*)calloc(nalm + 1, sizeof(double));
    const double* bx = periodic ? box : NULL;
    oracle_zeta(pos, w, n, bx, edges, (int)nbins, (int)lmax, (int)nk, (int)nlam, (int)nterm, t_lam, t_l, t_m, t_c,
                (int)nB, btab, prim, nprim, z, z + nout, z + 2 * nout, z + 3 * nout, (int)nthreads);
    oracle_alm(pos, w, n, bx, edges, (int)nbins, (int)lmax, prim, nprim, alm, (int)nthreads);
    FILE* o = fopen(argv[2], "wb");
    if (!o) return 2;
    fwrite(z, sizeof(double), 4 * nout, o);
    fwrite(alm, sizeof(double), nalm, o);
    fclose(o);
    free(h); free(pos); free(w); free(box); free(edges); free(t_lam); free(t_l); free(t_m); free(t_c);
    free(btab); free(prim); free(z); free(alm);
    return 0;
}
