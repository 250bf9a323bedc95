/*
 * EFGP oracle: direct O(N*M) exponential sums and the dense Toeplitz
 * (multilevel Toeplitz) matrix, in plain C, FP64 throughout.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is part of the correctness oracle.
 * It shares no code with the GPU library and must never be called by the
 * product path.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it.
 *
 * Conventions (paper Sec. 3.2, eqs. (88), (rhs), (223), (muws)):
 *   - multi-index j = (j^(1),...,j^(d)), each j^(l) in {-K..K}; arrays over
 *     J_K are stored in C order, offset j^(l)+K per dimension, last
 *     dimension fastest, length (2K+1)^d;
 *   - points are stored structure-of-arrays: coordinate l of point i is
 *     x[l*n + i];
 *   - complex arrays are interleaved (re, im) doubles.
 *
 * Every sum is evaluated literally: one complex exponential per
 * (point, frequency, dimension) from sin/cos of the phase reduced to
 * [-1/2, 1/2] cycles, then the tensor product.  Parallel sums use a fixed
 * chunking of the points and a fixed-order reduction, so results do not
 * depend on the number of threads.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define TWO_PI 6.283185307179586476925286766559

/* tab[j+K] = exp(sign * 2 pi i * h * j * x) for j = -K..K. */
static void phase_table(double h, double x, int K, int sign, double *re, double *im)
{
    for (int j = -K; j <= K; j++) {
        double t = h * (double)j * x;       /* phase in cycles */
        t -= nearbyint(t);                  /* reduce to [-1/2, 1/2] */
        double a = TWO_PI * t;
        re[j + K] = cos(a);
        im[j + K] = (double)sign * sin(a);
    }
}

static int64_t ipow(int64_t b, int e) { int64_t r = 1; while (e-- > 0) r *= b; return r; }

/*
 * Type-1 sum (eqs. (88) and (rhs)):
 *   out[j] = sum_n c_n * exp(sign * 2 pi i h <j, x_n>),   j in J_K.
 * c_re/c_im may be NULL: NULL c_re means unit strengths, NULL c_im means
 * real strengths.  out has (2K+1)^d complex entries.
 */
int or_type1(int d, int64_t n, const double *x, const double *c_re, const double *c_im,
             int K, double h, int sign, double *out)
{
    if (d < 1 || d > 3 || n < 0 || K < 0) return -1;
    const int W = 2 * K + 1;
    const int64_t Mk = ipow(W, d);
    const int nchunk = (int)(n < 64 ? (n > 0 ? n : 1) : 64);
    double *part = (double *)calloc((size_t)nchunk * (size_t)Mk * 2, sizeof(double));
    if (!part) return -2;

    #pragma omp parallel
    {
        double *tr = (double *)malloc(sizeof(double) * 3 * W);
        double *ti = (double *)malloc(sizeof(double) * 3 * W);
        #pragma omp for schedule(dynamic, 1)
        for (int ch = 0; ch < nchunk; ch++) {
            int64_t i0 = n * ch / nchunk, i1 = n * (ch + 1) / nchunk;
            double *acc = part + (size_t)ch * Mk * 2;
            for (int64_t i = i0; i < i1; i++) {
                double cr = c_re ? c_re[i] : 1.0;
                double ci = c_im ? c_im[i] : 0.0;
                for (int l = 0; l < d; l++)
                    phase_table(h, x[(int64_t)l * n + i], K, sign, tr + l * W, ti + l * W);
                if (d == 1) {
                    for (int a = 0; a < W; a++) {
                        acc[2 * a]     += cr * tr[a] - ci * ti[a];
                        acc[2 * a + 1] += cr * ti[a] + ci * tr[a];
                    }
                } else if (d == 2) {
                    for (int a = 0; a < W; a++) {
                        double pr = cr * tr[a] - ci * ti[a], pi = cr * ti[a] + ci * tr[a];
                        double *row = acc + (size_t)a * W * 2;
                        const double *er = tr + W, *ei = ti + W;
                        for (int b = 0; b < W; b++) {
                            row[2 * b]     += pr * er[b] - pi * ei[b];
                            row[2 * b + 1] += pr * ei[b] + pi * er[b];
                        }
                    }
                } else {
                    for (int a = 0; a < W; a++) {
                        double pr = cr * tr[a] - ci * ti[a], pi = cr * ti[a] + ci * tr[a];
                        for (int b = 0; b < W; b++) {
                            double qr = pr * tr[W + b] - pi * ti[W + b];
                            double qi = pr * ti[W + b] + pi * tr[W + b];
                            double *row = acc + ((size_t)a * W + b) * W * 2;
                            const double *er = tr + 2 * W, *ei = ti + 2 * W;
                            for (int c = 0; c < W; c++) {
                                row[2 * c]     += qr * er[c] - qi * ei[c];
                                row[2 * c + 1] += qr * ei[c] + qi * er[c];
                            }
                        }
                    }
                }
            }
        }
        free(tr); free(ti);
    }
    /* fixed-order reduction over chunks */
    #pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < Mk * 2; e++) {
        double s = 0.0;
        for (int ch = 0; ch < nchunk; ch++) s += part[(size_t)ch * Mk * 2 + e];
        out[e] = s;
    }
    free(part);
    return 0;
}

/*
 * Type-2 sum (eq. (muws) with the basis (basis), step 6 of the EFGP
 * algorithm):
 *   out[i] = sum_{j in J_K} c_j * exp(sign * 2 pi i h <j, t_i>),  i < q.
 * coef holds (2K+1)^d complex values; out holds q complex values.
 */
int or_type2(int d, int64_t q, const double *t, const double *coef, int K, double h,
             int sign, double *out)
{
    if (d < 1 || d > 3 || q < 0 || K < 0) return -1;
    const int W = 2 * K + 1;
    #pragma omp parallel
    {
        double *tr = (double *)malloc(sizeof(double) * 3 * W);
        double *ti = (double *)malloc(sizeof(double) * 3 * W);
        #pragma omp for schedule(static)
        for (int64_t i = 0; i < q; i++) {
            for (int l = 0; l < d; l++)
                phase_table(h, t[(int64_t)l * q + i], K, sign, tr + l * W, ti + l * W);
            double sr = 0.0, si = 0.0;
            if (d == 1) {
                for (int a = 0; a < W; a++) {
                    sr += coef[2 * a] * tr[a] - coef[2 * a + 1] * ti[a];
                    si += coef[2 * a] * ti[a] + coef[2 * a + 1] * tr[a];
                }
            } else if (d == 2) {
                for (int a = 0; a < W; a++) {
                    double rr = 0.0, ri = 0.0;
                    const double *row = coef + (size_t)a * W * 2;
                    for (int b = 0; b < W; b++) {
                        rr += row[2 * b] * tr[W + b] - row[2 * b + 1] * ti[W + b];
                        ri += row[2 * b] * ti[W + b] + row[2 * b + 1] * tr[W + b];
                    }
                    sr += rr * tr[a] - ri * ti[a];
                    si += rr * ti[a] + ri * tr[a];
                }
            } else {
                for (int a = 0; a < W; a++) {
                    double ar = 0.0, ai = 0.0;
                    for (int b = 0; b < W; b++) {
                        double rr = 0.0, ri = 0.0;
                        const double *row = coef + ((size_t)a * W + b) * W * 2;
                        for (int c = 0; c < W; c++) {
                            rr += row[2 * c] * tr[2 * W + c] - row[2 * c + 1] * ti[2 * W + c];
                            ri += row[2 * c] * ti[2 * W + c] + row[2 * c + 1] * tr[2 * W + c];
                        }
                        ar += rr * tr[W + b] - ri * ti[W + b];
                        ai += rr * ti[W + b] + ri * tr[W + b];
                    }
                    sr += ar * tr[a] - ai * ti[a];
                    si += ar * ti[a] + ai * tr[a];
                }
            }
            out[2 * i] = sr;
            out[2 * i + 1] = si;
        }
        free(tr); free(ti);
    }
    return 0;
}

/* decompose a C-order flat index over J_m into offsets j^(l)+m */
static void unflat(int64_t p, int d, int W, int *o)
{
    for (int l = d - 1; l >= 0; l--) { o[l] = (int)(p % W); p /= W; }
}

/*
 * Multilevel Toeplitz product (eq. (223)):
 *   out_p = sum_l v_{j_p - j_l} * beta_l,   p, l over J_m,
 * with v given on J_2m.  O(M^2).
 */
int or_toeplitz_apply(int d, int m, const double *v, const double *beta, double *out)
{
    if (d < 1 || d > 3 || m < 0) return -1;
    const int W = 2 * m + 1, W2 = 4 * m + 1;
    const int64_t M = ipow(W, d);
    #pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < M; p++) {
        int op[3] = {0, 0, 0}, ol[3] = {0, 0, 0};
        unflat(p, d, W, op);
        double sr = 0.0, si = 0.0;
        for (int64_t l = 0; l < M; l++) {
            unflat(l, d, W, ol);
            int64_t k = 0;
            for (int a = 0; a < d; a++) k = k * W2 + (op[a] - ol[a] + 2 * m);
            double vr = v[2 * k], vi = v[2 * k + 1];
            sr += vr * beta[2 * l] - vi * beta[2 * l + 1];
            si += vr * beta[2 * l + 1] + vi * beta[2 * l];
        }
        out[2 * p] = sr;
        out[2 * p + 1] = si;
    }
    return 0;
}

/*
 * Dense system matrix of eq. (97): A = D T D + sigma2 I with T_{pl} =
 * v_{j_p - j_l}.  out is M x M complex, row-major.
 */
int or_system_dense(int d, int m, const double *v, const double *D, double sigma2, double *out)
{
    if (d < 1 || d > 3 || m < 0) return -1;
    const int W = 2 * m + 1, W2 = 4 * m + 1;
    const int64_t M = ipow(W, d);
    #pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < M; p++) {
        int op[3] = {0, 0, 0}, ol[3] = {0, 0, 0};
        unflat(p, d, W, op);
        for (int64_t l = 0; l < M; l++) {
            unflat(l, d, W, ol);
            int64_t k = 0;
            for (int a = 0; a < d; a++) k = k * W2 + (op[a] - ol[a] + 2 * m);
            double s = D[p] * D[l];
            out[2 * (p * M + l)]     = s * v[2 * k] + (p == l ? sigma2 : 0.0);
            out[2 * (p * M + l) + 1] = s * v[2 * k + 1];
        }
    }
    return 0;
}

/*
 * Type-1 sums at selected multi-indices only (eqs. (88), (rhs)), for
 * checking single entries of very large problems:
 *   out[k] = sum_n c_n exp(sign * 2 pi i h <j_k, x_n>),  k < nj,
 * with j_k = jlist[k*d .. k*d+d-1].  Points are split into 256 fixed chunks
 * summed in a fixed order.
 */
int or_type1_select(int d, int64_t n, const double *x, const double *c_re, int nj,
                    const int *jlist, double h, int sign, double *out)
{
    if (d < 1 || d > 3 || n < 0 || nj < 0) return -1;
    const int nchunk = 256;
    double *part = (double *)calloc((size_t)nchunk * nj * 2, sizeof(double));
    if (!part) return -2;
    #pragma omp parallel for schedule(dynamic, 1)
    for (int ch = 0; ch < nchunk; ch++) {
        int64_t i0 = n * ch / nchunk, i1 = n * (ch + 1) / nchunk;
        double *acc = part + (size_t)ch * nj * 2;
        for (int64_t i = i0; i < i1; i++) {
            double cr = c_re ? c_re[i] : 1.0;
            for (int k = 0; k < nj; k++) {
                double t = 0.0;
                for (int l = 0; l < d; l++) {
                    double u = h * (double)jlist[k * d + l] * x[(int64_t)l * n + i];
                    t += u - nearbyint(u);   /* each term reduced to [-1/2, 1/2] cycles */
                }
                double a = TWO_PI * t;
                acc[2 * k]     += cr * cos(a);
                acc[2 * k + 1] += cr * (double)sign * sin(a);
            }
        }
    }
    for (int k = 0; k < nj * 2; k++) {
        double s = 0.0;
        for (int ch = 0; ch < nchunk; ch++) s += part[(size_t)ch * nj * 2 + k];
        out[k] = s;
    }
    free(part);
    return 0;
}

int or_num_threads(void) { return omp_get_max_threads(); }
