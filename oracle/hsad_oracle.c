/*
 * hsad_oracle.c -- plain FP64 CPU oracle for DWT-reduced local anomaly detection.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link or call
 * this file; only the tests, the smoke check and the benchmark's CPU-baseline leg use it.
 * It shares no code, header, table or constant with the HIP library.
 *
 * Method: Zare Baghbidi, Jamshidi, Naghsh Nilchi, Homayouni, "Improvement of anomaly
 * detection algorithms in hyperspectral images using discrete wavelet transform",
 * SIPIJ 2(4), 2011.
 *   - Sec. 3, eqs. (8)-(9), Fig. 1: one analysis level, low-pass y_low[k] = sum_n x[n] h[2k-n],
 *     high-pass with g, iterated on the low-pass branch.
 *   - Sec. 4: keep only the approximation coefficients of every pixel spectrum.
 *   - Sec. 2.1, eq. (1): RX score (r-mu)^T C^-1 (r-mu); local background window (LRX).
 *   - Sec. 2.2, eqs. (2)-(4): DWEST on the difference covariance of inner/outer windows.
 *   - Sec. 2.3, eq. (5): DWRX, m_diff^T C_outer^-1 m_diff.
 *
 * Everything is computed in double precision straight from the definitions: windows are
 * gathered pixel by pixel, means and covariances are two-pass (exact centring), the loaded
 * covariance is factored by an unblocked Cholesky, and DWEST uses a cyclic Jacobi
 * eigensolver.  Pixels are independent; OpenMP only splits the pixel list across threads.
 *
 * Readings of points the paper leaves open (each one is also listed in the design notes):
 *   periodised filtering with index (2k - m) mod n; an odd-length level input is extended
 *   by repeating its last sample; square windows centred on the pixel and clipped to the
 *   image; background = outer window minus inner window (inner = 0 means no guard window);
 *   covariances normalised by the sample count; diagonal loading
 *   lambda = load_rel * tr(C)/L' with a floor of 1e-30; DWEST keeps eigenvalues greater
 *   than 1e-12 * max|lambda| and reports ||V_P^T m_diff||_2 and sum_P |v_i^T m_diff|.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define ORC_LOAD_FLOOR 1e-30
#define ORC_POS_EIG_REL 1e-12

/* Thread count for the pixel loops (n <= 0 leaves the runtime default). */
void orc_set_threads(int n)
{
    if (n > 0) omp_set_num_threads(n);
}

int orc_max_threads(void) { return omp_get_max_threads(); }

/* ------------------------------------------------------------------------------------ */
/* DWT (Sec. 3, eqs. 8-9; Sec. 4)                                                        */
/* ------------------------------------------------------------------------------------ */

/* Length of the approximation after `levels` levels; -1 if a level input would be < 2. */
int64_t orc_dwt_out_len(int64_t L, int levels)
{
    if (L < 1 || levels < 0) return -1;
    int64_t n = L;
    for (int j = 0; j < levels; ++j) {
        if (n < 2) return -1;
        n = (n + 1) / 2;
    }
    return n;
}

static int64_t pmod(int64_t a, int64_t n)
{
    int64_t r = a % n;
    return r < 0 ? r + n : r;
}

/* One analysis level of eqs. (8)-(9) on a periodised signal.  If n is odd the signal is
 * first extended to n+1 samples by repeating x[n-1].  a (and d, if not NULL) receive
 * ne/2 values where ne is the (even) extended length. */
void orc_dwt_level(const double *x, int64_t n, const double *h, int ntaps,
                   double *a, double *d)
{
    int64_t ne = n + (n & 1);
    int64_t m = ne / 2;
    for (int64_t k = 0; k < m; ++k) {
        double sa = 0.0, sd = 0.0;
        for (int t = 0; t < ntaps; ++t) {
            int64_t i = pmod(2 * k - t, ne);
            double xv = (i < n) ? x[i] : x[n - 1];
            sa += h[t] * xv;
            if (d) {
                /* quadrature mirror: g[t] = (-1)^t h[ntaps-1-t] */
                double g = ((t & 1) ? -1.0 : 1.0) * h[ntaps - 1 - t];
                sd += g * xv;
            }
        }
        a[k] = sa;
        if (d) d[k] = sd;
    }
}

/* Approximation coefficients after `levels` levels for each of npix spectra of length L
 * (row-major pixel x band).  out holds npix * L' doubles. Returns L' or -1. */
int64_t orc_dwt_approx(const float *cube, int64_t npix, int64_t L, int levels,
                       const double *h, int ntaps, double *out)
{
    int64_t Lp = orc_dwt_out_len(L, levels);
    if (Lp < 0) return -1;
#pragma omp parallel
    {
        double *buf0 = (double *)malloc(sizeof(double) * (size_t)(L + 1));
        double *buf1 = (double *)malloc(sizeof(double) * (size_t)(L + 1));
#pragma omp for schedule(static)
        for (int64_t p = 0; p < npix; ++p) {
            const float *src = cube + p * L;
            for (int64_t i = 0; i < L; ++i) buf0[i] = (double)src[i];
            double *cur = buf0, *nxt = buf1;
            int64_t n = L;
            for (int j = 0; j < levels; ++j) {
                orc_dwt_level(cur, n, h, ntaps, nxt, NULL);
                n = (n + 1) / 2;
                double *t = cur; cur = nxt; nxt = t;
            }
            memcpy(out + p * Lp, cur, sizeof(double) * (size_t)Lp);
        }
        free(buf0);
        free(buf1);
    }
    return Lp;
}

/* Length of the full decomposition [a_J d_J d_{J-1} ... d_1] (Sec. 3, last paragraph):
 * level j maps its input of length n_{j-1} to a_j and d_j of n_j = ceil(n_{j-1}/2) samples
 * each (an odd input is first extended by repeating its last sample, as for the
 * approximation), so the total is n_J + n_J + n_{J-1} + ... + n_1.  -1 if a level input
 * would be shorter than 2. */
int64_t orc_dwt_full_len(int64_t L, int levels)
{
    if (L < 1 || levels < 0) return -1;
    int64_t n = L, tot = 0;
    for (int j = 0; j < levels; ++j) {
        if (n < 2) return -1;
        n = (n + 1) / 2;
        tot += n;
    }
    return tot + n;
}

/* Full decomposition of one signal of length n into out (orc_dwt_full_len values):
 * a_J first, then d_J, d_{J-1}, ..., d_1.  Returns 0 or -1. */
int orc_dwt_full(const double *x, int64_t n, int levels, const double *h, int ntaps,
                 double *out)
{
    const int64_t tot = orc_dwt_full_len(n, levels);
    if (tot < 0) return -1;
    double *cur = (double *)malloc(sizeof(double) * (size_t)(n + 1));
    double *a = (double *)malloc(sizeof(double) * (size_t)(n + 1));
    memcpy(cur, x, sizeof(double) * (size_t)n);
    int64_t len = n, end = tot;           /* d_j is written just below `end` */
    for (int j = 0; j < levels; ++j) {
        const int64_t m = (len + 1) / 2;
        orc_dwt_level(cur, len, h, ntaps, a, out + end - m);
        end -= m;
        memcpy(cur, a, sizeof(double) * (size_t)m);
        len = m;
    }
    memcpy(out, cur, sizeof(double) * (size_t)len);
    free(cur);
    free(a);
    return 0;
}

/* Synthesis of one level: the adjoint of the (orthogonal, for an even length n) analysis
 * matrix, x = A^T a + D^T d, with a and d of n/2 samples each. */
static void orc_level_adjoint(const double *a, const double *d, int64_t n, const double *h,
                              int ntaps, double *x)
{
    for (int64_t i = 0; i < n; ++i) x[i] = 0.0;
    for (int64_t k = 0; k < n / 2; ++k) {
        for (int t = 0; t < ntaps; ++t) {
            int64_t i = pmod(2 * k - t, n);
            double g = ((t & 1) ? -1.0 : 1.0) * h[ntaps - 1 - t];
            x[i] += h[t] * a[k] + g * d[k];
        }
    }
}

/* Inverse of orc_dwt_full for a signal of length n: level by level from the coarsest,
 * synthesis by the adjoint of the orthogonal level on the extended (even) length, then the
 * repeated sample of an odd level input is dropped.  Returns 0 or -1. */
int orc_idwt_full(const double *c, int64_t n, int levels, const double *h, int ntaps,
                  double *out)
{
    const int64_t tot = orc_dwt_full_len(n, levels);
    if (tot < 0) return -1;
    int64_t lens[64];
    lens[0] = n;
    for (int j = 0; j < levels; ++j) lens[j + 1] = (lens[j] + 1) / 2;
    double *cur = (double *)malloc(sizeof(double) * (size_t)(n + 1));
    double *nxt = (double *)malloc(sizeof(double) * (size_t)(n + 1));
    int64_t off = lens[levels];           /* d_J starts after a_J */
    memcpy(cur, c, sizeof(double) * (size_t)lens[levels]);
    for (int j = levels; j >= 1; --j) {
        const int64_t m = lens[j];
        orc_level_adjoint(cur, c + off, 2 * m, h, ntaps, nxt);
        off += m;
        memcpy(cur, nxt, sizeof(double) * (size_t)lens[j - 1]);   /* drops an extension */
    }
    memcpy(out, cur, sizeof(double) * (size_t)n);
    free(cur);
    free(nxt);
    return 0;
}

/* Full decomposition of every pixel spectrum of a cube (npix x L, float) into out
 * (npix x orc_dwt_full_len(L, levels) doubles).  Returns the output length or -1. */
int64_t orc_dwt_full_cube(const float *cube, int64_t npix, int64_t L, int levels, const double *h,
                          int ntaps, double *out)
{
    const int64_t tot = orc_dwt_full_len(L, levels);
    if (tot < 0) return -1;
#pragma omp parallel
    {
        double *buf = (double *)malloc(sizeof(double) * (size_t)L);
#pragma omp for schedule(static)
        for (int64_t p = 0; p < npix; ++p) {
            for (int64_t i = 0; i < L; ++i) buf[i] = (double)cube[p * L + i];
            orc_dwt_full(buf, L, levels, h, ntaps, out + p * tot);
        }
        free(buf);
    }
    return tot;
}

/* Inverse of orc_dwt_full_cube: npix rows of orc_dwt_full_len(L, levels) coefficients
 * (float) back to npix x L doubles.  Returns 0 or -1. */
int orc_idwt_full_cube(const float *coef, int64_t npix, int64_t L, int levels, const double *h,
                       int ntaps, double *out)
{
    const int64_t tot = orc_dwt_full_len(L, levels);
    if (tot < 0) return -1;
#pragma omp parallel
    {
        double *buf = (double *)malloc(sizeof(double) * (size_t)tot);
#pragma omp for schedule(static)
        for (int64_t p = 0; p < npix; ++p) {
            for (int64_t i = 0; i < tot; ++i) buf[i] = (double)coef[p * tot + i];
            orc_idwt_full(buf, L, levels, h, ntaps, out + p * L);
        }
        free(buf);
    }
    return 0;
}

/* ------------------------------------------------------------------------------------ */
/* Window statistics (Sec. 2.1 local background; Sec. 2.2 inner/outer windows)          */
/* ------------------------------------------------------------------------------------ */

typedef struct {
    int64_t n;          /* sample count */
    double *mean;       /* Lp */
    double *cov;        /* Lp*Lp, normalised by n */
} orc_stats;

static int in_box(int64_t dy, int64_t dx, int half)
{
    return llabs(dy) <= half && llabs(dx) <= half;
}

/* Rounding of a centred sample before it enters the covariance sums, for the
 * reduced-precision Gram modes: 0 keeps FP64; 1 rounds to binary32; 2 to bfloat16 and 3 to
 * binary16, each through binary32 first (round to nearest, ties to even at both steps). */
static double orc_round_sample(double v, int mode)
{
    if (mode == 0) return v;
    const float f = (float)v;
    if (mode == 1 || !isfinite(f)) return (double)f;
    if (mode == 2) {
        uint32_t b;
        memcpy(&b, &f, 4);
        b += 0x7FFFu + ((b >> 16) & 1u);
        b &= 0xFFFF0000u;
        float r;
        memcpy(&r, &b, 4);
        return (double)r;
    }
    /* binary16: 11 significant bits, quantum 2^(e - 11), at least 2^-24 (subnormals) */
    const double a = fabs((double)f);
    if (a == 0.0) return (double)f;
    int e;
    frexp(a, &e);
    int q = e - 11;
    if (q < -24) q = -24;
    const double r = ldexp(nearbyint(ldexp(a, -q)), q);
    return copysign(r > 65504.0 ? INFINITY : r, (double)f);
}

/* Exposed for tests: orc_round_sample over an array. */
void orc_round_samples(const double *v, int64_t n, int mode, double *out)
{
    for (int64_t i = 0; i < n; ++i) out[i] = orc_round_sample(v[i], mode);
}

/* Gathers the statistics of one pixel: annulus = outer window minus inner window (both
 * clipped to the image), and the inner window itself.  Two-pass: mean, then centred
 * outer products (of the centred samples rounded by orc_round_sample(., rnd)). */
static void orc_pixel_stats_r(const double *x, int64_t H, int64_t W, int64_t Lp, int inner,
                              int outer, int64_t py, int64_t px, orc_stats *ann,
                              orc_stats *inn, int rnd)
{
    const int ro = outer / 2, ri = inner / 2;
    const int64_t y0 = py - ro < 0 ? 0 : py - ro, y1 = py + ro >= H ? H - 1 : py + ro;
    const int64_t x0 = px - ro < 0 ? 0 : px - ro, x1 = px + ro >= W ? W - 1 : px + ro;
    orc_stats *sets[2] = {ann, inn};
    for (int s = 0; s < 2; ++s) {
        orc_stats *st = sets[s];
        if (!st) continue;
        st->n = 0;
        for (int64_t i = 0; i < Lp; ++i) st->mean[i] = 0.0;
        for (int64_t i = 0; i < Lp * Lp; ++i) st->cov[i] = 0.0;
    }
    /* pass 1: sums */
    for (int64_t y = y0; y <= y1; ++y)
        for (int64_t xx = x0; xx <= x1; ++xx) {
            int inside = inner > 0 && in_box(y - py, xx - px, ri);
            orc_stats *st = inside ? inn : ann;
            if (!st) continue;
            const double *v = x + (y * W + xx) * Lp;
            st->n += 1;
            for (int64_t i = 0; i < Lp; ++i) st->mean[i] += v[i];
        }
    for (int s = 0; s < 2; ++s) {
        orc_stats *st = sets[s];
        if (!st || st->n == 0) continue;
        for (int64_t i = 0; i < Lp; ++i) st->mean[i] /= (double)st->n;
    }
    /* pass 2: centred outer products */
    double *c = (double *)malloc(sizeof(double) * (size_t)Lp);
    for (int64_t y = y0; y <= y1; ++y)
        for (int64_t xx = x0; xx <= x1; ++xx) {
            int inside = inner > 0 && in_box(y - py, xx - px, ri);
            orc_stats *st = inside ? inn : ann;
            if (!st) continue;
            const double *v = x + (y * W + xx) * Lp;
            for (int64_t i = 0; i < Lp; ++i) c[i] = orc_round_sample(v[i] - st->mean[i], rnd);
            for (int64_t i = 0; i < Lp; ++i)
                for (int64_t j = 0; j < Lp; ++j) st->cov[i * Lp + j] += c[i] * c[j];
        }
    free(c);
    for (int s = 0; s < 2; ++s) {
        orc_stats *st = sets[s];
        if (!st || st->n == 0) continue;
        for (int64_t i = 0; i < Lp * Lp; ++i) st->cov[i] /= (double)st->n;
    }
}

static void orc_pixel_stats(const double *x, int64_t H, int64_t W, int64_t Lp, int inner,
                            int outer, int64_t py, int64_t px, orc_stats *ann,
                            orc_stats *inn)
{
    orc_pixel_stats_r(x, H, W, Lp, inner, outer, py, px, ann, inn, 0);
}

/* Exposed for tests: statistics of one pixel.  n_out = {n_annulus, n_inner}. */
void orc_window_stats(const double *x, int64_t H, int64_t W, int64_t Lp, int inner,
                      int outer, int64_t py, int64_t px, double *mu_a, double *C_a,
                      double *m_in, double *C_in, int64_t *n_out)
{
    orc_stats a = {0, mu_a, C_a}, b = {0, m_in, C_in};
    orc_pixel_stats(x, H, W, Lp, inner, outer, py, px, &a, &b);
    n_out[0] = a.n;
    n_out[1] = b.n;
}

/* ------------------------------------------------------------------------------------ */
/* Loading, Cholesky and the RX forms (eqs. 1 and 5)                                     */
/* ------------------------------------------------------------------------------------ */

double orc_loading(const double *C, int64_t Lp, double load_rel)
{
    double tr = 0.0;
    for (int64_t i = 0; i < Lp; ++i) tr += C[i * Lp + i];
    double lam = load_rel * tr / (double)Lp;
    return lam < ORC_LOAD_FLOOR ? ORC_LOAD_FLOOR : lam;
}

/* In-place lower Cholesky of A (n x n, row-major).  Returns 0, or -1 if a pivot is not
 * positive (the matrix is not numerically positive definite). */
int orc_cholesky(double *A, int64_t n)
{
    for (int64_t j = 0; j < n; ++j) {
        double s = A[j * n + j];
        for (int64_t k = 0; k < j; ++k) s -= A[j * n + k] * A[j * n + k];
        if (!(s > 0.0)) return -1;
        double ljj = sqrt(s);
        A[j * n + j] = ljj;
        for (int64_t i = j + 1; i < n; ++i) {
            double t = A[i * n + j];
            for (int64_t k = 0; k < j; ++k) t -= A[i * n + k] * A[j * n + k];
            A[i * n + j] = t / ljj;
        }
    }
    return 0;
}

/* ||L^-1 b||^2 = b^T (L L^T)^-1 b by forward substitution. */
static double orc_quad_form(const double *Lf, int64_t n, const double *b, double *z)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double t = b[i];
        for (int64_t k = 0; k < i; ++k) t -= Lf[i * n + k] * z[k];
        z[i] = t / Lf[i * n + i];
        s += z[i] * z[i];
    }
    return s;
}

/* LRX (eq. 1 with the annulus as local background) and DWRX (eq. 5) at the listed pixels.
 * x: H x W x Lp reduced cube.  Either output may be NULL.  A covariance that is not
 * positive definite after loading gives +inf. */
void orc_lrx_dwrx_rounded(const double *x, int64_t H, int64_t W, int64_t Lp, int inner, int outer,
                          double load_rel, const int64_t *idx, int64_t nidx, double *lrx,
                          double *dwrx, int rnd);

void orc_lrx_dwrx(const double *x, int64_t H, int64_t W, int64_t Lp, int inner, int outer,
                  double load_rel, const int64_t *idx, int64_t nidx, double *lrx,
                  double *dwrx)
{
    orc_lrx_dwrx_rounded(x, H, W, Lp, inner, outer, load_rel, idx, nidx, lrx, dwrx, 0);
}

/* As orc_lrx_dwrx, with each centred annulus sample rounded by orc_round_sample(., rnd)
 * before its outer product is summed (the Gram of the reduced-precision modes); the means
 * and the vectors x - mu, m_in - mu stay FP64. */
void orc_lrx_dwrx_rounded(const double *x, int64_t H, int64_t W, int64_t Lp, int inner, int outer,
                          double load_rel, const int64_t *idx, int64_t nidx, double *lrx,
                          double *dwrx, int rnd)
{
#pragma omp parallel
    {
        size_t l2 = (size_t)(Lp * Lp);
        double *mu = malloc(sizeof(double) * (size_t)Lp), *C = malloc(sizeof(double) * l2);
        double *mi = malloc(sizeof(double) * (size_t)Lp), *Ci = malloc(sizeof(double) * l2);
        double *d = malloc(sizeof(double) * (size_t)Lp), *z = malloc(sizeof(double) * (size_t)Lp);
#pragma omp for schedule(dynamic, 16)
        for (int64_t t = 0; t < nidx; ++t) {
            int64_t p = idx[t], py = p / W, px = p % W;
            orc_stats a = {0, mu, C}, b = {0, mi, Ci};
            orc_pixel_stats_r(x, H, W, Lp, inner, outer, py, px, &a, dwrx ? &b : NULL, rnd);
            double lam = orc_loading(C, Lp, load_rel);
            for (int64_t i = 0; i < Lp; ++i) C[i * Lp + i] += lam;
            int ok = orc_cholesky(C, Lp) == 0;
            if (lrx) {
                const double *r = x + p * Lp;
                for (int64_t i = 0; i < Lp; ++i) d[i] = r[i] - mu[i];
                lrx[t] = ok ? orc_quad_form(C, Lp, d, z) : INFINITY;
            }
            if (dwrx) {
                for (int64_t i = 0; i < Lp; ++i) d[i] = mi[i] - mu[i];
                /* |.| of eq. (5) is kept although the loaded form is never negative */
                dwrx[t] = ok ? fabs(orc_quad_form(C, Lp, d, z)) : INFINITY;
            }
        }
        free(mu); free(C); free(mi); free(Ci); free(d); free(z);
    }
}

/* Global RX (Sec. 2.1, eq. 1 with the background defined by all the image pixels):
 * mu and C = (1/N) sum (x - mu)(x - mu)^T over the N pixels (two passes, exact centring),
 * loading lambda = load_rel tr(C)/L' (floor 1e-30), and the score of each listed pixel.
 * The sums run over 64 fixed pixel ranges added in order, so the result does not depend
 * on the thread count.  mu_out (Lp) and C_out (Lp*Lp, before loading) may be NULL.
 * A covariance that is not positive definite after loading gives +inf everywhere. */
void orc_global_rx(const double *x, int64_t npix, int64_t Lp, double load_rel, const int64_t *idx,
                   int64_t nidx, double *scores, double *mu_out, double *C_out)
{
    enum { NR = 64 };
    const size_t l2 = (size_t)(Lp * Lp);
    double *mu = calloc((size_t)Lp, sizeof(double)), *C = calloc(l2, sizeof(double));
    double *pm = calloc((size_t)NR * (size_t)Lp, sizeof(double));
    double *pc = calloc((size_t)NR * l2, sizeof(double));
#pragma omp parallel for schedule(dynamic, 1)
    for (int r = 0; r < NR; ++r) {
        const int64_t p0 = npix * r / NR, p1 = npix * (r + 1) / NR;
        for (int64_t p = p0; p < p1; ++p)
            for (int64_t i = 0; i < Lp; ++i) pm[(size_t)r * Lp + i] += x[p * Lp + i];
    }
    for (int r = 0; r < NR; ++r)
        for (int64_t i = 0; i < Lp; ++i) mu[i] += pm[(size_t)r * Lp + i];
    for (int64_t i = 0; i < Lp; ++i) mu[i] /= (double)npix;
#pragma omp parallel for schedule(dynamic, 1)
    for (int r = 0; r < NR; ++r) {
        const int64_t p0 = npix * r / NR, p1 = npix * (r + 1) / NR;
        double *c = malloc(sizeof(double) * (size_t)Lp);
        double *acc = pc + (size_t)r * l2;
        for (int64_t p = p0; p < p1; ++p) {
            for (int64_t i = 0; i < Lp; ++i) c[i] = x[p * Lp + i] - mu[i];
            for (int64_t i = 0; i < Lp; ++i)
                for (int64_t j = 0; j < Lp; ++j) acc[i * Lp + j] += c[i] * c[j];
        }
        free(c);
    }
    for (int r = 0; r < NR; ++r)
        for (size_t e = 0; e < l2; ++e) C[e] += pc[(size_t)r * l2 + e];
    for (size_t e = 0; e < l2; ++e) C[e] /= (double)npix;
    if (mu_out) memcpy(mu_out, mu, sizeof(double) * (size_t)Lp);
    if (C_out) memcpy(C_out, C, sizeof(double) * l2);
    const double lam = orc_loading(C, Lp, load_rel);
    for (int64_t i = 0; i < Lp; ++i) C[i * Lp + i] += lam;
    const int ok = orc_cholesky(C, Lp) == 0;
#pragma omp parallel
    {
        double *d = malloc(sizeof(double) * (size_t)Lp), *z = malloc(sizeof(double) * (size_t)Lp);
#pragma omp for schedule(static)
        for (int64_t t = 0; t < nidx; ++t) {
            const double *r = x + idx[t] * Lp;
            for (int64_t i = 0; i < Lp; ++i) d[i] = r[i] - mu[i];
            scores[t] = ok ? orc_quad_form(C, Lp, d, z) : INFINITY;
        }
        free(d);
        free(z);
    }
    free(mu); free(C); free(pm); free(pc);
}

/* ------------------------------------------------------------------------------------ */
/* DWEST (Sec. 2.2, eqs. 2-4)                                                            */
/* ------------------------------------------------------------------------------------ */

/* Cyclic-by-row Jacobi eigensolver for a symmetric n x n matrix A (destroyed).
 * evals[i], eigenvector i in column i of V (row-major n x n).  Stops when the
 * off-diagonal Frobenius norm is <= tol_rel * ||A||_F.  Returns the sweeps used. */
int orc_jacobi_eig(int64_t n, double *A, double *evals, double *V, double tol_rel,
                   int max_sweeps)
{
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j) V[i * n + j] = (i == j) ? 1.0 : 0.0;
    double fro = 0.0;
    for (int64_t i = 0; i < n * n; ++i) fro += A[i] * A[i];
    fro = sqrt(fro);
    int sweep = 0;
    for (; sweep < max_sweeps; ++sweep) {
        double off = 0.0;
        for (int64_t i = 0; i < n; ++i)
            for (int64_t j = 0; j < n; ++j)
                if (i != j) off += A[i * n + j] * A[i * n + j];
        if (sqrt(off) <= tol_rel * fro) break;
        for (int64_t p = 0; p < n - 1; ++p)
            for (int64_t q = p + 1; q < n; ++q) {
                double apq = A[p * n + q];
                if (apq == 0.0) continue;
                /* rotation that annihilates A[p][q] (Golub & Van Loan, symmetric Schur) */
                double theta = (A[q * n + q] - A[p * n + p]) / (2.0 * apq);
                double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
                for (int64_t k = 0; k < n; ++k) {       /* A <- A J */
                    double akp = A[k * n + p], akq = A[k * n + q];
                    A[k * n + p] = c * akp - s * akq;
                    A[k * n + q] = s * akp + c * akq;
                }
                for (int64_t k = 0; k < n; ++k) {       /* A <- J^T A */
                    double apk = A[p * n + k], aqk = A[q * n + k];
                    A[p * n + k] = c * apk - s * aqk;
                    A[q * n + k] = s * apk + c * aqk;
                }
                for (int64_t k = 0; k < n; ++k) {       /* V <- V J */
                    double vkp = V[k * n + p], vkq = V[k * n + q];
                    V[k * n + p] = c * vkp - s * vkq;
                    V[k * n + q] = s * vkp + c * vkq;
                }
            }
    }
    for (int64_t i = 0; i < n; ++i) evals[i] = A[i * n + i];
    return sweep;
}

/* DWEST at the listed pixels: C_diff = C_inner - C_annulus (eq. 2), m_diff = m_inner -
 * m_annulus (eq. 3), projection of m_diff on the eigenvectors with positive eigenvalues
 * (eq. 4).  score = ||V_P^T m_diff||_2; literal = sum_P |v_i^T m_diff| (eq. 4 with each
 * eigenvector's sign chosen so that its projection is non-negative); npos = |P|.
 * Any output may be NULL. */
void orc_dwest(const double *x, int64_t H, int64_t W, int64_t Lp, int inner, int outer,
               const int64_t *idx, int64_t nidx, double *score, double *literal,
               int32_t *npos)
{
#pragma omp parallel
    {
        size_t l2 = (size_t)(Lp * Lp);
        double *mu = malloc(sizeof(double) * (size_t)Lp), *C = malloc(sizeof(double) * l2);
        double *mi = malloc(sizeof(double) * (size_t)Lp), *Ci = malloc(sizeof(double) * l2);
        double *ev = malloc(sizeof(double) * (size_t)Lp), *V = malloc(sizeof(double) * l2);
        double *md = malloc(sizeof(double) * (size_t)Lp);
#pragma omp for schedule(dynamic, 16)
        for (int64_t t = 0; t < nidx; ++t) {
            int64_t p = idx[t], py = p / W, px = p % W;
            orc_stats a = {0, mu, C}, b = {0, mi, Ci};
            orc_pixel_stats(x, H, W, Lp, inner, outer, py, px, &a, &b);
            for (int64_t i = 0; i < (int64_t)l2; ++i) Ci[i] -= C[i];
            for (int64_t i = 0; i < Lp; ++i) md[i] = mi[i] - mu[i];
            orc_jacobi_eig(Lp, Ci, ev, V, 1e-14, 100);
            double emax = 0.0;
            for (int64_t i = 0; i < Lp; ++i) emax = fmax(emax, fabs(ev[i]));
            double s2 = 0.0, s1 = 0.0;
            int32_t np = 0;
            for (int64_t i = 0; i < Lp; ++i) {
                if (!(ev[i] > ORC_POS_EIG_REL * emax)) continue;
                double pr = 0.0;
                for (int64_t k = 0; k < Lp; ++k) pr += V[k * Lp + i] * md[k];
                s2 += pr * pr;
                s1 += fabs(pr);
                ++np;
            }
            if (score) score[t] = sqrt(s2);
            if (literal) literal[t] = s1;
            if (npos) npos[t] = np;
        }
        free(mu); free(C); free(mi); free(Ci); free(ev); free(V); free(md);
    }
}
