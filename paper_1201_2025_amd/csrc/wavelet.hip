// wavelet.hip -- the full periodised DWT (approximation and every detail band, Sec. 3, Fig. 1)
// and its inverse for the Daubechies family of any order N = 1..16 (2N taps, N vanishing
// moments; N = 1 is Haar), per pixel spectrum.
//
// Filter design (host, once per order).  The scaling filter is H(w) = ((1 + w)/2)^N Q(w)
// (w = e^{-i xi}, tap n multiplies w^n), where |Q|^2 on the unit circle is Daubechies'
// polynomial P(sin^2(xi/2)), P(y) = sum_{k<N} C(N-1+k, k) y^k (Ten Lectures on Wavelets,
// Sec. 6.1), and Q is taken minimum phase (no zeros in |w| < 1).  Q comes from the cepstral
// (Kolmogorov) spectral factorisation: log P sampled on M = 2^14 points of the circle, its
// Fourier coefficients folded onto n >= 0, exponentiated on the circle and transformed back
// (long-double FFTs).  P has no zeros on the circle, so the truncation error falls
// geometrically with M.  A Newton iteration in long double on the defining equations then
// polishes the taps: sum_k h_k h_{k+2m} = delta_m (m < N) and sum_k (-1)^k T_p(t_k) h_k = 0
// (p < N), with T_p Chebyshev polynomials of the centred tap index t_k in [-1, 1] (the same
// vanishing moments as the monomials k^p, better conditioned), normalised to sum h = sqrt 2.
//
// Transform (eqs. 8-9 with periodic index, the odd-length extension of the approximation
// branch used on both branches): level j maps n_{j-1} samples (odd n extended to n+1 by
// repeating the last one) to a_j[k] = sum_t h_t x[(2k - t) mod n_e] and
// d_j[k] = sum_t g_t x[(2k - t) mod n_e], g_t = (-1)^t h_{2N-1-t}, k < n_e / 2.  The output
// per pixel is [a_J d_J d_{J-1} ... d_1].  The inverse applies the transpose of each
// (orthogonal, even-length) level from the coarsest, x[i] = sum_t h_t a_k + g_t d_k over the
// pairs with (2k - t) mod n_e = i, and keeps the first n_{j-1} samples.
//
// Kernels: one workgroup holds PB pixels' spectra in LDS (FP64); each level runs over the
// (pixel, output) pairs of the workgroup; detail bands go straight to global memory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <mutex>
#include <string>
#include <vector>

#include "internal.hpp"

namespace hsad {

static constexpr int kMaxOrder = 16;
static constexpr int kMaxLevels = 24;
static constexpr int64_t kFullMaxL = 4096;

// ---- filter design -------------------------------------------------------------------
typedef long double ld;
typedef std::complex<ld> cld;

static void fft_ld(std::vector<cld> &a, bool inverse)
{
    const size_t n = a.size();
    for (size_t i = 1, j = 0; i < n; ++i) {
        size_t bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) std::swap(a[i], a[j]);
    }
    const ld pi = 3.141592653589793238462643383279502884L;
    for (size_t len = 2; len <= n; len <<= 1) {
        const ld ang = (inverse ? 2 : -2) * pi / (ld)len;
        for (size_t i = 0; i < n; i += len)
            for (size_t k = 0; k < len / 2; ++k) {
                const cld w(std::cos(ang * (ld)k), std::sin(ang * (ld)k));
                const cld u = a[i + k], v = a[i + k + len / 2] * w;
                a[i + k] = u + v;
                a[i + k + len / 2] = u - v;
            }
    }
    if (inverse)
        for (auto &v : a) v /= (ld)n;
}

static void solve_ld(std::vector<ld> &M, std::vector<ld> &b, int n)
{
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (std::fabs(M[r * n + c]) > std::fabs(M[piv * n + c])) piv = r;
        if (piv != c) {
            for (int k = 0; k < n; ++k) std::swap(M[c * n + k], M[piv * n + k]);
            std::swap(b[c], b[piv]);
        }
        for (int r = c + 1; r < n; ++r) {
            const ld f = M[r * n + c] / M[c * n + c];
            for (int k = c; k < n; ++k) M[r * n + k] -= f * M[c * n + k];
            b[r] -= f * b[c];
        }
    }
    for (int r = n - 1; r >= 0; --r) {
        ld s = b[r];
        for (int k = r + 1; k < n; ++k) s -= M[r * n + k] * b[k];
        b[r] = s / M[r * n + r];
    }
}

static void design_daubechies(int N, double *out)
{
    const int nt = 2 * N;
    std::vector<ld> h(nt, 0.0L);
    // minimum-phase factor Q of P(sin^2(xi/2)) by the cepstrum
    const int M = 1 << 14;
    std::vector<cld> a(M);
    const ld pi = 3.141592653589793238462643383279502884L;
    for (int j = 0; j < M; ++j) {
        const ld s = std::sin(pi * (ld)j / (ld)M);   // sin(xi/2), xi = 2 pi j / M
        const ld y = s * s;
        ld P = 0.0L, c = 1.0L;                       // C(N-1+k, k), built incrementally
        ld yk = 1.0L;
        for (int k = 0; k < N; ++k) {
            P += c * yk;
            yk *= y;
            c = c * (ld)(N + k) / (ld)(k + 1);
        }
        a[j] = cld(std::log(P), 0.0L);
    }
    fft_ld(a, true);   // cepstrum s_n of log P (real, even in n)
    // log Q(w) = sum_{n >= 0} c_n w^n with 2 Re log Q = log P on the circle:
    // c_0 = s_0 / 2, c_n = s_n (n >= 1), nothing at negative n
    for (auto &v : a) v = cld(v.real(), 0.0L);
    a[0] *= 0.5L;
    a[M / 2] = 0.0L;
    for (int n = M / 2 + 1; n < M; ++n) a[n] = 0.0L;
    fft_ld(a, false);
    for (auto &v : a) v = std::exp(v);
    fft_ld(a, true);                                  // coefficients of Q
    std::vector<ld> q(N);
    for (int n = 0; n < N; ++n) q[n] = a[n].real();
    // h = (1 + w)^N Q(w)
    std::vector<ld> b(N + 1, 0.0L);
    b[0] = 1.0L;
    for (int k = 0; k < N; ++k)
        for (int i = k + 1; i >= 1; --i) b[i] += b[i - 1];
    for (int i = 0; i <= N; ++i)
        for (int n = 0; n < N; ++n) h[i + n] += b[i] * q[n];
    ld sum = 0.0L;
    for (ld v : h) sum += v;
    const ld rt2 = std::sqrt(2.0L);
    for (ld &v : h) v *= rt2 / sum;
    // Newton on the defining equations (square system of 2N equations)
    std::vector<ld> tk(nt);
    const ld cen = (ld)(nt - 1) / 2.0L;
    for (int k = 0; k < nt; ++k) tk[k] = cen > 0 ? ((ld)k - cen) / cen : 0.0L;
    for (int it = 0; it < 12 && N > 1; ++it) {
        std::vector<ld> J((size_t)nt * nt, 0.0L), F(nt, 0.0L);
        for (int m = 0; m < N; ++m) {
            ld d = 0.0L;
            for (int k = 0; k + 2 * m < nt; ++k) {
                d += h[k] * h[k + 2 * m];
                J[(size_t)m * nt + k] += h[k + 2 * m];
                J[(size_t)m * nt + k + 2 * m] += h[k];
            }
            F[m] = d - (m == 0 ? 1.0L : 0.0L);
        }
        for (int k = 0; k < nt; ++k) {
            // Chebyshev T_p(t_k) by the recurrence, times (-1)^k
            ld t0 = 1.0L, t1 = tk[k];
            const ld sg = (k & 1) ? -1.0L : 1.0L;
            for (int p = 0; p < N; ++p) {
                const ld tp = p == 0 ? t0 : p == 1 ? t1 : 0.0L;
                ld v = tp;
                if (p >= 2) {
                    v = 2.0L * tk[k] * t1 - t0;
                    t0 = t1;
                    t1 = v;
                }
                J[(size_t)(N + p) * nt + k] = sg * v;
                F[N + p] += sg * v * h[k];
            }
        }
        ld fmax = 0.0L;
        for (ld v : F) fmax = std::max(fmax, std::fabs(v));
        solve_ld(J, F, nt);
        for (int k = 0; k < nt; ++k) h[k] -= F[k];
        if (fmax < 1e-19L) break;
    }
    for (int k = 0; k < nt; ++k) out[k] = (double)h[k];
}

static std::mutex g_filt_mu;
static std::vector<double> g_filt[kMaxOrder + 1];

const double *daubechies_filter(int N)
{
    if (N < 1 || N > kMaxOrder) return nullptr;
    std::lock_guard<std::mutex> lk(g_filt_mu);
    if (g_filt[N].empty()) {
        std::vector<double> h(2 * N);
        design_daubechies(N, h.data());
        g_filt[N] = h;
    }
    return g_filt[N].data();
}

// ---- kernels -------------------------------------------------------------------------
struct FullArgs {
    double h[2 * kMaxOrder], g[2 * kMaxOrder];
    int ntaps, J, L, tot;
    int len[kMaxLevels + 1];   // n_0 = L, n_1, ..., n_J
    int doff[kMaxLevels + 1];  // offset of d_j in the output row
    int PB, ldb;               // pixels per workgroup, LDS stride per pixel (doubles)
};

__global__ __launch_bounds__(256) void dwt_full_kernel(const float *__restrict__ in, float *__restrict__ out,
                                                       int64_t npix, FullArgs a)
{
    extern __shared__ double lds[];
    double *hs = lds, *gs = lds + 2 * kMaxOrder;
    double *bufA = lds + 4 * kMaxOrder, *bufB = bufA + (size_t)a.PB * a.ldb;
    const int t = threadIdx.x;
    const int64_t p0 = (int64_t)blockIdx.x * a.PB;
    const int np = (int)std::min<int64_t>(a.PB, npix - p0);
    if (t < a.ntaps) {
        hs[t] = a.h[t];
        gs[t] = a.g[t];
    }
    const int L = a.L;
    for (int e = t; e < np * L; e += 256) {
        const int pix = e / L, i = e - pix * L;
        bufA[pix * a.ldb + i] = (double)in[(p0 + pix) * L + i];
    }
    __syncthreads();
    double *cur = bufA, *nxt = bufB;
    for (int j = 1; j <= a.J; ++j) {
        const int n = a.len[j - 1], m = a.len[j], ne = 2 * m;
        if (n & 1) {
            if (t < np) cur[t * a.ldb + n] = cur[t * a.ldb + n - 1];
            __syncthreads();
        }
        for (int e = t; e < np * m; e += 256) {
            const int pix = e / m, k = e - pix * m;
            const double *x = cur + pix * a.ldb;
            double sa = 0.0, sd = 0.0;
            int i = 2 * k;
            for (int tt = 0; tt < a.ntaps; ++tt) {
                int ii = i - tt;
                while (ii < 0) ii += ne;
                const double v = x[ii];
                sa = fma(hs[tt], v, sa);
                sd = fma(gs[tt], v, sd);
            }
            float *orow = out + (p0 + pix) * a.tot;
            orow[a.doff[j] + k] = (float)sd;
            if (j < a.J)
                nxt[pix * a.ldb + k] = sa;
            else
                orow[k] = (float)sa;
        }
        __syncthreads();
        double *tmp = cur;
        cur = nxt;
        nxt = tmp;
    }
    if (a.J == 0)
        for (int e = t; e < np * L; e += 256) {
            const int pix = e / L, i = e - pix * L;
            out[(p0 + pix) * L + i] = (float)bufA[pix * a.ldb + i];
        }
}

__global__ __launch_bounds__(256) void idwt_full_kernel(const float *__restrict__ in, float *__restrict__ out,
                                                        int64_t npix, FullArgs a)
{
    extern __shared__ double lds[];
    double *hs = lds, *gs = lds + 2 * kMaxOrder;
    double *bufA = lds + 4 * kMaxOrder, *bufB = bufA + (size_t)a.PB * a.ldb, *dbuf = bufB + (size_t)a.PB * a.ldb;
    const int t = threadIdx.x;
    const int64_t p0 = (int64_t)blockIdx.x * a.PB;
    const int np = (int)std::min<int64_t>(a.PB, npix - p0);
    if (t < a.ntaps) {
        hs[t] = a.h[t];
        gs[t] = a.g[t];
    }
    const int nJ = a.len[a.J];
    for (int e = t; e < np * nJ; e += 256) {
        const int pix = e / nJ, i = e - pix * nJ;
        bufA[pix * a.ldb + i] = (double)in[(p0 + pix) * a.tot + i];
    }
    double *cur = bufA, *nxt = bufB;
    for (int j = a.J; j >= 1; --j) {
        const int m = a.len[j], ne = 2 * m, nprev = a.len[j - 1];
        for (int e = t; e < np * m; e += 256) {
            const int pix = e / m, k = e - pix * m;
            dbuf[pix * a.ldb + k] = (double)in[(p0 + pix) * a.tot + a.doff[j] + k];
        }
        __syncthreads();
        for (int e = t; e < np * nprev; e += 256) {
            const int pix = e / nprev, i = e - pix * nprev;
            const double *ac = cur + pix * a.ldb, *dc = dbuf + pix * a.ldb;
            double s = 0.0;
            for (int tt = i & 1; tt < a.ntaps; tt += 2) {
                int q = i + tt;
                while (q >= ne) q -= ne;
                const int k = q >> 1;
                s = fma(hs[tt], ac[k], s);
                s = fma(gs[tt], dc[k], s);
            }
            if (j > 1)
                nxt[pix * a.ldb + i] = s;
            else
                out[(p0 + pix) * a.L + i] = (float)s;
        }
        __syncthreads();
        double *tmp = cur;
        cur = nxt;
        nxt = tmp;
    }
    if (a.J == 0) {
        __syncthreads();
        for (int e = t; e < np * a.L; e += 256) {
            const int pix = e / a.L, i = e - pix * a.L;
            out[(p0 + pix) * a.L + i] = (float)bufA[pix * a.ldb + i];
        }
    }
}

static int full_setup(const char *fn, int64_t npix, int64_t L, int levels, int order, FullArgs *a, size_t *lds,
                      bool inverse)
{
    if (npix < 1) return fail(HSAD_EINVAL, std::string(fn) + ": npix must be >= 1");
    if (order < 1 || order > kMaxOrder) return fail(HSAD_EINVAL, std::string(fn) + ": order must be 1..16");
    if (L < 1 || levels < 0) return fail(HSAD_EINVAL, std::string(fn) + ": L < 1 or levels < 0");
    if (L > kFullMaxL) return fail(HSAD_EUNSUPPORTED, std::string(fn) + ": L above 4096");
    if (levels > kMaxLevels) return fail(HSAD_EINVAL, std::string(fn) + ": levels too deep for L");
    a->len[0] = (int)L;
    int tot = 0;
    for (int j = 1; j <= levels; ++j) {
        if (a->len[j - 1] < 2) return fail(HSAD_EINVAL, std::string(fn) + ": levels too deep for L");
        a->len[j] = (a->len[j - 1] + 1) / 2;
        tot += a->len[j];
    }
    tot += a->len[levels];
    a->tot = levels ? tot : (int)L;
    // d_J right after a_J, then d_{J-1}, ..., d_1 at the end
    int off = a->len[levels];
    for (int j = levels; j >= 1; --j) {
        a->doff[j] = off;
        off += a->len[j];
    }
    a->doff[0] = 0;
    a->J = levels;
    a->L = (int)L;
    const double *h = daubechies_filter(order);
    if (!h) return fail(HSAD_EINVAL, std::string(fn) + ": order must be 1..16");
    a->ntaps = 2 * order;
    for (int k = 0; k < 2 * kMaxOrder; ++k) {
        a->h[k] = k < a->ntaps ? h[k] : 0.0;
        a->g[k] = k < a->ntaps ? ((k & 1) ? -1.0 : 1.0) * h[a->ntaps - 1 - k] : 0.0;
    }
    a->ldb = (int)(L + 2) | 1;
    const int nbuf = inverse ? 3 : 2;
    const size_t per = (size_t)nbuf * a->ldb * sizeof(double);
    const size_t budget = 64 * 1024 - 4 * kMaxOrder * sizeof(double);
    int PB = (int)std::max<size_t>(1, budget / per);
    PB = std::min(PB, 64);
    a->PB = PB;
    *lds = 4 * kMaxOrder * sizeof(double) + (size_t)PB * per;
    return HSAD_OK;
}

}  // namespace hsad

using namespace hsad;

extern "C" int hsad_wavelet_filter(int order, double *h)
{
    clear_error();
    if (!h) return fail(HSAD_EINVAL, "hsad_wavelet_filter: h is NULL");
    const double *f = daubechies_filter(order);
    if (!f) return fail(HSAD_EINVAL, "hsad_wavelet_filter: order must be 1..16");
    std::copy(f, f + 2 * order, h);
    return HSAD_OK;
}

extern "C" int hsad_dwt_full_len(int64_t L, int levels, int64_t *n)
{
    clear_error();
    if (!n) return fail(HSAD_EINVAL, "hsad_dwt_full_len: n is NULL");
    if (L < 1 || levels < 0) return fail(HSAD_EINVAL, "hsad_dwt_full_len: L < 1 or levels < 0");
    int64_t m = L, tot = 0;
    for (int j = 0; j < levels; ++j) {
        if (m < 2) return fail(HSAD_EINVAL, "hsad_dwt_full_len: levels too deep for L");
        m = (m + 1) / 2;
        tot += m;
    }
    *n = levels ? tot + m : L;
    return HSAD_OK;
}

extern "C" int hsad_dwt_full(const float *cube, int64_t npix, int64_t L, int levels, int order, float *coef,
                             hipStream_t stream)
{
    clear_error();
    if (!cube || !coef) return fail(HSAD_EINVAL, "hsad_dwt_full: NULL pointer");
    FullArgs a;
    size_t lds = 0;
    if (int rc = full_setup("hsad_dwt_full", npix, L, levels, order, &a, &lds, false)) return rc;
    if (int rc = allow_lds((const void *)dwt_full_kernel, lds, "dwt_full_kernel")) return rc;
    const int64_t grid = (npix + a.PB - 1) / a.PB;
    if (grid > 0x7fffffff) return fail(HSAD_EUNSUPPORTED, "hsad_dwt_full: too many pixels");
    hipLaunchKernelGGL(dwt_full_kernel, dim3((unsigned)grid), dim3(256), lds, stream, cube, coef, npix, a);
    return check_launch("dwt_full_kernel");
}

extern "C" int hsad_idwt_full(const float *coef, int64_t npix, int64_t L, int levels, int order, float *cube,
                              hipStream_t stream)
{
    clear_error();
    if (!cube || !coef) return fail(HSAD_EINVAL, "hsad_idwt_full: NULL pointer");
    FullArgs a;
    size_t lds = 0;
    if (int rc = full_setup("hsad_idwt_full", npix, L, levels, order, &a, &lds, true)) return rc;
    if (int rc = allow_lds((const void *)idwt_full_kernel, lds, "idwt_full_kernel")) return rc;
    const int64_t grid = (npix + a.PB - 1) / a.PB;
    if (grid > 0x7fffffff) return fail(HSAD_EUNSUPPORTED, "hsad_idwt_full: too many pixels");
    hipLaunchKernelGGL(idwt_full_kernel, dim3((unsigned)grid), dim3(256), lds, stream, coef, cube, npix, a);
    return check_launch("idwt_full_kernel");
}
