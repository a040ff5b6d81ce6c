// eig.hip -- DWEST projection (Sec. 2.2, eqs. 2-4) by Householder tridiagonalisation and
// the implicit QL iteration, FP64, in two kernels.
//
// Input per pixel (chunk workspace, written by the Gram kernel in DWEST mode):
// rows 0..L'-1 = C_diff = C_inner - C_outer, row L' = m_diff = m_inner - m_outer.
// DWEST needs the eigenvalues of C_diff and the projections y_i = v_i^T m_diff, never the
// eigenvectors themselves.  Every orthogonal similarity applied to C_diff is therefore
// also applied to m_diff, as a vector:
//   1. tridiag_dwest_kernel (16, 32 or 64 lanes per pixel, the matrix in LDS, lane = row):
//      n-2 Householder reflections H_k = I - beta v v^T, each annihilating column k below
//      the subdiagonal, give T = Q^T C_diff Q tridiagonal and y = Q^T m_diff.  Per step:
//      p = beta A v, q = p - (beta/2)(v^T p) v, A <- A - v q^T - q v^T on the trailing
//      block, y <- y - beta (v^T y) v (Golub & Van Loan, Sec. 8.3.1).  The diagonal d,
//      the subdiagonal e and y overwrite the pixel's workspace.
//   2. ql_dwest_kernel (lane = pixel, d, e, y in LDS columns): the implicit QL iteration
//      with Wilkinson's shift on T (Golub & Van Loan, Sec. 8.3.5; the tql2 procedure of
//      Bowdler, Martin, Reinsch and Wilkinson); the rotation's 1/r is the hardware
//      reciprocal square root with two Newton steps.  Each plane rotation of a sweep is also
//      applied to y, which keeps y = V^T m_diff.  A subdiagonal entry counts as zero once
//      |e_m| <= eps max(|d_m| + |d_m+1|, max|d| + max|e| of the initial T), eps = 2^-52.
//      At most 64 sweeps per eigenvalue; a pixel that does not converge gets NaN scores.
// Eigenvalues above 1e-12 max|lambda| are "positive".  Outputs:
//   score   = ||V_P^T m_diff||_2 = sqrt(sum_P y_i^2)
//   literal = sum_P |y_i|          (eq. 4 with v_i signed so that v_i^T m_diff >= 0)
//   npos    = |P|
// Work per pixel: about 4/3 n^3 flops for step 1 and O(n^2) for step 2, against roughly
// 8 sweeps x 4 n^3 for a cyclic Jacobi solver.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <cstdint>

#include "internal.hpp"
#include "dev_lane.hpp"

namespace hsad {



__device__ __forceinline__ int tri(int i) { return i * (i + 1) / 2; }

// Sum over the G lanes of a lane group (G = 16, 32 or 64, aligned), the same value in every
// lane of the group: DPP within rows of 16, then one exchange between the two rows of a
// 32-lane group, or wave_sum64 for the whole wavefront.
template <int G> __device__ __forceinline__ double group_sum(double v)
{
    if constexpr (G == 64) {
        return wave_sum64(v);
    } else {
        v += dpp_f64<0xB1>(v);
        v += dpp_f64<0x4E>(v);
        v += dpp_f64<0x141>(v);
        v += dpp_f64<0x140>(v);
        if constexpr (G == 32) v += __shfl_xor(v, 16, 64);
        return v;
    }
}

// G lanes per pixel (64 / G pixels per 64-thread workgroup); rows i = gl, gl + G, ... of the
// group's pixel.  The symmetric matrix is kept as its packed lower triangle (row i at
// tri(i)): half the LDS of a square.  Element (i, j) of the trailing block is read at
// tri(max) + min; the rank-2 update writes the lower triangle only (a predicated store after
// an unconditional read).  A column that is already reduced takes no reflection (beta = 0,
// v = 0: every update adds exact zeros), so the groups of a wavefront stay in step.
// With dey set, d, e and y go to dey[i * S], dey[(n + i) * S] and dey[(2n + i) * S] (dey is
// offset to the pixel's column, S the column count), else to the pixel's workspace.
// rec_stride: doubles per pixel record.  raw = 0: a Gram record (rows 0..n-1 = C_diff,
// row n = m_diff).  raw = 1: a box-statistics record with inner moments (rows 0..n-1 the
// annulus moments R (j >= i), row n+1 m = m_inner - mu_ann, row n+2 mu_ann, rows n+3..2n+2
// the inner moments R_in (j >= i), all of f = x - ref): C_diff = (R_in - mu_in mu_in^T) -
// (R - mu_ann mu_ann^T) with mu_in = m + mu_ann, and m_diff = m.
template <int G>
__global__ __launch_bounds__(64) void tridiag_dwest_kernel(double *__restrict__ ws, int n, int npix,
                                                           double *__restrict__ dey, int64_t S,
                                                           int64_t rec_stride, int raw)
{
    extern __shared__ double sm[];
    const int lane = threadIdx.x, grp = lane / G, gl = lane - grp * G;
    const int per = tri(n) + 3 * n;
    double *A = sm + (size_t)grp * per;   // packed lower triangle, tri(n) doubles
    double *v = A + tri(n);               // n (Householder vector; entries <= k unused)
    double *q = v + n;                    // n
    double *y = q + n;                    // n
    const int want = blockIdx.x * (64 / G) + grp;
    const bool active = want < npix;
    const int local = active ? want : npix - 1;   // an idle group repeats a pixel, writes nothing
    double *pix = ws + (size_t)local * rec_stride;

    // load: unconditional reads (index clamped) four at a time, predicated LDS stores
    const int nn = n * n;
    if (!raw) {
        for (int t0 = 0; t0 < nn; t0 += 4 * G) {
            double val[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int t = t0 + G * u + gl;
                val[u] = pix[t < nn ? t : nn - 1];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int t = t0 + G * u + gl;
                const int i = t / n, j = t - i * n;
                if (t < nn && j <= i) A[tri(i) + j] = val[u];
            }
        }
        for (int i = gl; i < n; i += G) y[i] = pix[(size_t)n * n + i];
    } else {
        // v <- mu_ann, q <- mu_in, y <- m first; then the upper triangles of R and R_in
        for (int i = gl; i < n; i += G) {
            const double m = pix[(size_t)(n + 1) * n + i], mu = pix[(size_t)(n + 2) * n + i];
            v[i] = mu;
            q[i] = m + mu;
            y[i] = m;
        }
        __syncthreads();
        const double *rin = pix + (size_t)(n + 3) * n;
        for (int t0 = 0; t0 < nn; t0 += 2 * G) {
            double ra[2], ri[2];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int t = t0 + G * u + gl, tc = t < nn ? t : nn - 1;
                ra[u] = pix[tc];
                ri[u] = rin[tc];
            }
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int t = t0 + G * u + gl;
                const int r = t / n, c = t - r * n;   // stored at (r, c), c >= r: element (c, r)
                if (t < nn && c >= r)
                    A[tri(c) + r] = (ri[u] - q[r] * q[c]) - (ra[u] - v[r] * v[c]);
            }
        }
    }
    __syncthreads();

    for (int k = 0; k + 2 < n; ++k) {
        // column k below the diagonal: x = A[k+1.., k]
        double s2 = 0.0;
        for (int i = k + 1 + gl; i < n; i += G) s2 += A[tri(i) + k] * A[tri(i) + k];
        s2 = group_sum<G>(s2);
        const double x0 = A[tri(k + 1) + k];
        const bool refl = s2 - x0 * x0 != 0.0;   // else already reduced: e_k = x0
        const double alpha = x0 >= 0.0 ? -sqrt(s2) : sqrt(s2);
        const double beta = refl ? 1.0 / (alpha * (alpha - x0)) : 0.0;   // 2 / v^T v
        for (int i = k + 1 + gl; i < n; i += G) v[i] = !refl ? 0.0 : i == k + 1 ? x0 - alpha : A[tri(i) + k];
        __syncthreads();
        // p = beta A' v on the trailing block; K = (beta/2) v^T p; q = p - K v
        double vp = 0.0, vy = 0.0;
        for (int i = k + 1 + gl; i < n; i += G) {
            const int ti = tri(i);
            double p0 = 0.0, p1 = 0.0, p2 = 0.0, p3 = 0.0;   // four chains hide the FMA latency
            int j = k + 1;
            for (; j + 3 < n; j += 4) {
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int jj = j + u;
                    const double a = A[jj <= i ? ti + jj : tri(jj) + i];
                    if (u == 0) p0 = fma(a, v[jj], p0);
                    else if (u == 1) p1 = fma(a, v[jj], p1);
                    else if (u == 2) p2 = fma(a, v[jj], p2);
                    else p3 = fma(a, v[jj], p3);
                }
            }
            for (; j < n; ++j) p0 = fma(A[j <= i ? ti + j : tri(j) + i], v[j], p0);
            const double p = beta * ((p0 + p1) + (p2 + p3));
            q[i] = p;
            vp = fma(v[i], p, vp);
            vy = fma(v[i], y[i], vy);
        }
        vp = group_sum<G>(vp);
        vy = group_sum<G>(vy);
        const double K = 0.5 * beta * vp, gam = beta * vy;
        for (int i = k + 1 + gl; i < n; i += G) {
            q[i] = fma(-K, v[i], q[i]);
            y[i] = fma(-gam, v[i], y[i]);
        }
        __syncthreads();
        // A' <- A' - v q^T - q v^T on the lower triangle (j <= i).  tri(i) + j stays inside
        // the packed array for j < n; past the row's end it is read and left alone.
        for (int i = k + 1 + gl; i < n; i += G) {
            double *row = A + tri(i);
            const double vi = v[i], qi = q[i];
#pragma unroll 4
            for (int j = k + 1; j < n; ++j) {
                const double a = row[j] - fma(vi, q[j], qi * v[j]);
                if (j <= i) row[j] = a;
            }
        }
        // column k itself becomes alpha e_1 (only the subdiagonal is read later)
        if (gl == 0 && refl) A[tri(k + 1) + k] = alpha;
        __syncthreads();
    }
    // d, e, y -> the start of the pixel's workspace (the matrix is in LDS now), or to the
    // pixel's column of dey
    if (active) {
        for (int i = gl; i < n; i += G) {
            const double di = A[tri(i) + i], ei = i + 1 < n ? A[tri(i + 1) + i] : 0.0;
            if (dey) {
                double *c = dey + local;
                c[(int64_t)i * S] = di;
                c[(int64_t)(n + i) * S] = ei;
                c[(int64_t)(2 * n + i) * S] = y[i];
            } else {
                pix[i] = di;
                pix[n + i] = ei;
                pix[2 * n + i] = y[i];
            }
        }
    }
}

// The implicit QL iteration of one pixel on its columns d, e, y (entry i at i * st), and
// the outputs: ok (converged), s2 = sum_P y_i^2, s1 = sum_P |y_i|, cnt = |P|.
__device__ __forceinline__ void ql_pixel(double *__restrict__ d, double *__restrict__ e, double *__restrict__ y,
                                         int64_t st, int n, bool &ok, double &s2, double &s1, int &cnt)
{
#define D(i) d[(int64_t)(i) * st]
#define E(i) e[(int64_t)(i) * st]
#define Y(i) y[(int64_t)(i) * st]
    ok = true;
    E(n - 1) = 0.0;
    // deflation floor: eps times a bound of ||T|| (the iteration keeps the spectrum, so the
    // bound of the initial T holds throughout).  Near-zero eigenvalues, which a rank-deficient
    // C_diff has when a window holds fewer samples than bands, meet it; the pair test alone
    // would never call their subdiagonal negligible.
    double dnm = 0.0, enm = 0.0;
    for (int i = 0; i < n; ++i) {
        dnm = fmax(dnm, fabs(D(i)));
        enm = fmax(enm, fabs(E(i)));
    }
    const double tst = DBL_EPSILON * (dnm + enm);
    for (int l = 0; l < n && ok; ++l) {
        int iter = 0;
        for (;;) {
            // first m >= l with a negligible e_m (n - 1 if none): eight entries per step,
            // loaded (clamped) before any is tested
            int m = l;
            for (;;) {
                if (m + 1 >= n) {
                    m = n - 1;
                    break;
                }
                double ev[8], dv[9];
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const int t = m + k < n ? m + k : n - 1;
                    ev[k] = E(t);
                    dv[k] = D(t);
                }
                dv[8] = D(m + 8 < n ? m + 8 : n - 1);
                int hit = -1;
#pragma unroll
                for (int k = 7; k >= 0; --k)
                    if (m + k + 1 < n && fabs(ev[k]) <= fmax(DBL_EPSILON * (fabs(dv[k]) + fabs(dv[k + 1])), tst))
                        hit = k;
                if (hit >= 0) {
                    m += hit;
                    break;
                }
                m += 8;
            }
            if (m == l) break;
            if (++iter > 64) {
                ok = false;
                break;
            }
            // Wilkinson shift from the leading 2 x 2 block of the unreduced part
            double g = (D(l + 1) - D(l)) / (2.0 * E(l));
            double r = hypot(g, 1.0);
            g = D(m) - D(l) + E(l) / (g + (g >= 0.0 ? r : -r));
            double s = 1.0, c = 1.0, p = 0.0;
            bool underflow = false;
            // the sweep reads d_i, e_i, y_i once each (prefetched one rotation ahead) and
            // carries d_i+1 (still the value from before the sweep) and the rotated y_i+1
            double dcar = D(m), ycar = Y(m);
            double ei = E(m - 1), di = D(m - 1), yi = Y(m - 1);
            for (int i = m - 1; i >= l; --i) {
                // next operands: an unconditional load (index clamped at 0; unused after the
                // last rotation), so it is in flight during this rotation
                const int in = i > 0 ? i - 1 : 0;
                const double en = E(in), dn = D(in), yn = Y(in);
                const double f = s * ei, b = c * ei;
                // r = hypot(f, g) and 1/r from the hardware reciprocal square root refined by
                // two Newton steps (|f|, |g| stay far from the FP64 range limits here)
                const double r2 = fma(f, f, g * g);
                if (r2 == 0.0) {         // the chase split the matrix: restart at l
                    E(i + 1) = 0.0;
                    D(i + 1) = dcar - p;
                    Y(i + 1) = ycar;
                    E(m) = 0.0;
                    underflow = true;
                    break;
                }
                double ir = __builtin_amdgcn_rsq(r2);
                ir = fma(0.5 * ir, fma(-r2 * ir, ir, 1.0), ir);
                ir = fma(0.5 * ir, fma(-r2 * ir, ir, 1.0), ir);
                r = r2 * ir;
                E(i + 1) = r;
                s = f * ir;
                c = g * ir;
                g = dcar - p;
                r = (di - g) * s + 2.0 * c * b;
                p = s * r;
                D(i + 1) = g + p;
                g = c * r - b;
                Y(i + 1) = fma(s, yi, c * ycar);
                ycar = fma(c, yi, -s * ycar);
                dcar = di;
                ei = en;
                di = dn;
                yi = yn;
            }
            if (!underflow) Y(l) = ycar;
            if (underflow) continue;
            D(l) -= p;
            E(l) = g;
            E(m) = 0.0;
        }
    }
    double emax = 0.0;
    for (int i = 0; i < n; ++i) emax = fmax(emax, fabs(D(i)));
    s2 = 0.0;
    s1 = 0.0;
    cnt = 0;
    for (int i = 0; i < n; ++i) {
        const double pr = Y(i);     // loaded whatever the branch: no round trip inside it
        if (D(i) > 1e-12 * emax) {
            s2 += pr * pr;
            s1 += fabs(pr);
            ++cnt;
        }
    }
#undef D
#undef E
#undef Y
}

// lane = pixel; d, e, y of pixel lane in LDS columns (entry i at i * P + lane).
__global__ void ql_dwest_kernel(const double *__restrict__ ws, int n, int npix, int64_t pix0, int P,
                                float *__restrict__ score, float *__restrict__ literal,
                                int32_t *__restrict__ npos, int64_t rec_stride)
{
    extern __shared__ double sm[];
    const int lane = threadIdx.x;
    const int local = blockIdx.x * P + lane;
    double *d = sm, *e = sm + (size_t)n * P, *y = sm + (size_t)2 * n * P;
    const bool act = lane < P && local < npix;
    if (!act) return;      // no barriers below: lanes are independent
    const double *pix = ws + (size_t)local * rec_stride;
    for (int i = 0; i < n; ++i) {
        d[i * P + lane] = pix[i];
        e[i * P + lane] = pix[n + i];
        y[i * P + lane] = pix[2 * n + i];
    }
    bool ok;
    double s2, s1;
    int cnt;
    ql_pixel(d + lane, e + lane, y + lane, P, n, ok, s2, s1, cnt);
    const int64_t o = pix0 + local;
    score[o] = ok ? (float)sqrt(s2) : NAN;
    if (literal) literal[o] = ok ? (float)s1 : NAN;
    if (npos) npos[o] = ok ? cnt : -1;
}

// lane = pixel q of a run of S pixels; d, e, y of pixel q in global columns: dey[i * S + q],
// dey[(n + i) * S + q], dey[(2n + i) * S + q] (coalesced across a wavefront), updated in
// place.  No LDS, so a launch holds as many pixels as the registers allow.
__global__ __launch_bounds__(256) void ql_dwest_global_kernel(double *__restrict__ dey, int n, int64_t S,
                                                              int64_t pix0, float *__restrict__ score,
                                                              float *__restrict__ literal,
                                                              int32_t *__restrict__ npos)
{
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= S) return;
    double *d = dey + q, *e = dey + (int64_t)n * S + q, *y = dey + (int64_t)2 * n * S + q;
    bool ok;
    double s2, s1;
    int cnt;
    ql_pixel(d, e, y, S, n, ok, s2, s1, cnt);
    const int64_t o = pix0 + q;
    score[o] = ok ? (float)sqrt(s2) : NAN;
    if (literal) literal[o] = ok ? (float)s1 : NAN;
    if (npos) npos[o] = ok ? cnt : -1;
}

size_t eig_smem(int64_t n) { return (size_t)(n * (n + 1) / 2 + 3 * n) * sizeof(double); }

// pixels per workgroup of the QL kernel: the largest power of two <= 64 whose three LDS
// columns stay within 48 KiB
static int ql_pixels(int64_t n)
{
    int P = 64;
    while (P > 1 && (size_t)(3 * n * P) * sizeof(double) > 48 * 1024) P >>= 1;
    return P;
}

int ql_lds_pixels(int64_t n) { return ql_pixels(n); }

// lanes per pixel of the tridiagonalisation: the smallest group of 16, 32 or 64 lanes that
// holds one row per lane (0: chosen by L'; tests force a size through hsad_internal_dwest_lanes)
static int g_tridiag_lanes = 0;

int tridiag_dwest_launch(double *ws, int64_t n, int npix, double *dey, int64_t S, hipStream_t s, int raw)
{
    const int G = g_tridiag_lanes ? g_tridiag_lanes : n <= 16 ? 16 : n <= 32 ? 32 : 64;
    const size_t sh = eig_smem(n) * (size_t)(64 / G);
    const void *k = G == 16 ? (const void *)tridiag_dwest_kernel<16>
                    : G == 32 ? (const void *)tridiag_dwest_kernel<32> : (const void *)tridiag_dwest_kernel<64>;
    if (int rc = allow_lds(k, sh, "tridiag_dwest_kernel")) return rc;
    int64_t stride = raw ? (int64_t)((2 * n + 3) * n) : (int64_t)((n + 2) * n);
    int ni = (int)n;
    void *args[] = {(void *)&ws, &ni, &npix, (void *)&dey, &S, &stride, &raw};
    if (hipLaunchKernel(k, dim3((unsigned)((npix + 64 / G - 1) / (64 / G))), dim3(64), args, sh, s) != hipSuccess)
        return fail(HSAD_EHIP, "tridiag_dwest_kernel: launch failed");
    return check_launch("tridiag_dwest_kernel");
}

int ql_dwest_global_launch(double *dey, int64_t n, int64_t S, int64_t pix0, float *score, float *literal,
                           int32_t *npos, hipStream_t s)
{
    hipLaunchKernelGGL(ql_dwest_global_kernel, dim3((unsigned)((S + 255) / 256)), dim3(256), 0, s, dey, (int)n, S,
                       pix0, score, literal, npos);
    return check_launch("ql_dwest_global_kernel");
}

int eig_dwest_launch(double *ws, int64_t n, int npix, int64_t pix0, float *score, float *literal,
                     int32_t *npos, hipStream_t s, int raw)
{
    if (int rc = tridiag_dwest_launch(ws, n, npix, nullptr, 0, s, raw)) return rc;
    const int P = ql_pixels(n);
    const size_t sq = (size_t)(3 * n * P) * sizeof(double);
    const int64_t stride = raw ? (int64_t)((2 * n + 3) * n) : (int64_t)((n + 2) * n);
    hipLaunchKernelGGL(ql_dwest_kernel, dim3((unsigned)((npix + P - 1) / P)), dim3(P), sq, s,
                       (const double *)ws, (int)n, npix, pix0, P, score, literal, npos, stride);
    return check_launch("ql_dwest_kernel");
}

}  // namespace hsad

extern "C" int hsad_internal_dwest_lanes(int g)
{
    if (g != 0 && g != 16 && g != 32 && g != 64) return HSAD_EINVAL;
    hsad::g_tridiag_lanes = g;
    return 0;
}
