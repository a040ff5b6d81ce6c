// jacobi.hip -- DWEST projection (Sec. 2.2, eqs. 2-4) with an FP64 parallel cyclic Jacobi
// eigensolver, one wavefront per pixel.
//
// Input per pixel (chunk workspace, written by the Gram kernel in DWEST mode):
// rows 0..L'-1 = C_diff = C_inner - C_outer, row L' = m_diff = m_inner - m_outer.
// The symmetric eigenproblem of C_diff is solved by Jacobi rotations in round-robin
// ("chess tournament") order.  Each round rotates m/2 disjoint index pairs at once
// (m = L' rounded up to even; an odd L' gets a dummy index).  A sweep of m-1 rounds
// touches every pair once.  Sweeps stop when the off-diagonal Frobenius norm is at most
// 1e-14 ||C_diff||_F.  The rotation annihilating A_pq is the symmetric Schur rotation
// (Golub & Van Loan, Alg. 8.4.1): theta = (A_qq - A_pp)/(2 A_pq),
// t = sign(theta)/(|theta| + sqrt(1 + theta^2)), c = 1/sqrt(1+t^2), s = t c.
// Eigenvalues above 1e-12 max|lambda| are "positive".  Outputs:
//   score   = ||V_P^T m_diff||_2        (independent of eigenvector signs)
//   literal = sum_P |v_i^T m_diff|      (eq. 4 with v_i signed so that v_i^T m_diff >= 0)
//   npos    = |P|
// Only the projections y = V^T m_diff are needed, never V itself: every rotation J applied
// to A as J^T A J is applied to y as J^T y, which keeps y = V^T m_diff throughout.  A, y and
// the round's pairs and rotations live in LDS (A with stride n+1 doubles); lanes split the
// (pair, index) updates of each round.
#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace hsad {

__device__ __forceinline__ double wave_sum(double v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__device__ __forceinline__ void tournament_pair(int i, int r, int m, int &p, int &q)
{
    // player 0 fixed, players 1..m-1 rotate by r positions
    auto at = [&](int j) { return 1 + (j + r) % (m - 1); };
    if (i == 0) {
        p = 0;
        q = at(0);
    } else {
        p = at(i);
        q = at(m - 1 - i);
    }
}

// floor(t / d) from mg = ceil(2^32 / d) (d >= 2; mg = 0 stands for d = 1).  Exact while
// t * (mg d - 2^32) < 2^32; with t < d^2 and an excess below d that holds for d <= 1625.
__device__ __forceinline__ unsigned div_magic(unsigned t, unsigned mg) { return mg ? __umulhi(t, mg) : t; }

__global__ __launch_bounds__(64) void jacobi_dwest_kernel(const double *__restrict__ ws, int n,
                                                          int npix, int64_t pix0, unsigned mg,
                                                          float *__restrict__ score,
                                                          float *__restrict__ literal,
                                                          int32_t *__restrict__ npos)
{
    extern __shared__ double sm[];
    const int ld = n + 1;
    const int m = n + (n & 1);
    const int np = m / 2;
    double *A = sm;                            // n x ld
    double *cs = A + (size_t)n * ld;           // np x 2 (c, s)
    double *y = cs + 2 * np;                   // n: V^T m_diff
    int *pq = reinterpret_cast<int *>(y + n);  // np x 2 (p, q); q >= n marks the dummy pair
    const int lane = threadIdx.x;
    const int local = blockIdx.x;
    if (local >= npix) return;
    const double *src = ws + (size_t)local * (n + 2) * n;

    double fro2 = 0.0;
    for (int t = lane; t < n * n; t += 64) {
        const unsigned i = div_magic((unsigned)t, mg), j = (unsigned)t - i * (unsigned)n;
        const double v = src[t];
        A[i * ld + j] = v;
        fro2 += v * v;
    }
    for (int k = lane; k < n; k += 64) y[k] = src[(size_t)n * n + k];
    fro2 = wave_sum(fro2);
    const double tol2 = 1e-28 * fro2;          // (1e-14 ||A||_F)^2
    __syncthreads();
    const int nu = np * n;

    for (int sweep = 0; sweep < 60; ++sweep) {
        double off2 = 0.0;
        for (int t = lane; t < n * n; t += 64) {
            const unsigned i = div_magic((unsigned)t, mg), j = (unsigned)t - i * (unsigned)n;
            if (i != j) off2 += A[i * ld + j] * A[i * ld + j];
        }
        off2 = wave_sum(off2);
        if (off2 <= tol2) break;
        for (int r = 0; r < m - 1; ++r) {
            // pairs and rotation parameters, one lane per pair; the projection vector is
            // rotated here too (the pairs of a round are disjoint)
            for (int i = lane; i < np; i += 64) {
                int p, q;
                tournament_pair(i, r, m, p, q);
                double c = 1.0, s = 0.0;
                if (q < n && p < n) {
                    const double apq = A[p * ld + q];
                    if (apq != 0.0) {
                        const double theta = (A[q * ld + q] - A[p * ld + p]) / (2.0 * apq);
                        const double t = (theta >= 0.0 ? 1.0 : -1.0) /
                                         (fabs(theta) + sqrt(theta * theta + 1.0));
                        c = 1.0 / sqrt(t * t + 1.0);
                        s = t * c;
                    }
                    const double yp = y[p], yq = y[q];
                    y[p] = c * yp - s * yq;
                    y[q] = s * yp + c * yq;
                } else {
                    p = p < q ? p : q;
                    q = n;                     // dummy index of an odd n
                }
                cs[2 * i] = c;
                cs[2 * i + 1] = s;
                pq[2 * i] = p;
                pq[2 * i + 1] = q;
            }
            __syncthreads();
            // A <- J^T A (rows p, q)
            for (int t = lane; t < nu; t += 64) {
                const unsigned i = div_magic((unsigned)t, mg), k = (unsigned)t - i * (unsigned)n;
                const int p = pq[2 * i], q = pq[2 * i + 1];
                if (q >= n) continue;
                const double c = cs[2 * i], s = cs[2 * i + 1];
                const double apk = A[p * ld + k], aqk = A[q * ld + k];
                A[p * ld + k] = c * apk - s * aqk;
                A[q * ld + k] = s * apk + c * aqk;
            }
            __syncthreads();
            // A <- A J (columns p, q)
            for (int t = lane; t < nu; t += 64) {
                const unsigned i = div_magic((unsigned)t, mg), k = (unsigned)t - i * (unsigned)n;
                const int p = pq[2 * i], q = pq[2 * i + 1];
                if (q >= n) continue;
                const double c = cs[2 * i], s = cs[2 * i + 1];
                const double akp = A[k * ld + p], akq = A[k * ld + q];
                A[k * ld + p] = c * akp - s * akq;
                A[k * ld + q] = s * akp + c * akq;
            }
            __syncthreads();
        }
    }
    // classification and projection
    double emax = 0.0;
    for (int i = lane; i < n; i += 64) emax = fmax(emax, fabs(A[i * ld + i]));
    for (int o = 32; o > 0; o >>= 1) emax = fmax(emax, __shfl_xor(emax, o));
    double s2 = 0.0, s1 = 0.0, cnt = 0.0;
    for (int i = lane; i < n; i += 64) {
        if (A[i * ld + i] > 1e-12 * emax) {
            const double pr = y[i];
            s2 += pr * pr;
            s1 += fabs(pr);
            cnt += 1.0;
        }
    }
    s2 = wave_sum(s2);
    s1 = wave_sum(s1);
    cnt = wave_sum(cnt);
    if (lane == 0) {
        const int64_t p = pix0 + local;
        score[p] = (float)sqrt(s2);
        if (literal) literal[p] = (float)s1;
        if (npos) npos[p] = (int32_t)cnt;
    }
}

size_t jacobi_smem(int64_t n)
{
    const int64_t np = (n + 1) / 2;
    return (size_t)(n * (n + 1) + 2 * np + n + np) * sizeof(double);
}

int jacobi_launch(const double *ws, int64_t n, int npix, int64_t pix0, float *score,
                  float *literal, int32_t *npos, hipStream_t s)
{
    if (n < 1 || n > 1024) return fail(HSAD_EUNSUPPORTED, "jacobi_dwest: L' must be in [1, 1024]");
    const size_t sh = jacobi_smem(n);
    if (int rc = allow_lds((const void *)jacobi_dwest_kernel, sh, "jacobi_dwest_kernel")) return rc;
    const unsigned mg = n == 1 ? 0u : (unsigned)((0x100000000ull + (uint64_t)n - 1) / (uint64_t)n);
    hipLaunchKernelGGL(jacobi_dwest_kernel, dim3((unsigned)npix), dim3(64), sh, s, ws, (int)n, npix,
                       pix0, mg, score, literal, npos);
    return check_launch("jacobi_dwest_kernel");
}

}  // namespace hsad
