// dev_chol.hpp -- device body of the per-pixel loading + FP64 Cholesky + RX quadratic forms
// on the (L'+2) x L' trapezoid, shared by the per-chunk kernel and the persistent batch
// kernel.  See chol.hip for the method notes.
#pragma once
#include <hip/hip_runtime.h>

namespace hsad {

static constexpr int NB = 32;

__device__ __forceinline__ double block_sum(double v, double *red)
{
    // wave reduction then across waves through LDS (red holds >= 4 doubles)
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if (lane == 0) red[wv] = v;
    __syncthreads();
    double s = 0.0;
    for (int i = 0; i < nw; ++i) s += red[i];
    __syncthreads();
    return s;
}

// Factorises one pixel's trapezoid A ((L'+2) x L', FP64) in place and writes the two
// scores to *lrx_out / *dwrx_out (either may be NULL).  Whole workgroup; sm holds
// chol_smem_doubles(L') doubles.
__device__ inline void chol_pixel(double *__restrict__ A, int Lp, double load_rel,
                                  float *lrx_out, float *dwrx_out, double *sm)
{
    const int rows = Lp + 2;
    double *panel = sm;                        // rows x NB (row stride NB+1)
    double *red = sm + (size_t)rows * (NB + 1);
    double &bad = red[6];                      // 0/1 flag shared by the workgroup
    const int tid = threadIdx.x, nt = blockDim.x;

    // trace -> loading
    double tr = 0.0;
    for (int i = tid; i < Lp; i += nt) tr += A[(size_t)i * Lp + i];
    tr = block_sum(tr, red);
    double lam = load_rel * tr / (double)Lp;
    lam = lam < 1e-30 ? 1e-30 : lam;
    if (tid == 0) bad = 0.0;
    for (int i = tid; i < Lp; i += nt) A[(size_t)i * Lp + i] += lam;
    __syncthreads();

    for (int kb = 0; kb < Lp; kb += NB) {
        const int nb = Lp - kb < NB ? Lp - kb : NB;
        const int prow = rows - kb;            // panel rows kb..rows-1
        // load panel columns kb..kb+nb-1 of rows kb..rows-1
        for (int t = tid; t < prow * nb; t += nt) {
            const int r = t / nb, c = t - r * nb;
            panel[(size_t)r * (NB + 1) + c] = A[(size_t)(kb + r) * Lp + kb + c];
        }
        __syncthreads();
        // unblocked factorisation of the panel
        for (int j = 0; j < nb; ++j) {
            const double d = panel[(size_t)j * (NB + 1) + j];
            if (!(d > 0.0) && tid == 0) bad = 1.0;
            const double inv = 1.0 / sqrt(d);
            __syncthreads();
            for (int r = j + tid; r < prow; r += nt) panel[(size_t)r * (NB + 1) + j] *= inv;
            __syncthreads();
            // rank-1 update of panel columns j+1..nb-1, rows >= column
            const int ncol = nb - j - 1;
            if (ncol > 0) {
                const int nrow = prow - j - 1;
                for (int t = tid; t < nrow * ncol; t += nt) {
                    const int r = j + 1 + t / ncol, c = j + 1 + t % ncol;
                    if (c <= r) panel[(size_t)r * (NB + 1) + c] -=
                        panel[(size_t)r * (NB + 1) + j] * panel[(size_t)c * (NB + 1) + j];
                }
            }
            __syncthreads();
        }
        // write the factored panel back (only the part the later panels / scores read)
        for (int t = tid; t < prow * nb; t += nt) {
            const int r = t / nb, c = t - r * nb;
            if (c <= r) A[(size_t)(kb + r) * Lp + kb + c] = panel[(size_t)r * (NB + 1) + c];
        }
        // trailing update: rows i >= k0, columns k in [k0, Lp), k <= i, where k0 = kb+nb
        const int k0 = kb + nb;
        if (k0 < Lp) {
            const int nr = rows - k0, ncl = Lp - k0;
            const int br = (nr + 3) / 4, bc = (ncl + 3) / 4;
            for (int t = tid; t < br * bc; t += nt) {
                const int bi = t / bc, bk = t - bi * bc;
                const int i0 = 4 * bi, c0 = 4 * bk;   // relative to k0
                if (c0 > i0 + 3) continue;            // block strictly above the diagonal
                double acc[4][4];
#pragma unroll
                for (int u = 0; u < 4; ++u)
#pragma unroll
                    for (int v = 0; v < 4; ++v) acc[u][v] = 0.0;
                for (int j = 0; j < nb; ++j) {
                    double li[4], lk[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int ri = i0 + u, rk = c0 + u;
                        li[u] = ri < nr ? panel[(size_t)(nb + ri) * (NB + 1) + j] : 0.0;
                        lk[u] = rk < ncl ? panel[(size_t)(nb + rk) * (NB + 1) + j] : 0.0;
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u)
#pragma unroll
                        for (int v = 0; v < 4; ++v) acc[u][v] = fma(li[u], lk[v], acc[u][v]);
                }
#pragma unroll
                for (int u = 0; u < 4; ++u)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int ri = i0 + u, ck = c0 + v;
                        if (ri < nr && ck < ncl && ck <= ri)
                            A[(size_t)(k0 + ri) * Lp + k0 + ck] -= acc[u][v];
                    }
            }
        }
        __syncthreads();
    }
    // scores: squared norms of the two extra rows
    double s1 = 0.0, s2 = 0.0;
    for (int k = tid; k < Lp; k += nt) {
        const double a = A[(size_t)Lp * Lp + k], b = A[(size_t)(Lp + 1) * Lp + k];
        s1 += a * a;
        s2 += b * b;
    }
    s1 = block_sum(s1, red);
    s2 = block_sum(s2, red);
    if (tid == 0) {
        if (lrx_out) *lrx_out = bad != 0.0 ? INFINITY : (float)s1;
        if (dwrx_out) *dwrx_out = bad != 0.0 ? INFINITY : (float)s2;
    }
    __syncthreads();
}


__host__ __device__ inline size_t chol_smem_doubles(int Lp) { return (size_t)(Lp + 2) * (NB + 1) + 8; }

}  // namespace hsad
