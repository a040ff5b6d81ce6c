// dev_chol.hpp -- device body of the per-pixel loading + FP64 Cholesky + RX quadratic forms
// on the (L'+2) x L' trapezoid, shared by the per-chunk kernel and the persistent batch
// kernel.  See chol.hip for the method notes.
#pragma once
#include <hip/hip_runtime.h>

namespace hsad {

static constexpr int NB = 32;
// smallest L' that takes the blocked factorisation by default (chol_pixel_blk below)
static constexpr int kCholBlkMinLp = 129;

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
// raw != 0: A is a box-statistics record (dev_boxg.hpp): the upper triangle holds the
// second moments R and row L'+2 the mean mu_f; the covariance C = R - mu_f mu_f^T is
// formed in the lower triangle first.
__device__ inline void chol_pixel(double *__restrict__ A, int Lp, double load_rel,
                                  float *lrx_out, float *dwrx_out, double *sm, int raw = 0)
{
    const int rows = Lp + 2;
    double *panel = sm;                        // rows x NB (row stride NB+1)
    double *red = sm + (size_t)rows * (NB + 1);
    double &bad = red[6];                      // 0/1 flag shared by the workgroup
    double *pinv = red + 8;                    // NB reciprocal pivots of the current panel
    const int tid = threadIdx.x, nt = blockDim.x;
    if (raw) {
        const double *mu = A + (size_t)(Lp + 2) * Lp;
        for (int t = tid; t < Lp * Lp; t += nt) {
            const int i = t / Lp, j = t - i * Lp;
            if (j >= i) A[(size_t)j * Lp + i] = A[(size_t)i * Lp + j] - mu[i] * mu[j];
        }
        __syncthreads();
    }

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
        // unblocked factorisation of the panel, one barrier per column: column j is left
        // unscaled during its step and the rank-1 update takes a_rj a_cj / d_j; the panel's
        // columns are scaled by 1/sqrt(d_j) in one pass at the end.  Thread (tid & 31, tid >> 5)
        // updates column j+1+(tid & 31), rows j+1+(tid >> 5) + k (nt / 32).
        const int cl = tid & 31, rg = tid >> 5, nrg = nt >> 5;
        for (int j = 0; j < nb; ++j) {
            const double d = panel[(size_t)j * (NB + 1) + j];
            if (!(d > 0.0) && tid == 0) bad = 1.0;
            const int c = j + 1 + cl;
            if (c < nb) {
                const double acj = panel[(size_t)c * (NB + 1) + j] / d;
                for (int r = j + 1 + rg; r < prow; r += nrg)
                    if (c <= r) panel[(size_t)r * (NB + 1) + c] -= panel[(size_t)r * (NB + 1) + j] * acj;
            }
            __syncthreads();
        }
        if (tid < nb) pinv[tid] = 1.0 / sqrt(panel[(size_t)tid * (NB + 1) + tid]);
        __syncthreads();
        if (cl < nb)
            for (int r = cl + rg; r < prow; r += nrg) panel[(size_t)r * (NB + 1) + cl] *= pinv[cl];
        __syncthreads();
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

__host__ __device__ inline size_t chol_smem_doubles(int Lp) { return (size_t)(Lp + 2) * (NB + 1) + 8 + NB; }
__host__ __device__ inline size_t chol_blk_smem_doubles(int Lp)
{
    return (size_t)(Lp + 2) * (NB + 2) + 8 + NB + 2 * (size_t)NB * (NB + 2);
}

}  // namespace hsad

namespace hsad {

// ------------------------------------------------------------------------------------
// One wavefront per pixel, L' <= 64: the record is copied once into LDS with coalesced
// loads, then (raw records) C = R - mu mu^T, the loading, the unblocked right-looking
// Cholesky of the (L'+2) x L' trapezoid and the two squared norms run there, with wave
// barriers only.  Same definitions and operation order per column as chol_pixel's single
// panel.  lds holds chol_wave_lds_doubles(L') doubles for this wavefront.
// ------------------------------------------------------------------------------------
__host__ __device__ inline int chol_wave_lda(int Lp) { return Lp | 1; }
__host__ __device__ inline size_t chol_wave_lds_doubles(int Lp)
{
    return (size_t)(Lp + 2) * chol_wave_lda(Lp) + (size_t)Lp;
}

__device__ __forceinline__ void wave_sync_lds()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

typedef double f64x4 __attribute__((ext_vector_type(4)));

// value of v in lane l (l wave-uniform), as an FP64 scalar
__device__ __forceinline__ double lane_read_d(double v, int l)
{
    const unsigned long long b = __double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, l);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Blocked variant of chol_pixel for L' > 64 (same arguments, definitions and outputs;
// sm holds chol_blk_smem_doubles(L') doubles).  Panels of NB columns.  One wavefront
// factors a panel's NB x NB diagonal block and inverts its triangle in registers.  The rows
// below are solved as one product with that inverse, and the trailing lower trapezoid takes
// the rank-NB update in place; both products run on the FP64 matrix cores in 16 x 16 tiles
// (coalesced rows of 16 doubles).  Look-ahead: during panel p's trailing update one
// wavefront updates the first tiles, which hold panel p+1's diagonal block, and factors
// that block at once, while the other wavefronts update the rest.  The two extra rows are
// ordinary rows of this elimination; their squared norms are summed panel by panel from
// LDS.
__device__ inline void chol_pixel_blk(double *__restrict__ A, int Lp, double load_rel,
                                      float *lrx_out, float *dwrx_out, double *sm, int raw = 0)
{
    // row stride NB + 2: a matrix-core operand read (16 rows x 2 columns per half
    // wavefront) then touches 64 distinct LDS banks
    constexpr int LD = NB + 2;
    const int rows = Lp + 2;
    double *P = sm;                            // panel: rows x NB (row stride LD)
    double *red = sm + (size_t)rows * LD;
    double &bad = red[6];
    double *Wm = red + 8 + NB;                 // inverse of the diagonal block, NB x NB (stride LD)
    double *D = Wm + NB * LD;                  // next diagonal block before its factorisation
    const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63, wv = tid >> 6, nw = nt >> 6;
    const int c16 = lane & 15, g4 = lane >> 4;
    if (raw) {
        const double *mu = A + (size_t)(Lp + 2) * Lp;
        for (int t = tid; t < Lp * Lp; t += nt) {
            const int i = t / Lp, j = t - i * Lp;
            if (j >= i) A[(size_t)j * Lp + i] = A[(size_t)i * Lp + j] - mu[i] * mu[j];
        }
        __syncthreads();
    }
    double tr = 0.0;
    for (int i = tid; i < Lp; i += nt) tr += A[(size_t)i * Lp + i];
    tr = block_sum(tr, red);
    double lam = load_rel * tr / (double)Lp;
    lam = lam < 1e-30 ? 1e-30 : lam;
    if (tid == 0) bad = 0.0;
    for (int i = tid; i < Lp; i += nt) A[(size_t)i * Lp + i] += lam;
    __syncthreads();

    // Cholesky factor L of the nbd x nbd block in src (row stride LD) and W = L^-1, by one
    // wavefront, lane i (mod 32) holding row i of the block and row i of W (identity to
    // start) in registers.  Step j: l_jj = sqrt(a_jj), l_ij = a_ij / l_jj; row j of W is
    // final once divided by l_jj; rows i > j then take a_ic -= l_ij l_cj (c > j) and
    // W_ic -= l_ij W_jc (c <= j).  Every broadcast is a lane read of a compile-time
    // register, so the step has no LDS round trip.  L goes to P's first rows, W to Wm (zero
    // outside the nbd x nbd lower triangle).
    auto factor_diag = [&](const double *src, int nbd) {
        const int i = lane & 31;
        double a[NB], w[NB];
#pragma unroll
        for (int c = 0; c < NB; ++c) {
            a[c] = src[i * LD + c];
            w[c] = c == i ? 1.0 : 0.0;
        }
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            if (j < nbd) {
                const double d = lane_read_d(a[j], j);
                const double sq = sqrt(d), iv = 1.0 / sq;
                if (lane == 0 && !(d > 0.0)) bad = 1.0;
                const double lij = i == j ? sq : a[j] * iv;
                a[j] = lij;
                const double ws = i == j ? iv : 1.0, lw = i > j ? lij : 0.0;
#pragma unroll
                for (int c = 0; c <= j; ++c) w[c] *= ws;
                // rows i <= j only change entries above their diagonal, which are not used
#pragma unroll
                for (int c = j + 1; c < NB; ++c) {
                    a[c] = fma(-lij, lane_read_d(a[j], c), a[c]);
                    // few lane reads in flight: each holds two scalar registers
                    if ((c & 7) == 7) __builtin_amdgcn_sched_barrier(0);
                }
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int c = 0; c <= j; ++c) {
                    w[c] = fma(-lw, lane_read_d(w[c], j), w[c]);
                    if ((c & 7) == 7) __builtin_amdgcn_sched_barrier(0);
                }
                __builtin_amdgcn_sched_barrier(0);
            }
        }
        if (lane < 32) {
#pragma unroll
            for (int c = 0; c < NB; ++c) {
                const bool in = i < nbd && c <= i;
                if (in) P[i * LD + c] = a[c];
                Wm[i * LD + c] = in ? w[c] : 0.0;
            }
        }
    };

    // panel 0: the whole panel, then its diagonal block
    {
        const int nb = Lp < NB ? Lp : NB;
        for (int t = tid; t < rows * nb; t += nt) {
            const int r = t / nb, c = t - r * nb;
            P[(size_t)r * LD + c] = A[(size_t)r * Lp + c];
        }
        __syncthreads();
        if (wv == 0) factor_diag(P, nb);
        __syncthreads();
    }

    double s1 = 0.0, s2 = 0.0;   // partial squared norms of the extra rows (threads < NB)
    for (int kb = 0; kb < Lp; kb += NB) {
        const int nb = Lp - kb < NB ? Lp - kb : NB;
        const int prow = rows - kb;
        if (kb > 0) {
            // the rows below the diagonal block (factored during the previous trailing update)
            for (int t = tid; t < (prow - nb) * nb; t += nt) {
                const int r = nb + t / nb, c = t - (r - nb) * nb;
                P[(size_t)r * LD + c] = A[(size_t)(kb + r) * Lp + kb + c];
            }
            __syncthreads();
        }
        // rows below the block: X = A_below L_kk^-T = A_below W^T with W = L_kk^-1,
        // 16 rows x 32 columns per wavefront on the matrix cores.
        // Columns >= nb (last panel) are zero on both operands and never stored.
        {
            const int nrb = (prow - nb + 15) >> 4;
            const int nk = (nb + 3) >> 2;
            for (int rb = wv; rb < nrb; rb += nw) {
                f64x4 x0 = {0.0, 0.0, 0.0, 0.0}, x1 = {0.0, 0.0, 0.0, 0.0};
                const int ra = nb + 16 * rb + c16;
                for (int kk = 0; kk < nk; ++kk) {
                    const int col = 4 * kk + g4;
                    const double av = ra < prow && col < nb ? P[(size_t)ra * LD + col] : 0.0;
                    x0 = __builtin_amdgcn_mfma_f64_16x16x4f64(av, Wm[c16 * LD + col], x0, 0, 0, 0);
                    x1 = __builtin_amdgcn_mfma_f64_16x16x4f64(av, Wm[(16 + c16) * LD + col], x1, 0, 0, 0);
                }
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int r = nb + 16 * rb + 4 * e + g4;
                    if (r < prow) {
                        if (c16 < nb) P[(size_t)r * LD + c16] = x0[e];
                        if (16 + c16 < nb) P[(size_t)r * LD + 16 + c16] = x1[e];
                    }
                }
            }
        }
        __syncthreads();
        if (tid < nb) {
            const double u = P[(size_t)(prow - 2) * LD + tid], v = P[(size_t)(prow - 1) * LD + tid];
            s1 += u * u;
            s2 += v * v;
        }
        // trailing update A[i][k] -= sum_j L[i][j] L[k][j], k0 <= k <= i, on 16 x 16 tiles
        const int k0 = kb + nb;
        if (k0 < Lp) {
            const int nr = rows - k0, ncl = Lp - k0;
            const int TI = (nr + 15) >> 4, TJ = (ncl + 15) >> 4;
            const int ntri = TJ * (TJ + 1) / 2, ntile = ntri + (TI - TJ) * TJ;
            const int nk = (nb + 3) >> 2;
            const int nb1 = Lp - k0 < NB ? Lp - k0 : NB;   // the next panel's width
            // the next diagonal block lies in the first ns tiles: (0,0), then (1,0), (1,1)
            const int ns = nb1 > 16 ? 3 : 1;
            const int la = (kb / NB + 1) % nw;             // rotates over the SIMDs
            // tile t -> (I, J): row-major over the triangle J <= I < TJ, then full rows of TJ
            auto tile_of = [&](int t, int &I, int &J) {
                if (t < ntri) {
                    I = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
                    while ((I + 1) * (I + 2) / 2 <= t) ++I;
                    while (I * (I + 1) / 2 > t) --I;
                    J = t - I * (I + 1) / 2;
                } else {
                    const int u = t - ntri;
                    I = TJ + u / TJ;
                    J = u - (I - TJ) * TJ;
                }
            };
            // products of the tiles in tij[] (16 I | 16 J << 16) with this panel's L
            auto tile_products = [&](f64x4 *acc, const int *tij, int ntb) {
                for (int kk = 0; kk < nk; ++kk) {
                    const int col = 4 * kk + g4;
                    for (int q = 0; q < ntb; ++q) {
                        const int ra = nb + (tij[q] & 0xffff) + c16, rb = nb + (tij[q] >> 16) + c16;
                        const double av = ra < prow && col < nb ? -P[(size_t)ra * LD + col] : 0.0;
                        const double bv = rb < prow && col < nb ? P[(size_t)rb * LD + col] : 0.0;
                        acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[q], 0, 0, 0);
                    }
                }
            };
            if (wv == la) {
                // the next diagonal block: its tiles updated (written back too, for the rows
                // of a partial last block that lie below it) and kept in D, then factored
                f64x4 acc[3];
                int tij[3];
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    int I, J;
                    tile_of(q < ns ? q : 0, I, J);
                    tij[q] = 16 * I | (16 * J) << 16;
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int r = k0 + 16 * I + 4 * e + g4, c = k0 + 16 * J + c16;
                        acc[q][e] = r < rows && c < Lp ? A[(size_t)r * Lp + c] : 0.0;
                    }
                }
                tile_products(acc, tij, ns);
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    if (q < ns) {
                        const int I16 = tij[q] & 0xffff, J16 = tij[q] >> 16;
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            // FP64 16x16x4: element e of lane l is row 4e + (l >> 4), column l & 15
                            const int r = k0 + I16 + 4 * e + g4, c = k0 + J16 + c16;
                            if (r < rows && c < Lp && c <= r) A[(size_t)r * Lp + c] = acc[q][e];
                            D[(I16 + 4 * e + g4) * LD + J16 + c16] = acc[q][e];
                        }
                    }
                }
                if (ns == 3) {
#pragma unroll
                    for (int e = 0; e < 4; ++e) D[(4 * e + g4) * LD + 16 + c16] = 0.0;   // above the diagonal
                }
                wave_sync_lds();
                factor_diag(D, nb1);
            } else {
                // the remaining tiles over the other wavefronts, TB per step, the next step's
                // tiles loaded before this step's products are issued
                constexpr int TB = 2;
                const int wi = wv < la ? wv : wv - 1, nwr = nw - 1;
                auto load_tiles = [&](int t0, f64x4 *acc, int *tij) {
#pragma unroll
                    for (int q = 0; q < TB; ++q) {
                        int I, J;
                        tile_of(t0 + q < ntile ? t0 + q : ntile - 1, I, J);
                        tij[q] = 16 * I | (16 * J) << 16;
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            const int r = k0 + 16 * I + 4 * e + g4, c = k0 + 16 * J + c16;
                            acc[q][e] = r < rows && c < Lp ? A[(size_t)r * Lp + c] : 0.0;
                        }
                    }
                };
                f64x4 acc[TB], nacc[TB];
                int tij[TB], nij[TB];
                const int first = ns + TB * wi;
                if (first < ntile) load_tiles(first, acc, tij);
                for (int t0 = first; t0 < ntile; t0 += TB * nwr) {
                    const int t1 = t0 + TB * nwr;
                    if (t1 < ntile) load_tiles(t1, nacc, nij);
                    tile_products(acc, tij, TB);
#pragma unroll
                    for (int q = 0; q < TB; ++q) {
                        if (t0 + q < ntile) {
#pragma unroll
                            for (int e = 0; e < 4; ++e) {
                                const int r = k0 + (tij[q] & 0xffff) + 4 * e + g4, c = k0 + (tij[q] >> 16) + c16;
                                if (r < rows && c < Lp && c <= r) A[(size_t)r * Lp + c] = acc[q][e];
                            }
                        }
                        acc[q] = nacc[q];
                        tij[q] = nij[q];
                    }
                }
            }
        }
        __syncthreads();
    }
    s1 = block_sum(s1, red);
    s2 = block_sum(s2, red);
    if (tid == 0) {
        if (lrx_out) *lrx_out = bad != 0.0 ? INFINITY : (float)s1;
        if (dwrx_out) *dwrx_out = bad != 0.0 ? INFINITY : (float)s2;
    }
    __syncthreads();
}

__device__ __forceinline__ double wave_sum_d(double v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ inline void chol_wave_pixel(const double *__restrict__ rec, int Lp, int raw, double load_rel,
                                       float *lrx_out, float *dwrx_out, double *A)
{
    const int lane = threadIdx.x & 63;
    const int lda = chol_wave_lda(Lp), rows = Lp + 2;
    double *mu = A + (size_t)rows * lda;
    for (int t = lane; t < rows * Lp; t += 64) {
        const int r = t / Lp, c = t - r * Lp;
        A[r * lda + c] = rec[t];
    }
    if (raw)
        for (int c = lane; c < Lp; c += 64) mu[c] = rec[(size_t)rows * Lp + c];
    wave_sync_lds();
    if (raw) {
        for (int t = lane; t < Lp * Lp; t += 64) {
            const int i = t / Lp, j = t - i * Lp;
            if (j >= i) A[j * lda + i] = A[i * lda + j] - mu[i] * mu[j];
        }
        wave_sync_lds();
    }
    double tr = 0.0;
    for (int i = lane; i < Lp; i += 64) tr += A[i * lda + i];
    tr = wave_sum_d(tr);
    double lam = load_rel * tr / (double)Lp;
    lam = lam < 1e-30 ? 1e-30 : lam;
    for (int i = lane; i < Lp; i += 64) A[i * lda + i] += lam;
    wave_sync_lds();
    bool bad = false;
    for (int j = 0; j < Lp; ++j) {
        const double d = A[j * lda + j];
        bad = bad || !(d > 0.0);
        const double inv = 1.0 / sqrt(d);
        wave_sync_lds();
        for (int r = j + lane; r < rows; r += 64) A[r * lda + j] *= inv;
        wave_sync_lds();
        const int ncol = Lp - j - 1, nrow = rows - j - 1;
        if (ncol > 0) {
            // t / ncol by a multiply-high; ceil(2^32 / ncol) fits 32 bits only for ncol >= 2
            const uint32_t magic =
                ncol > 1 ? (uint32_t)((((uint64_t)1 << 32) + (uint64_t)ncol - 1) / (uint64_t)ncol) : 0u;
            for (int t = lane; t < nrow * ncol; t += 64) {
                const int q = ncol > 1 ? (int)__umulhi((uint32_t)t, magic) : t;
                const int r = j + 1 + q, c = j + 1 + (t - q * ncol);
                if (c <= r) A[r * lda + c] -= A[r * lda + j] * A[c * lda + j];
            }
        }
        wave_sync_lds();
    }
    double s1 = 0.0, s2 = 0.0;
    for (int k = lane; k < Lp; k += 64) {
        const double a = A[Lp * lda + k], b = A[(Lp + 1) * lda + k];
        s1 += a * a;
        s2 += b * b;
    }
    s1 = wave_sum_d(s1);
    s2 = wave_sum_d(s2);
    if (lane == 0) {
        if (lrx_out) *lrx_out = bad ? INFINITY : (float)s1;
        if (dwrx_out) *dwrx_out = bad ? INFINITY : (float)s2;
    }
}

}  // namespace hsad

namespace hsad {

// ------------------------------------------------------------------------------------
// Register-resident Cholesky: a group of G lanes (G = 16, 32 or 64; 64/G pixels per
// wavefront) owns one pixel, lane r of the group holds row r of the (L'+2) x L' trapezoid
// (its lower part) in registers, L' + 2 <= G.  Column j: the pivot comes from lane j,
// each lane scales its element j and publishes it in the group's LDS column buffer, and
// the rank-1 update of column c reads l_cj there (a broadcast read).  Same operations in
// the same order per column as the unblocked factorisation of chol_pixel (loading added
// before factorising).  All indices into the register row are compile-time constants
// (loops over the G - 2 register columns are unrolled; the column loop itself is not, and
// columns past L' are skipped by uniform branches).  rec is the record of the pixel ((L'+2) x L' for Gram records, (L'+3) x L'
// for raw box-statistics records); col is this lane's group's G-double LDS buffer.
// ------------------------------------------------------------------------------------
template <int G, int CB = 16>
__device__ inline void chol_group_pixel(const double *__restrict__ rec, int Lp, int raw, double load_rel,
                                        bool active, float *lrx_out, float *dwrx_out, double *col)
{
    constexpr int CM = G - 2;                  // largest L' of this group size
    const int lane = threadIdx.x & 63, r = lane & (G - 1), base = lane & ~(G - 1);
    const bool row_in = active && r < Lp + 2;
    // Touch every 128-byte line of the record first with independent loads (one round trip
    // to memory for the whole record); the row loads below, which run one after another,
    // then hit the cache.
    if constexpr (G >= 32) {
        const int nl = (int)(((size_t)(raw ? Lp + 3 : Lp + 2) * Lp * sizeof(double) + 127) / 128);
#pragma unroll
        for (int k = 0; k < (G == 64 ? 4 : 2); ++k) {
            int line = r + G * k;
            line = line < nl ? line : nl - 1;
            const double t = rec[(size_t)line * 16];
            asm volatile("" ::"v"(t));
        }
    }
    double mur = 0.0;
    if (raw && active && r < Lp) mur = rec[(size_t)(Lp + 2) * Lp + r];
    // diagonal for the trace (rows < L')
    double diag = 0.0;
    if (active && r < Lp) diag = raw ? rec[(size_t)r * Lp + r] - mur * mur : rec[(size_t)r * Lp + r];
    double tr = diag;
#pragma unroll
    for (int o = 1; o < G; o <<= 1) tr += __shfl_xor(tr, o, 64);
    double lam = load_rel * tr / (double)Lp;
    lam = lam < 1e-30 ? 1e-30 : lam;
    // row r: lower part (c <= r) of C + lam I, or the d / m rows (r = L', L'+1)
    double A[CM];
#pragma unroll
    for (int c = 0; c < CM; ++c) {
        double v = 0.0;
        if (row_in && c < Lp && (c <= r || r >= Lp)) {
            if (r >= Lp) v = rec[(size_t)r * Lp + c];
            else if (raw) v = rec[(size_t)c * Lp + r] - rec[(size_t)(Lp + 2) * Lp + c] * mur;
            else v = rec[(size_t)r * Lp + c];
            if (c == r) v += lam;
        }
        A[c] = v;
    }
    bool bad = false;
    double s = 0.0;
    // Columns go in blocks of CB: the block loop is not unrolled (a fully unrolled G = 64
    // body is over 100 KB of code, beyond the instruction cache), the CB columns inside a
    // block are.  After each block the register row shifts left by CB, so column j0 + c of
    // block j0 sits in A[c]: every register index stays a compile-time constant.  The
    // eliminated element of the d / m rows is z_j of L z = d; its squares sum to the score.
    for (int j0 = 0; j0 < Lp; j0 += CB) {
#pragma unroll
        for (int jj = 0; jj < CB; ++jj) {
            const int j = j0 + jj;
            if (j < Lp) {
                const double aj = A[jj];
                const double d = __shfl(aj, base + j, 64);
                bad = bad || !(d > 0.0);
                const double inv = 1.0 / sqrt(d);
                const double l = aj * inv;
                s = fma(l, l, s);
                col[r] = l;
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
                // rank-1 update of the rows below: rows above column j0 + c take a zero
                // multiplier instead of a branch (their entries there are never read)
#pragma unroll
                for (int c = jj + 1; c < CM; ++c) {
                    if (j0 + c < Lp) {
                        const double lc = col[j0 + c];
                        const double m = r >= j0 + c ? l : 0.0;
                        A[c] = fma(-m, lc, A[c]);
                    }
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            }
        }
#pragma unroll
        for (int c = 0; c < CM; ++c) A[c] = c + CB < CM ? A[c + CB] : 0.0;
    }
    if (active && r == Lp && lrx_out) *lrx_out = bad ? INFINITY : (float)s;
    if (active && r == Lp + 1 && dwrx_out) *dwrx_out = bad ? INFINITY : (float)s;
}

}  // namespace hsad
