// grx.hip -- global RX: eq. (1) of Sec. 2.1 with the background formed by every pixel of
// the image, so one mean and one covariance serve all pixels.
//
//   mu = (1/N) sum_p x_p,   C = (1/N) sum_p (x_p - mu)(x_p - mu)^T   (two passes, exact centring)
//   lambda = load_rel tr(C) / L' (at least 1e-30),   C + lambda I = L L^T
//   score_p = (x_p - mu)^T (C + lambda I)^-1 (x_p - mu) = || W (x_p - mu) ||^2,   W = L^-1
//
// Kernels (all on the caller's stream, FP64 arithmetic, FP32 storage of the cube):
//   grx_mean_kernel     fixed pixel ranges -> per-range band sums (fixed order), then
//   grx_mean_final      the ranges in order -> mu
//   grx_gram_kernel     centred samples staged in LDS, upper 16 x 16 tiles of the Gram on
//                       FP64 matrix cores (v_mfma_f64_16x16x4f64), one partial per range
//   grx_gram_reduce     partials summed in range order, / N, mirrored into the padded matrix
//   grx_factor_kernel   loading and the blocked Cholesky (16-column blocks), one workgroup,
//                       matrix in the workspace (L2-resident); inverses of the diagonal blocks
//   grx_inverse_kernel  W = L^-1 by blocked forward substitution, one workgroup per column block
//   grx_score_kernel<T> Z = D W^T on matrix cores, 16 pixels per wavefront with their centred
//                       samples held in registers, W staged in LDS one 16-row block at a time,
//                       score = row sums of Z^2
// Every reduction runs in a fixed order, so the result is deterministic.  The matrix is
// padded to L'pad = 16 ceil(L'/16) with an identity block, so the factor and the inverse are
// block-diagonal with identity padding and the padded bands (zero samples) add nothing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "internal.hpp"

namespace hsad {

typedef double f64x4_g __attribute__((ext_vector_type(4)));

static constexpr int kGrxMaxLp = 256;
static constexpr int kGrxMeanBlocks = 1024;
static constexpr int kGrxTilesPerWave = 8;

__host__ __device__ inline int grx_lds_stride(int Lpad)
{
    // a row stride of 32 (mod 64) four-byte words: the two halves of a wavefront's 4-row x
    // 16-column fragment read fall on disjoint banks
    return ((Lpad / 16) & 1) ? Lpad : Lpad + 16;
}

// ---- mean ----------------------------------------------------------------------------
__global__ __launch_bounds__(256) void grx_mean_kernel(const float *__restrict__ x, int64_t npix, int Lp,
                                                       int nblk, double *__restrict__ part)
{
    __shared__ double red[256];
    const int t = threadIdx.x, blk = blockIdx.x;
    const int64_t p0 = npix * blk / nblk, p1 = npix * (blk + 1) / nblk;
    const int PL = 256 / Lp;            // pixel lanes
    const int q = t / Lp, b = t - q * Lp;
    double acc = 0.0;
    if (q < PL)
        for (int64_t p = p0 + q; p < p1; p += PL) acc += (double)x[p * Lp + b];
    red[t] = acc;
    __syncthreads();
    if (t < Lp) {
        double s = 0.0;
        for (int k = 0; k < PL; ++k) s += red[k * Lp + t];
        part[(size_t)blk * Lp + t] = s;
    }
}

// fixed-order sum of the 256 values in red (a pairwise tree), result in red[0]
__device__ inline void grx_tree256(double *red)
{
    const int t = threadIdx.x;
    for (int h = 128; h > 0; h >>= 1) {
        __syncthreads();
        if (t < h) red[t] += red[t + h];
    }
    __syncthreads();
}

// one workgroup per band b < Lpad: thread t sums the ranges t, t + 256, ... in order, then
// a fixed tree over the threads
__global__ __launch_bounds__(256) void grx_mean_final(const double *__restrict__ part, int nblk, int Lp, int Lpad,
                                                      int64_t npix, double *__restrict__ mu,
                                                      double *__restrict__ mean_out)
{
    __shared__ double red[256];
    const int b = blockIdx.x, t = threadIdx.x;
    double s = 0.0;
    if (b < Lp)
        for (int k = t; k < nblk; k += 256) s += part[(size_t)k * Lp + b];
    red[t] = s;
    grx_tree256(red);
    if (t == 0) {
        const double m = b < Lp ? red[0] / (double)npix : 0.0;
        mu[b] = m;
        if (mean_out && b < Lp) mean_out[b] = m;
    }
}

// ---- Gram ----------------------------------------------------------------------------
__device__ inline void grx_tile_of(int t, int T, int &bi, int &bj)
{
    // tile t of the upper triangle (bi <= bj), row-major
    bi = 0;
    while (t >= T - bi) {
        t -= T - bi;
        ++bi;
    }
    bj = bi + t;
}

// grid: S pixel ranges x G tile groups, blockIdx.x = s * G + g (the groups of one range
// are dispatched together, so their staging reads share the caches)
__global__ __launch_bounds__(256) void grx_gram_kernel(const float *__restrict__ x, int64_t npix, int Lp, int Lpad,
                                                       const double *__restrict__ mu, int S, int G, int P,
                                                       double *__restrict__ part)
{
    extern __shared__ double stage[];
    const int T = Lpad / 16, ntiles = T * (T + 1) / 2;
    const int g = blockIdx.x % G, s = blockIdx.x / G;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int ld = grx_lds_stride(Lpad);
    const int64_t p0 = npix * s / S, p1 = npix * (s + 1) / S;
    double *mus = stage + (size_t)P * ld;
    for (int b = t; b < Lpad; b += 256) mus[b] = mu[b];
    // padded bands stay zero for the whole kernel
    for (int e = t; e < P * (ld - Lp); e += 256) {
        const int r = e / (ld - Lp), c = Lp + e - r * (ld - Lp);
        stage[(size_t)r * ld + c] = 0.0;
    }
    int tbi[kGrxTilesPerWave], tbj[kGrxTilesPerWave];
    bool on[kGrxTilesPerWave];
#pragma unroll
    for (int m = 0; m < kGrxTilesPerWave; ++m) {
        const int tile = g * 4 * kGrxTilesPerWave + wv + 4 * m;
        on[m] = tile < ntiles;
        grx_tile_of(on[m] ? tile : 0, T, tbi[m], tbj[m]);
    }
    f64x4_g acc[kGrxTilesPerWave];
#pragma unroll
    for (int m = 0; m < kGrxTilesPerWave; ++m)
        for (int e = 0; e < 4; ++e) acc[m][e] = 0.0;
    // per-thread element walk over a P x Lp chunk without divisions in the loop
    const int step_r = 256 / Lp, step_c = 256 - step_r * Lp;
    const int r0 = t / Lp, c0 = t - r0 * Lp;
    const int c16 = lane & 15, g4 = lane >> 4;
    for (int64_t base = p0; base < p1; base += P) {
        __syncthreads();   // previous chunk consumed (and mus / padding written)
        int r = r0, c = c0;
        for (int e = t; e < P * Lp; e += 256) {
            const int64_t p = base + r;
            const double v = p < p1 ? (double)x[p * Lp + c] - mus[c] : 0.0;
            stage[(size_t)r * ld + c] = v;
            r += step_r;
            c += step_c;
            if (c >= Lp) {
                c -= Lp;
                ++r;
            }
        }
        __syncthreads();
        for (int k = 0; k < P; k += 4) {
            const double *row = stage + (size_t)(k + g4) * ld + c16;
#pragma unroll
            for (int m = 0; m < kGrxTilesPerWave; ++m) {
                if (on[m]) {
                    const double a = row[16 * tbi[m]], b = row[16 * tbj[m]];
                    acc[m] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[m], 0, 0, 0);
                }
            }
        }
    }
#pragma unroll
    for (int m = 0; m < kGrxTilesPerWave; ++m) {
        if (on[m]) {
            const int tile = g * 4 * kGrxTilesPerWave + wv + 4 * m;
            double *o = part + ((size_t)s * ntiles + tile) * 256;
#pragma unroll
            for (int e = 0; e < 4; ++e) o[e * 64 + lane] = acc[m][e];
        }
    }
}

// one workgroup of 1024 threads per tile: group g = thread / 256 sums the partials
// g, g + 4, ... of element q = thread % 256 in order, the four groups are added in order;
// then scale by 1/N and write the tile and its mirror into the padded Lpad x Lpad matrix
// (identity on the padding)
__global__ __launch_bounds__(1024) void grx_gram_reduce(const double *__restrict__ part, int S, int Lp, int Lpad,
                                                        int64_t npix, double *__restrict__ A,
                                                        double *__restrict__ cov_out)
{
    __shared__ double red[4][256];
    const int T = Lpad / 16, ntiles = T * (T + 1) / 2;
    const int tile = blockIdx.x, q = threadIdx.x & 255, grp = threadIdx.x >> 8;
    int bi, bj;
    grx_tile_of(tile, T, bi, bj);
    double acc = 0.0;
#pragma unroll 8
    for (int k = grp; k < S; k += 4) acc += part[((size_t)k * ntiles + tile) * 256 + q];
    red[grp][q] = acc;
    __syncthreads();
    if (grp) return;
    const double s = (red[0][q] + red[1][q]) + (red[2][q] + red[3][q]);
    const int e = q >> 6, lane = q & 63;
    // FP64 16x16x4: output element e of lane l is row 4e + (l >> 4), column l & 15
    const int r = 16 * bi + 4 * e + (lane >> 4), c = 16 * bj + (lane & 15);
    double v;
    if (r < Lp && c < Lp)
        v = s / (double)npix;
    else
        v = r == c ? 1.0 : 0.0;
    if (bi < bj || r <= c) {
        A[(size_t)r * Lpad + c] = v;
        A[(size_t)c * Lpad + r] = v;
        if (cov_out && r < Lp && c < Lp) {
            cov_out[(size_t)r * Lp + c] = v;
            cov_out[(size_t)c * Lp + r] = v;
        }
    }
}

// ---- loading and blocked Cholesky (one workgroup of 1024 threads) ----------------------
__global__ __launch_bounds__(1024) void grx_factor_kernel(double *__restrict__ A, double *__restrict__ Wm, int Lp,
                                                          int Lpad, double load_rel, double *__restrict__ flag)
{
    __shared__ double Dl[16][17], Di[16][17];
    __shared__ double P[kGrxMaxLp][17];     // panel of the current block column
    __shared__ double red[16];
    __shared__ int bad;
    const int t = threadIdx.x, nt = blockDim.x, lane = t & 63, wv = t >> 6;
    const int T = Lpad / 16;
    if (t == 0) bad = 0;
    // W starts as zero (its upper part and padding stay so)
    for (int e = t; e < Lpad * Lpad; e += nt) Wm[e] = 0.0;
    // loading: lambda = load_rel tr(C) / L'
    double tr = 0.0;
    for (int i = t; i < Lp; i += nt) tr += A[(size_t)i * Lpad + i];
    for (int o = 32; o > 0; o >>= 1) tr += __shfl_xor(tr, o);
    if (lane == 0) red[wv] = tr;
    __syncthreads();
    double trs = 0.0;
    for (int k = 0; k < nt / 64; ++k) trs += red[k];
    double lam = load_rel * trs / (double)Lp;
    lam = lam < 1e-30 ? 1e-30 : lam;
    for (int i = t; i < Lp; i += nt) A[(size_t)i * Lpad + i] += lam;
    __syncthreads();

#pragma unroll 1
    for (int kb = 0; kb < T; ++kb) {
        const int k0 = 16 * kb;
        // (a) diagonal block: unblocked Cholesky and its inverse, wavefront 0
        if (wv == 0) {
            for (int e = lane; e < 256; e += 64) Dl[e >> 4][e & 15] = A[(size_t)(k0 + (e >> 4)) * Lpad + k0 + (e & 15)];
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
#pragma unroll 1
            for (int j = 0; j < 16; ++j) {
                const double d = Dl[j][j];
                if (!(d > 0.0) && lane == 0) bad = 1;
                const double inv = 1.0 / sqrt(d);
                __builtin_amdgcn_wave_barrier();
                if (lane >= j && lane < 16) Dl[lane][j] = lane == j ? d * inv : Dl[lane][j] * inv;
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
                for (int e = lane; e < 256; e += 64) {
                    const int r = e >> 4, c = e & 15;
                    if (c > j && r >= c) Dl[r][c] -= Dl[r][j] * Dl[c][j];
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            }
            // inverse of the lower-triangular block, column c by lane c
            if (lane < 16) {
                const int c = lane;
#pragma unroll 1
                for (int r = 0; r < 16; ++r) {
                    double v = 0.0;
                    if (r >= c) {
                        double s = r == c ? 1.0 : 0.0;
                        for (int k = c; k < r; ++k) s -= Dl[r][k] * Di[k][c];
                        v = s / Dl[r][r];
                    }
                    Di[r][c] = v;
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            for (int e = lane; e < 256; e += 64) {
                const int r = e >> 4, c = e & 15;
                A[(size_t)(k0 + r) * Lpad + k0 + c] = c <= r ? Dl[r][c] : 0.0;
                Wm[(size_t)(k0 + r) * Lpad + k0 + c] = Di[r][c];
            }
        }
        __syncthreads();
        // (b) panel below the block: L_ik = A_ik Di^T (rows i >= k0 + 16)
        const int nrow = Lpad - k0 - 16;
        for (int e = t; e < nrow * 16; e += nt) {
            const int i = e >> 4, c = e & 15;
            const double *arow = A + (size_t)(k0 + 16 + i) * Lpad + k0;
            double s = 0.0;
            for (int q = 0; q <= c; ++q) s += arow[q] * Di[c][q];
            P[i][c] = s;
        }
        __syncthreads();
        for (int e = t; e < nrow * 16; e += nt) {
            const int i = e >> 4, c = e & 15;
            A[(size_t)(k0 + 16 + i) * Lpad + k0 + c] = P[i][c];
        }
        // (c) trailing update A_ij -= sum_q P_iq P_jq for j <= i, in 4 x 4 blocks
        const int nb4 = nrow / 4;
        for (int e = t; e < nb4 * nb4; e += nt) {
            const int bi = e / nb4, bj = e - bi * nb4;
            if (bj > bi) continue;
            double acc[4][4];
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[u][v] = 0.0;
#pragma unroll 2
            for (int q = 0; q < 16; ++q) {
                double li[4], lj[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    li[u] = P[4 * bi + u][q];
                    lj[u] = P[4 * bj + u][q];
                }
#pragma unroll
                for (int u = 0; u < 4; ++u)
#pragma unroll
                    for (int v = 0; v < 4; ++v) acc[u][v] = fma(li[u], lj[v], acc[u][v]);
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int i = 4 * bi + u, j = 4 * bj + v;
                    if (j <= i) A[(size_t)(k0 + 16 + i) * Lpad + k0 + 16 + j] -= acc[u][v];
                }
        }
        __syncthreads();
    }
    if (t == 0) flag[0] = bad ? 1.0 : 0.0;
}

// ---- inverse W = L^-1, one workgroup per 16-column block jb -----------------------------
// Forward substitution over the row blocks below the diagonal:
//   W_ib,jb = -Di_ib sum_{kb = jb}^{ib - 1} L_ib,kb W_kb,jb   (ib > jb),  W_jb,jb = Di_jb,
// with Di_ib = L_ib,ib^-1 (written by the factorisation).  The workgroup keeps its column
// block of W in LDS and stages each row block of L (columns jb .. ib - 1) before using it.
// LDS (doubles): Wc [Lpad][16], Lr [16][Lpad + 1], S [16][17], Di [16][17].
__global__ __launch_bounds__(256) void grx_inverse_kernel(const double *__restrict__ A, double *__restrict__ Wm,
                                                          int Lpad)
{
    extern __shared__ double sh[];
    const int ldl = Lpad + 1;
    double *Wc = sh, *Lr = Wc + (size_t)Lpad * 16, *Sb = Lr + (size_t)16 * ldl, *Db = Sb + 16 * 17;
    const int T = Lpad / 16, jb = blockIdx.x, j0 = 16 * jb, t = threadIdx.x;
    const int r = t >> 4, c = t & 15;
    Wc[(size_t)(j0 + r) * 16 + c] = Wm[(size_t)(j0 + r) * Lpad + j0 + c];
    for (int ib = jb + 1; ib < T; ++ib) {
        const int i0 = 16 * ib, w = i0 - j0;
        for (int e = t; e < 16 * w; e += 256) {
            const int rr = e / w, k = e - rr * w;
            Lr[(size_t)rr * ldl + k] = A[(size_t)(i0 + rr) * Lpad + j0 + k];
        }
        Db[r * 17 + c] = Wm[(size_t)(i0 + r) * Lpad + i0 + c];
        __syncthreads();
        double acc = 0.0;
        for (int k = 0; k < w; ++k) acc = fma(Lr[(size_t)r * ldl + k], Wc[(size_t)(j0 + k) * 16 + c], acc);
        Sb[r * 17 + c] = acc;
        __syncthreads();
        double v = 0.0;
        for (int q = 0; q <= r; ++q) v = fma(Db[r * 17 + q], Sb[q * 17 + c], v);
        Wc[(size_t)(i0 + r) * 16 + c] = -v;
        __syncthreads();
    }
    for (int e = t; e < (Lpad - j0) * 16; e += 256) {
        const int rr = j0 + (e >> 4), cc = e & 15;
        Wm[(size_t)rr * Lpad + j0 + cc] = Wc[(size_t)rr * 16 + cc];
    }
}

static size_t grx_inverse_lds(int Lpad) { return ((size_t)Lpad * 16 + 16 * (size_t)(Lpad + 1) + 2 * 16 * 17) * sizeof(double); }

// ---- scores --------------------------------------------------------------------------
// 8 wavefronts x 16 pixels per workgroup.  Lane l supplies the centred sample of pixel
// (l & 15), band 4c + (l >> 4) as the A operand of k-chunk c (held in registers for all
// c); the B operand B[k][j] = W[16 jb + j][k] comes from the LDS copy of W's row block jb,
// stored transposed.  Z tile element e of lane l is pixel 4e + (l >> 4), column l & 15.
template <int T>
__global__ __launch_bounds__(512) void grx_score_kernel(const float *__restrict__ x, int64_t npix, int Lp,
                                                        const double *__restrict__ mu,
                                                        const double *__restrict__ Wm,
                                                        const double *__restrict__ flag, float *__restrict__ scores)
{
    constexpr int Lpad = 16 * T;
    __shared__ double WsT[Lpad * 17];   // [k][j], k < Lpad, row stride 17
    __shared__ double mus[Lpad];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    for (int b = t; b < Lpad; b += 512) mus[b] = mu[b];
    __syncthreads();
    const int64_t pb = (int64_t)blockIdx.x * 128 + 16 * wv;
    const int64_t pp = pb + (lane & 15);
    const bool pin = pp < npix;
    double dA[4 * T];
#pragma unroll
    for (int c = 0; c < 4 * T; ++c) {
        const int b = 4 * c + (lane >> 4);
        const int bc = b < Lp ? b : Lp - 1;
        const double v = (double)x[(pin ? pp : 0) * Lp + bc] - mus[bc];
        dA[c] = (pin && b < Lp) ? v : 0.0;
    }
    double sq[4] = {0.0, 0.0, 0.0, 0.0};
    for (int jb = 0; jb < T; ++jb) {
        const int kmax = 16 * (jb + 1);
        __syncthreads();
        for (int e = t; e < 16 * kmax; e += 512) {
            const int j = e / kmax, k = e - j * kmax;
            WsT[k * 17 + j] = Wm[(size_t)(16 * jb + j) * Lpad + k];
        }
        __syncthreads();
        f64x4_g acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int c = 0; c < 4 * T; ++c) {
            if (c < 4 * (jb + 1)) {
                const double b = WsT[(4 * c + (lane >> 4)) * 17 + (lane & 15)];
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(dA[c], b, acc, 0, 0, 0);
            }
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) sq[e] += acc[e] * acc[e];
    }
    // sum over the 16 columns held by the lanes of one 16-lane group
#pragma unroll
    for (int e = 0; e < 4; ++e)
        for (int o = 1; o < 16; o <<= 1) sq[e] += __shfl_xor(sq[e], o);
    const bool bad = flag[0] != 0.0;
    const int e = lane & 15;
    if (e < 4) {
        const int64_t p = pb + 4 * e + (lane >> 4);
        double v = e == 0 ? sq[0] : e == 1 ? sq[1] : e == 2 ? sq[2] : sq[3];
        if (p < npix) scores[p] = bad ? INFINITY : (float)v;
    }
}

// ---- workspace layout ----------------------------------------------------------------
struct GrxPlan {
    int Lp, Lpad, T, ntiles;
    int nblk;            // mean ranges
    int S, G, P;         // Gram ranges, tile groups, staged pixels per chunk
    size_t off_mu, off_part, off_gpart, off_A, off_W, off_flag, total;   // in doubles
};

static size_t al32(size_t d) { return (d + 31) & ~(size_t)31; }   // 256-byte multiples

static GrxPlan grx_plan(int64_t npix, int64_t Lp)
{
    GrxPlan g;
    g.Lp = (int)Lp;
    g.T = (int)((Lp + 15) / 16);
    g.Lpad = 16 * g.T;
    g.ntiles = g.T * (g.T + 1) / 2;
    g.nblk = (int)std::min<int64_t>(kGrxMeanBlocks, std::max<int64_t>(1, npix / 64));
    const int ld = grx_lds_stride(g.Lpad);
    int P = (int)((64 * 1024 / sizeof(double) - g.Lpad) / ld) & ~3;
    g.P = std::max(4, std::min(256, P));
    g.G = (g.ntiles + 4 * kGrxTilesPerWave - 1) / (4 * kGrxTilesPerWave);
    // pixel ranges: enough workgroups to fill the GPU, at least 2048 pixels each
    const int64_t ranges = std::max<int64_t>(1, npix / 2048);
    g.S = (int)std::max<int64_t>(1, std::min<int64_t>((1024 + g.G - 1) / g.G, ranges));
    size_t o = 0;
    g.off_mu = o;    o += al32((size_t)g.Lpad);
    g.off_part = o;  o += al32((size_t)g.nblk * g.Lp);
    g.off_gpart = o; o += al32((size_t)g.S * g.ntiles * 256);
    g.off_A = o;     o += al32((size_t)g.Lpad * g.Lpad);
    g.off_W = o;     o += al32((size_t)g.Lpad * g.Lpad);
    g.off_flag = o;  o += 32;
    g.total = o;
    return g;
}

template <int T>
static int launch_score(const float *x, int64_t npix, int Lp, const double *mu, const double *Wm,
                        const double *flag, float *scores, hipStream_t s)
{
    const unsigned grid = (unsigned)((npix + 127) / 128);
    hipLaunchKernelGGL(grx_score_kernel<T>, dim3(grid), dim3(512), 0, s, x, npix, Lp, mu, Wm, flag, scores);
    return check_launch("grx_score_kernel");
}

}  // namespace hsad

using namespace hsad;

extern "C" size_t hsad_global_rx_workspace_bytes(int64_t npix, int64_t Lp)
{
    if (npix < 1 || Lp < 1 || Lp > kGrxMaxLp) return 0;
    return grx_plan(npix, Lp).total * sizeof(double);
}

extern "C" int hsad_global_rx(const float *x, int64_t npix, int64_t Lp, double load_rel, float *scores,
                              double *mean, double *cov, void *ws, size_t ws_bytes, hipStream_t stream)
{
    clear_error();
    if (!x || !scores) return fail(HSAD_EINVAL, "hsad_global_rx: x and scores are required");
    if (npix < 1 || Lp < 1) return fail(HSAD_EINVAL, "hsad_global_rx: npix and L' must be >= 1");
    if (npix > ((int64_t)1 << 31)) return fail(HSAD_EUNSUPPORTED, "hsad_global_rx: more than 2^31 pixels");
    if (Lp > kGrxMaxLp) return fail(HSAD_EUNSUPPORTED, "hsad_global_rx: L' above 256");
    if (!(load_rel >= 0.0) || !std::isfinite(load_rel))
        return fail(HSAD_EINVAL, "hsad_global_rx: load_rel must be finite and >= 0");
    const GrxPlan g = grx_plan(npix, Lp);
    if (!ws || ws_bytes < g.total * sizeof(double))
        return fail(HSAD_ENOMEM, "hsad_global_rx: workspace too small (see hsad_global_rx_workspace_bytes)");
    double *base = (double *)ws;
    double *mu = base + g.off_mu, *part = base + g.off_part, *gpart = base + g.off_gpart;
    double *A = base + g.off_A, *Wm = base + g.off_W, *flag = base + g.off_flag;

    hipLaunchKernelGGL(grx_mean_kernel, dim3(g.nblk), dim3(256), 0, stream, x, npix, g.Lp, g.nblk, part);
    if (int rc = check_launch("grx_mean_kernel")) return rc;
    hipLaunchKernelGGL(grx_mean_final, dim3((unsigned)g.Lpad), dim3(256), 0, stream, part, g.nblk, g.Lp, g.Lpad,
                       npix, mu, mean);
    if (int rc = check_launch("grx_mean_final")) return rc;
    const size_t sh = ((size_t)g.P * grx_lds_stride(g.Lpad) + g.Lpad) * sizeof(double);
    if (int rc = allow_lds((const void *)grx_gram_kernel, sh, "grx_gram_kernel")) return rc;
    hipLaunchKernelGGL(grx_gram_kernel, dim3((unsigned)(g.S * g.G)), dim3(256), sh, stream, x, npix, g.Lp, g.Lpad,
                       (const double *)mu, g.S, g.G, g.P, gpart);
    if (int rc = check_launch("grx_gram_kernel")) return rc;
    hipLaunchKernelGGL(grx_gram_reduce, dim3((unsigned)g.ntiles), dim3(1024), 0, stream, (const double *)gpart, g.S,
                       g.Lp, g.Lpad, npix, A, cov);
    if (int rc = check_launch("grx_gram_reduce")) return rc;
    hipLaunchKernelGGL(grx_factor_kernel, dim3(1), dim3(1024), 0, stream, A, Wm, g.Lp, g.Lpad, load_rel, flag);
    if (int rc = check_launch("grx_factor_kernel")) return rc;
    if (g.T > 1) {
        const size_t shi = grx_inverse_lds(g.Lpad);
        if (int rc = allow_lds((const void *)grx_inverse_kernel, shi, "grx_inverse_kernel")) return rc;
        hipLaunchKernelGGL(grx_inverse_kernel, dim3((unsigned)(g.T - 1)), dim3(256), shi, stream,
                           (const double *)A, Wm, g.Lpad);
        if (int rc = check_launch("grx_inverse_kernel")) return rc;
    }
    switch (g.T) {
#define HSAD_GRX_T(n) \
    case n: return launch_score<n>(x, npix, g.Lp, mu, Wm, flag, scores, stream);
        HSAD_GRX_T(1) HSAD_GRX_T(2) HSAD_GRX_T(3) HSAD_GRX_T(4) HSAD_GRX_T(5) HSAD_GRX_T(6)
        HSAD_GRX_T(7) HSAD_GRX_T(8) HSAD_GRX_T(9) HSAD_GRX_T(10) HSAD_GRX_T(11) HSAD_GRX_T(12)
        HSAD_GRX_T(13) HSAD_GRX_T(14) HSAD_GRX_T(15) HSAD_GRX_T(16)
#undef HSAD_GRX_T
    default: return fail(HSAD_EUNSUPPORTED, "hsad_global_rx: L' above 256");
    }
}
