// surrogate.hip -- a learned per-pixel surrogate of the LRX score (eq. 1): features, a
// small MLP trained and evaluated with BF16 matrix-core kernels, and the hybrid run that
// sends the pixels near the eq. (12) threshold, plus a seeded audit sample, back to the
// exact detector.
//
// Features of pixel p (3 L' inputs, from the reduced cube and the annulus = outer minus
// inner window of Sec. 2.2), per band i < L':
//   z_i  = (x_i - mu_i) / sqrt(v_i + 1e-12),   lv_i = log(v_i + 1e-12),   mu_i,
// with mu_i, v_i the annulus mean and 1/n variance of band i.  This carries the same
// information as (coefficients, annulus mean, annulus diagonal variance), parameterised so
// that the standardised residual, which drives the score, is an input.  The sums are FP64
// box sums over LDS tiles, as in the exact small-L' detector, restricted to the diagonal.
// Network: D = 3 L' inputs, normalised per column and zero-padded to Dp (a multiple of
// 32) -> 128 -> ReLU -> 128 -> ReLU -> 1.  Trained by mean squared error on log1p(LRX).
// The two wide layers run on v_mfma_f32_16x16x32_bf16: BF16 operands (inputs, weights,
// activations, back-propagated errors), FP32 accumulation, FP32 master weights and Adam
// moments.  Operand layout used throughout: lane l holds row (l & 15) of the 16 x 32 A
// block at k = 8 (l >> 4) .. 8 (l >> 4) + 7, and column (l & 15) of B at the same k; the
// result element e of lane l is row 4 (l >> 4) + e, column (l & 15).
// Parameter vector (FP32): W1 [Dp][128] | b1 [128] | W2 [128][128] | b2 [128] | w3 [128] |
// b3 | 3 pad, with h1 = relu(x W1 + b1), h2 = relu(h1 W2 + b2), y = h2 . w3 + b3.
// BF16 copies (the matrix-core operands): W1t [128][Dp], W2t [128][128] (both out x in)
// and W2n [128][128] (in x out, for the backward pass).
#include <hip/hip_runtime.h>

#include <vector>

#include <algorithm>
#include <cmath>

#include "internal.hpp"

namespace hsad {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

static constexpr int HID = 128;
static constexpr int LDH = HID + 8;      // padded LDS row of a hidden activation tile
static constexpr int MAX_DP = 256;

__host__ __device__ inline int64_t off_b1(int Dp) { return (int64_t)Dp * HID; }
__host__ __device__ inline int64_t off_W2(int Dp) { return off_b1(Dp) + HID; }
__host__ __device__ inline int64_t off_b2(int Dp) { return off_W2(Dp) + HID * HID; }
__host__ __device__ inline int64_t off_w3(int Dp) { return off_b2(Dp) + HID; }
__host__ __device__ inline int64_t off_b3(int Dp) { return off_w3(Dp) + HID; }
__host__ __device__ inline int64_t mlp_nparams(int Dp) { return off_b3(Dp) + 4; }
__host__ __device__ inline int64_t mlp_nbf16(int Dp) { return (int64_t)HID * Dp + 2 * HID * HID; }

__device__ __forceinline__ uint16_t bf16_bits(float v) { return __builtin_bit_cast(uint16_t, (__bf16)v); }
__device__ __forceinline__ float bf16_val(uint16_t b) { return (float)__builtin_bit_cast(__bf16, b); }

namespace {

// ------------------------------------------------------------------------------------
// features
// ------------------------------------------------------------------------------------
constexpr int FTY = 16;

__device__ __forceinline__ int fclip(int c, int r, int n)
{
    const int lo = c - r < 0 ? 0 : c - r, hi = c + r > n - 1 ? n - 1 : c + r;
    return hi - lo + 1;
}

template <int FCC, int FTX>
size_t features_smem(int R)
{
    const size_t EX = FTX + 2 * R, EY = FTY + 2 * R;
    return (size_t)FTY * EX * (2 * FCC) * sizeof(double) + EY * EX * FCC * sizeof(float);
}

// One FTX x 16 pixel tile per workgroup (FTX = 32 or 16); bands in chunks of FCC.  Per chunk: stage the tile
// and its halo (values shifted by a per-chunk reference so the FP64 sums stay small),
// vertical running sums per (column, 4-row block), running sums along each row, then the
// window sums as differences (outer minus inner).  Output: FP32 features [p][3 L'] when
// norm is NULL, else normalised BF16 rows [p][Dp] (zero padded).
template <int FCC, int FTX>
__global__ __launch_bounds__(FTX * FTY) void surr_features_kernel(const float *__restrict__ x, int H, int W,
                                                            int Lp, int R, int RI, int has_inner,
                                                            const float *__restrict__ norm, int Dp,
                                                            float *__restrict__ feat,
                                                            uint16_t *__restrict__ packed)
{
    extern __shared__ double smem[];
    constexpr int GP = 2 * FCC, FNT = FTX * FTY;
    const int EX = FTX + 2 * R, EY = FTY + 2 * R;
    double *V = smem;                                                      // FTY*EX*GP
    float *xs = reinterpret_cast<float *>(smem + (size_t)FTY * EX * GP);   // EY*EX*FCC
    const int tid = threadIdx.x;
    const int y0 = blockIdx.y * FTY, x0 = blockIdx.x * FTX;
    const int ty = tid / FTX, tx = tid - ty * FTX;
    const int py = y0 + ty, px = x0 + tx;
    const bool valid = py < H && px < W;
    int n_a = 1;
    if (valid) {
        const int n_o = fclip(py, R, H) * fclip(px, R, W);
        const int n_i = has_inner ? fclip(py, RI, H) * fclip(px, RI, W) : 0;
        n_a = n_o - n_i;
    }
    const int D = 3 * Lp;
    const size_t pix = (size_t)py * W + px;
    for (int c0 = 0; c0 < Lp; c0 += FCC) {
        const int cc = Lp - c0 < FCC ? Lp - c0 : FCC;
        double ref[FCC];
        {
            const int ry = min(y0 + FTY / 2, H - 1), rx = min(x0 + FTX / 2, W - 1);
#pragma unroll
            for (int i = 0; i < FCC; ++i) {
                const float v = i < cc ? x[((size_t)ry * W + rx) * Lp + c0 + i] : 0.f;
                ref[i] = isfinite(v) ? (double)v : 0.0;
            }
        }
        __syncthreads();
        // unconditional loads from clamped coordinates, several iterations in flight
#pragma unroll 4
        for (int t = tid; t < EY * EX; t += FNT) {
            const int ey = t / EX, ex = t - ey * EX;
            const int gy = y0 - R + ey, gx = x0 - R + ex;
            const bool in = gy >= 0 && gy < H && gx >= 0 && gx < W;
            const int cy = gy < 0 ? 0 : gy >= H ? H - 1 : gy, cx = gx < 0 ? 0 : gx >= W ? W - 1 : gx;
            const float *src = x + ((size_t)cy * W + cx) * Lp + c0;
#pragma unroll
            for (int i = 0; i < FCC; ++i) {
                const float v = src[i < cc ? i : cc - 1];
                xs[(size_t)t * FCC + i] = (in && i < cc) ? v : (float)ref[i];
            }
        }
        __syncthreads();
        double S[GP];
#pragma unroll
        for (int g = 0; g < GP; ++g) S[g] = 0.0;
        for (int win = has_inner ? 0 : 1; win < 2; ++win) {
            const int h = win == 0 ? RI : R;
            const int eoff = R - h;
            for (int job = tid; job < EX * (FTY / 4); job += FNT) {
                const int rb = job / EX, c = job - rb * EX, r0 = rb * 4;
                double acc[GP];
#pragma unroll
                for (int g = 0; g < GP; ++g) acc[g] = 0.0;
                // uniform trip count (2h+1) and counter: the loop is unrolled and its LDS
                // reads overlap (a per-lane bound would wait for each read in turn)
#pragma unroll 4
                for (int k = 0; k <= 2 * h; ++k) {
                    const int ey = r0 + eoff + k;
#pragma unroll
                    for (int i = 0; i < FCC; ++i) {
                        const double f = (double)xs[((size_t)ey * EX + c) * FCC + i] - ref[i];
                        acc[i] += f;
                        acc[FCC + i] += f * f;
                    }
                }
#pragma unroll
                for (int g = 0; g < GP; ++g) V[((size_t)r0 * EX + c) * GP + g] = acc[g];
                for (int r = 1; r < 4; ++r) {
                    const size_t ta = (size_t)(r0 + r + eoff + 2 * h) * EX + c;
                    const size_t tb = (size_t)(r0 + r - 1 + eoff) * EX + c;
#pragma unroll
                    for (int i = 0; i < FCC; ++i) {
                        const double fa = (double)xs[ta * FCC + i] - ref[i];
                        const double fb = (double)xs[tb * FCC + i] - ref[i];
                        acc[i] += fa - fb;
                        acc[FCC + i] += fa * fa - fb * fb;
                    }
#pragma unroll
                    for (int g = 0; g < GP; ++g) V[((size_t)(r0 + r) * EX + c) * GP + g] = acc[g];
                }
            }
            __syncthreads();
            for (int job = tid; job < FTY * GP; job += FNT) {
                const int r = job / GP, g = job - r * GP;
                double run = 0.0;
                double *v = V + (size_t)r * EX * GP + g;
                for (int c = 0; c < EX; ++c) {
                    run += v[(size_t)c * GP];
                    v[(size_t)c * GP] = run;
                }
            }
            __syncthreads();
            const int c_hi = tx + eoff + 2 * h, c_lo = tx + eoff - 1;
#pragma unroll
            for (int g = 0; g < GP; ++g) {
                const double hs = V[((size_t)ty * EX + c_hi) * GP + g] -
                                  (c_lo < 0 ? 0.0 : V[((size_t)ty * EX + c_lo) * GP + g]);
                S[g] += win == 0 ? -hs : hs;
            }
            __syncthreads();
        }
        if (valid) {
            const double inv = 1.0 / (double)n_a;
            const float *pc = x + pix * Lp + c0;
            float f3[3][FCC];
#pragma unroll
            for (int i = 0; i < FCC; ++i) {
                if (i < cc) {
                    const double mf = S[i] * inv;
                    double var = S[FCC + i] * inv - mf * mf;
                    var = var < 0.0 ? 0.0 : var;
                    const double mu = ref[i] + mf;
                    const double ve = var + 1e-12;
                    f3[0][i] = (float)(((double)pc[i] - mu) / sqrt(ve));
                    f3[1][i] = (float)log(ve);
                    f3[2][i] = (float)mu;
                }
            }
            // the pixel's features go to three runs of cc consecutive columns; with an even
            // L' the runs start at even columns and go out as 32-bit pairs of BF16 values
            const bool pairs = norm && (Lp & 1) == 0 && (c0 & 1) == 0;
            const bool quads = FCC == 4 && norm && (Lp & 3) == 0 && (c0 & 3) == 0 && cc == 4;
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                if (quads) {     // four columns from a multiple of four: one 64-bit store
                    const int k = q * Lp + c0;
                    uint32_t w[2];
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const uint32_t lo = bf16_bits((f3[q][2 * h] - norm[2 * (k + 2 * h)]) * norm[2 * (k + 2 * h) + 1]);
                        const uint32_t hi =
                            bf16_bits((f3[q][2 * h + 1] - norm[2 * (k + 2 * h + 1)]) * norm[2 * (k + 2 * h + 1) + 1]);
                        w[h] = lo | (hi << 16);
                    }
                    *reinterpret_cast<uint2 *>(packed + pix * Dp + k) = make_uint2(w[0], w[1]);
                    continue;
                }
#pragma unroll
                for (int i = 0; i < FCC; i += 2) {
                    const int k = q * Lp + c0 + i;
                    if (pairs && i + 1 < cc) {
                        const uint32_t lo = bf16_bits((f3[q][i] - norm[2 * k]) * norm[2 * k + 1]);
                        const uint32_t hi = bf16_bits((f3[q][i + 1] - norm[2 * k + 2]) * norm[2 * k + 3]);
                        *reinterpret_cast<uint32_t *>(packed + pix * Dp + k) = lo | (hi << 16);
                    } else {
#pragma unroll
                        for (int u = 0; u < 2; ++u) {
                            if (i + u < cc) {
                                if (norm)
                                    packed[pix * Dp + k + u] =
                                        bf16_bits((f3[q][i + u] - norm[2 * (k + u)]) * norm[2 * (k + u) + 1]);
                                else
                                    feat[pix * D + k + u] = f3[q][i + u];
                            }
                        }
                    }
                }
            }
        }
    }
    if (valid && norm)
        for (int k = D; k < Dp; ++k) packed[pix * Dp + k] = 0;
}

// per-column normalisation of an n x D FP32 matrix: norm[2c] = mean, norm[2c+1] = 1/std
// (population std, two FP64 passes; 1 when the column is constant).  One block per column.
__global__ __launch_bounds__(256) void norm_stats_kernel(const float *__restrict__ a, int64_t n, int D,
                                                         float *__restrict__ norm)
{
    __shared__ double red[4];
    __shared__ double mean_s;
    const int c = blockIdx.x;
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) s += (double)a[i * D + c];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) mean_s = (red[0] + red[1] + red[2] + red[3]) / (double)n;
    __syncthreads();
    const double m = mean_s;
    double q = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        const double d = (double)a[i * D + c] - m;
        q += d * d;
    }
    for (int o = 32; o > 0; o >>= 1) q += __shfl_xor(q, o);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = q;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double sd = sqrt((red[0] + red[1] + red[2] + red[3]) / (double)n);
        norm[2 * c] = (float)m;
        norm[2 * c + 1] = sd > 1e-12 ? (float)(1.0 / sd) : 1.f;
    }
}

// (f - shift) * scale -> BF16 rows of Dp (zero padded)
__global__ __launch_bounds__(256) void mlp_pack_kernel(const float *__restrict__ feat, int64_t n, int D,
                                                       int Dp, const float *__restrict__ norm,
                                                       uint16_t *__restrict__ out)
{
    const int64_t total = n * Dp;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = t / Dp;
        const int k = (int)(t - r * Dp);
        out[t] = k < D ? bf16_bits((feat[r * D + k] - norm[2 * k]) * norm[2 * k + 1]) : (uint16_t)0;
    }
}

// training targets log1p(score); non-finite scores give NaN targets, which training skips
__global__ __launch_bounds__(256) void targets_kernel(const float *__restrict__ s, int64_t n, float *__restrict__ t)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float v = s[i];
        t[i] = isfinite(v) && v > -1.f ? (float)log1p((double)v) : __builtin_nanf("");
    }
}

// ------------------------------------------------------------------------------------
// matrix-core pieces
// ------------------------------------------------------------------------------------
__device__ __forceinline__ bf16x8 ld8(const uint16_t *p) { return *reinterpret_cast<const bf16x8 *>(p); }

__device__ __forceinline__ bf16x8 ld8s(const uint16_t *p, int stride)
{
    bf16x8 v;
#pragma unroll
    for (int t = 0; t < 8; ++t) v[t] = __builtin_bit_cast(__bf16, p[(size_t)t * stride]);
    return v;
}

__device__ __forceinline__ f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Forward pass of 16 rows by one wavefront.  Row r of the input is X + min(r, nrows-1)*ldx
// (Dp BF16 values).  W1t (ld ldw1) and W2t (ld ldw2) are BF16, out x in.  Writes the ReLU
// outputs h1, h2 as BF16 into the wave's tiles h1s, h2s ([16][LDH]) and returns the four
// outputs of rows 4 (l >> 4) + e in y4 (every lane of a 16-lane group holds the same).
__device__ inline void mlp_fwd16(const uint16_t *X, int ldx, int nrows, int Dp, const uint16_t *W1t, int ldw1,
                                 const float *b1, const uint16_t *W2t, int ldw2, const float *b2,
                                 const float *w3, float b3, uint16_t *h1s, uint16_t *h2s, float *y4)
{
    const int lane = threadIdx.x & 63, r16 = lane & 15, g = lane >> 4;
    const uint16_t *xr = X + (size_t)(r16 < nrows ? r16 : nrows - 1) * ldx;
    f32x4 acc[8];
#pragma unroll
    for (int jt = 0; jt < 8; ++jt) acc[jt] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < Dp; k0 += 32) {
        const bf16x8 a = ld8(xr + k0 + 8 * g);
#pragma unroll
        for (int jt = 0; jt < 8; ++jt)
            acc[jt] = mfma(a, ld8(W1t + (size_t)(16 * jt + r16) * ldw1 + k0 + 8 * g), acc[jt]);
    }
#pragma unroll
    for (int jt = 0; jt < 8; ++jt)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int col = 16 * jt + r16;
            const float v = acc[jt][e] + b1[col];
            h1s[(4 * g + e) * LDH + col] = bf16_bits(v > 0.f ? v : 0.f);
        }
    wave_lds_sync();
#pragma unroll
    for (int jt = 0; jt < 8; ++jt) acc[jt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int k0 = 0; k0 < HID; k0 += 32) {
        const bf16x8 a = ld8(h1s + r16 * LDH + k0 + 8 * g);
#pragma unroll
        for (int jt = 0; jt < 8; ++jt)
            acc[jt] = mfma(a, ld8(W2t + (size_t)(16 * jt + r16) * ldw2 + k0 + 8 * g), acc[jt]);
    }
    float ys[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int jt = 0; jt < 8; ++jt)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int col = 16 * jt + r16;
            float v = acc[jt][e] + b2[col];
            v = v > 0.f ? v : 0.f;
            const uint16_t hb = bf16_bits(v);
            h2s[(4 * g + e) * LDH + col] = hb;
            ys[e] += bf16_val(hb) * w3[col];
        }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        float v = ys[e];
        for (int o = 1; o < 16; o <<= 1) v += __shfl_xor(v, o, 64);
        y4[e] = v + b3;
    }
    wave_lds_sync();
}

size_t infer_smem(int Dp)
{
    return ((size_t)HID * (Dp + 8) + (size_t)HID * LDH + 4 * 2 * 16 * LDH) * sizeof(uint16_t) +
           (3 * HID + 4) * sizeof(float);
}

// inference: weights staged in LDS once per workgroup, then each wavefront takes tiles of
// 16 rows (grid-stride)
__global__ __launch_bounds__(256) void mlp_infer_kernel(const uint16_t *__restrict__ X, int64_t n, int Dp,
                                                        const uint16_t *__restrict__ wbf,
                                                        const float *__restrict__ params,
                                                        float *__restrict__ yhat)
{
    extern __shared__ uint16_t sh[];
    const int ldw1 = Dp + 8;
    uint16_t *W1t = sh;                                  // HID x ldw1
    uint16_t *W2t = W1t + (size_t)HID * ldw1;            // HID x LDH
    uint16_t *act = W2t + (size_t)HID * LDH;             // 4 waves x 2 x 16 x LDH
    float *fp = reinterpret_cast<float *>(act + 4 * 2 * 16 * LDH);   // b1 | b2 | w3 | b3
    for (int t = threadIdx.x; t < HID * Dp / 8; t += blockDim.x) {
        const int r = (t * 8) / Dp, k = (t * 8) - r * Dp;
        *reinterpret_cast<bf16x8 *>(W1t + r * ldw1 + k) = ld8(wbf + (size_t)t * 8);
    }
    const uint16_t *w2 = wbf + (size_t)HID * Dp;
    for (int t = threadIdx.x; t < HID * HID / 8; t += blockDim.x) {
        const int r = (t * 8) / HID, k = (t * 8) - r * HID;
        *reinterpret_cast<bf16x8 *>(W2t + r * LDH + k) = ld8(w2 + (size_t)t * 8);
    }
    for (int t = threadIdx.x; t < 3 * HID + 1; t += blockDim.x) {
        const int64_t src = t < HID ? off_b1(Dp) + t
                            : t < 2 * HID ? off_b2(Dp) + (t - HID)
                            : t < 3 * HID ? off_w3(Dp) + (t - 2 * HID) : off_b3(Dp);
        fp[t] = params[src];
    }
    __syncthreads();
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    uint16_t *h1s = act + (size_t)wv * 2 * 16 * LDH, *h2s = h1s + 16 * LDH;
    const int64_t ntile = (n + 15) / 16;
    for (int64_t tile = (int64_t)blockIdx.x * 4 + wv; tile < ntile; tile += (int64_t)gridDim.x * 4) {
        const int64_t r0 = tile * 16;
        const int nr = n - r0 < 16 ? (int)(n - r0) : 16;
        float y4[4];
        mlp_fwd16(X + r0 * Dp, Dp, nr, Dp, W1t, ldw1, fp, W2t, LDH, fp + HID, fp + 2 * HID, fp[3 * HID], h1s,
                  h2s, y4);
        if ((lane & 15) == 0) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int r = 4 * (lane >> 4) + e;
                if (r < nr) yhat[r0 + r] = y4[e];
            }
        }
    }
}

size_t grad_smem(int Dp)
{
    return ((size_t)64 * (Dp + 8) + 4 * 64 * LDH) * sizeof(uint16_t) + (64 + 4) * sizeof(float);
}

// Forward and backward of 64 rows per workgroup (4 wavefronts x 16 rows).  rows[] maps the
// batch to rows of X / tgt (nX rows); batch slots past nrows, row indices outside [0, nX)
// and NaN targets carry zero loss weight.  Each
// workgroup writes its own gradient partial (nparams values + the sum of squared errors),
// reduced later in a fixed order, so a step is deterministic.
__global__ __launch_bounds__(256) void mlp_grad_kernel(const uint16_t *__restrict__ X, int64_t nX,
                                                       const float *__restrict__ tgt,
                                                       const int32_t *__restrict__ rows, int64_t nrows,
                                                       int Dp, const uint16_t *__restrict__ wbf,
                                                       const float *__restrict__ params, float inv_batch,
                                                       float *__restrict__ partial)
{
    extern __shared__ uint16_t sh[];
    const int ldx = Dp + 8;
    uint16_t *Xs = sh;                                   // 64 x ldx
    uint16_t *H1 = Xs + 64 * ldx;                        // 64 x LDH
    uint16_t *H2 = H1 + 64 * LDH;
    uint16_t *D2 = H2 + 64 * LDH;                        // dL/dh2pre
    uint16_t *D1 = D2 + 64 * LDH;                        // dL/dh1pre
    float *dy = reinterpret_cast<float *>(D1 + 64 * LDH);   // 64
    float *red = dy + 64;                                    // 4
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, r16 = lane & 15, g = lane >> 4;
    const int64_t row0 = (int64_t)blockIdx.x * 64;
    const uint16_t *W1t = wbf, *W2t = wbf + (size_t)HID * Dp, *W2n = W2t + HID * HID;
    const float *b1 = params + off_b1(Dp), *b2 = params + off_b2(Dp), *w3 = params + off_w3(Dp);
    const float b3 = params[off_b3(Dp)];
    for (int t = threadIdx.x; t < 64 * Dp / 8; t += blockDim.x) {
        const int r = (t * 8) / Dp, k = (t * 8) - r * Dp;
        bf16x8 v;
        const int64_t xr = row0 + r < nrows ? (int64_t)rows[row0 + r] : -1;
        if (xr >= 0 && xr < nX) {
            v = ld8(X + (size_t)xr * Dp + k);
        } else {
#pragma unroll
            for (int q = 0; q < 8; ++q) v[q] = (__bf16)0.f;
        }
        *reinterpret_cast<bf16x8 *>(Xs + r * ldx + k) = v;
    }
    __syncthreads();
    float y4[4];
    mlp_fwd16(Xs + (size_t)(16 * wv) * ldx, ldx, 16, Dp, W1t, Dp, b1, W2t, HID, b2, w3, b3, H1 + 16 * wv * LDH,
              H2 + 16 * wv * LDH, y4);
    float lossp = 0.f;
    if (r16 == 0) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int r = 16 * wv + 4 * g + e;
            const int64_t gr = row0 + r;
            float d = 0.f;
            const int64_t xr = gr < nrows ? (int64_t)rows[gr] : -1;
            if (xr >= 0 && xr < nX) {
                const float t = tgt[xr];
                if (!__builtin_isnan(t)) {
                    const float diff = y4[e] - t;
                    lossp += diff * diff;
                    d = 2.f * diff * inv_batch;
                }
            }
            dy[r] = d;
        }
    }
    __syncthreads();
    // dL/dh2pre = dy w3 where h2 > 0
    for (int t = threadIdx.x; t < 64 * HID; t += blockDim.x) {
        const int r = t / HID, c = t - r * HID;
        D2[r * LDH + c] = bf16_bits(bf16_val(H2[r * LDH + c]) > 0.f ? dy[r] * w3[c] : 0.f);
    }
    __syncthreads();
    // dL/dh1pre = (D2 W2^T) where h1 > 0; operand B[k = out][col = in] = W2n[in][out]
    {
        f32x4 acc[8];
#pragma unroll
        for (int jt = 0; jt < 8; ++jt) acc[jt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int k0 = 0; k0 < HID; k0 += 32) {
            const bf16x8 a = ld8(D2 + (16 * wv + r16) * LDH + k0 + 8 * g);
#pragma unroll
            for (int jt = 0; jt < 8; ++jt)
                acc[jt] = mfma(a, ld8(W2n + (size_t)(16 * jt + r16) * HID + k0 + 8 * g), acc[jt]);
        }
#pragma unroll
        for (int jt = 0; jt < 8; ++jt)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int row = 16 * wv + 4 * g + e, col = 16 * jt + r16;
                D1[row * LDH + col] = bf16_bits(bf16_val(H1[row * LDH + col]) > 0.f ? acc[jt][e] : 0.f);
            }
    }
    __syncthreads();
    float *out = partial + (size_t)blockIdx.x * (mlp_nparams(Dp) + 4);
    // dW2 = H1^T D2 (128 x 128, K = 64 rows), 16 output tiles per wavefront
    for (int tt = 0; tt < 16; ++tt) {
        const int tile = wv * 16 + tt, it = tile >> 3, jt = tile & 7;
        f32x4 acc = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int k0 = 0; k0 < 64; k0 += 32)
            acc = mfma(ld8s(H1 + (k0 + 8 * g) * LDH + 16 * it + r16, LDH),
                       ld8s(D2 + (k0 + 8 * g) * LDH + 16 * jt + r16, LDH), acc);
#pragma unroll
        for (int e = 0; e < 4; ++e) out[off_W2(Dp) + (16 * it + 4 * g + e) * HID + 16 * jt + r16] = acc[e];
    }
    // dW1 = X^T D1 (Dp x 128, K = 64 rows)
    const int nt1 = (Dp / 16) * 8;
    for (int tile = wv; tile < nt1; tile += 4) {
        const int it = tile >> 3, jt = tile & 7;
        f32x4 acc = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int k0 = 0; k0 < 64; k0 += 32)
            acc = mfma(ld8s(Xs + (k0 + 8 * g) * ldx + 16 * it + r16, ldx),
                       ld8s(D1 + (k0 + 8 * g) * LDH + 16 * jt + r16, LDH), acc);
#pragma unroll
        for (int e = 0; e < 4; ++e) out[(size_t)(16 * it + 4 * g + e) * HID + 16 * jt + r16] = acc[e];
    }
    // bias and output-layer gradients: column sums over the 64 rows in a fixed order
    for (int c = threadIdx.x; c < HID; c += blockDim.x) {
        float s1 = 0.f, s2 = 0.f, s3 = 0.f;
        for (int r = 0; r < 64; ++r) {
            s1 += bf16_val(D1[r * LDH + c]);
            s2 += bf16_val(D2[r * LDH + c]);
            s3 += bf16_val(H2[r * LDH + c]) * dy[r];
        }
        out[off_b1(Dp) + c] = s1;
        out[off_b2(Dp) + c] = s2;
        out[off_w3(Dp) + c] = s3;
    }
    for (int o = 1; o < 64; o <<= 1) lossp += __shfl_xor(lossp, o, 64);
    if (lane == 0) red[wv] = lossp;
    __syncthreads();
    if (threadIdx.x == 0) {
        float sdy = 0.f;
        for (int r = 0; r < 64; ++r) sdy += dy[r];
        out[off_b3(Dp)] = sdy;
        out[off_b3(Dp) + 1] = 0.f;
        out[off_b3(Dp) + 2] = 0.f;
        out[off_b3(Dp) + 3] = 0.f;
        out[mlp_nparams(Dp)] = (red[0] + red[1]) + (red[2] + red[3]);
    }
}

// Total over the nwg gradient partials of element i = 64 blockIdx.x + (threadIdx.x & 63),
// in a fixed order: wavefront g sums the partials w = g, g + 4, ... in sequence, then the
// four sums are combined as (s0 + s1) + (s2 + s3).  Blocks of 256 threads; the result is
// returned to the first wavefront (false elsewhere and past np).
__device__ inline bool partial_total(const float *__restrict__ part, int nwg, int64_t np, float *red, float *total,
                                     int64_t *index)
{
    const int g = threadIdx.x >> 6, j = threadIdx.x & 63;
    const int64_t i = (int64_t)blockIdx.x * 64 + j, stride = np + 4;
    float s = 0.f;
    if (i <= np) {
#pragma unroll 8
        for (int w = g; w < nwg; w += 4) s += part[(size_t)w * stride + i];
    }
    red[g * 64 + j] = s;
    __syncthreads();
    if (g != 0 || i > np) return false;
    *total = (red[j] + red[64 + j]) + (red[128 + j] + red[192 + j]);
    *index = i;
    return true;
}

// grad[i] for i < nparams, grad[nparams] = mean loss
__global__ __launch_bounds__(256) void grad_sum_kernel(const float *__restrict__ part, int nwg, int Dp,
                                                       float inv_batch, float *__restrict__ grad)
{
    __shared__ float red[256];
    const int64_t np = mlp_nparams(Dp);
    float gs;
    int64_t i;
    if (partial_total(part, nwg, np, red, &gs, &i)) grad[i] = i == np ? gs * inv_batch : gs;
}

__device__ __forceinline__ void store_bf16_copy(int64_t i, float w, int Dp, uint16_t *wbf)
{
    if (i < off_b1(Dp)) {
        const int64_t k = i / HID, j = i - k * HID;
        wbf[j * Dp + k] = bf16_bits(w);
    } else if (i >= off_W2(Dp) && i < off_b2(Dp)) {
        const int64_t q = i - off_W2(Dp), in = q / HID, o = q - in * HID;
        wbf[(int64_t)HID * Dp + o * HID + in] = bf16_bits(w);
        wbf[(int64_t)HID * Dp + HID * HID + in * HID + o] = bf16_bits(w);
    }
}

// Adam (Kingma and Ba 2015, Algorithm 1: beta1 0.9, beta2 0.999, eps 1e-8) on the FP32
// master weights from the fixed-order total of the partials; refreshes the BF16 copies.
__global__ __launch_bounds__(256) void mlp_adam_kernel(const float *__restrict__ part, int nwg, int Dp,
                                                       float *__restrict__ params, float *__restrict__ m,
                                                       float *__restrict__ v, uint16_t *__restrict__ wbf,
                                                       float lr, float b1c, float b2c, float inv_batch,
                                                       float *__restrict__ loss_out)
{
    __shared__ float red[256];
    const int64_t np = mlp_nparams(Dp);
    float gs;
    int64_t i;
    if (!partial_total(part, nwg, np, red, &gs, &i)) return;
    if (i == np) {
        if (loss_out) loss_out[0] = gs * inv_batch;
        return;
    }
    const float mi = 0.9f * m[i] + 0.1f * gs;
    const float vi = 0.999f * v[i] + 0.001f * gs * gs;
    m[i] = mi;
    v[i] = vi;
    const float w = params[i] - lr * (mi / b1c) / (sqrtf(vi / b2c) + 1e-8f);
    params[i] = w;
    store_bf16_copy(i, w, Dp, wbf);
}

__global__ __launch_bounds__(256) void mlp_sync_kernel(const float *__restrict__ params, int Dp, uint16_t *__restrict__ wbf)
{
    const int64_t n = off_b2(Dp);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        store_bf16_copy(i, params[i], Dp, wbf);
}

// ------------------------------------------------------------------------------------
// selection and error statistics
// ------------------------------------------------------------------------------------
// SplitMix64 output i of a stream started at `seed` (Steele, Lea and Flood, OOPSLA 2014):
// state = seed + (i + 1) * 0x9E3779B97F4A7C15, then the variant-13 finaliser.
__device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t i)
{
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Selection in three passes, so that the list is deterministic and sorted:
//  1. flags[i] = 1 when |yhat_i - log1p(tau)| <= band (NaN predictions count as inside)
//     | 2 when the top 32 bits of SplitMix64(seed, i) fall below audit_cut; block b covers
//     the contiguous range [b seg, (b + 1) seg) and stores its {flagged, band, audit} counts;
//  2. one block scans the per-block counts (exclusive offsets, totals into counts);
//  3. every block writes the indices of its flagged pixels in ascending order.
constexpr int kSelMaxBlocks = 4096;

__device__ inline unsigned block_sum_u32(unsigned v, unsigned *red)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    return (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ __launch_bounds__(256) void select_flags_kernel(const float *__restrict__ yhat, int64_t n,
                                                           const double *__restrict__ stats, double band,
                                                           uint64_t seed, uint32_t audit_cut, int64_t seg,
                                                           uint8_t *__restrict__ flags, unsigned *__restrict__ bcnt,
                                                           int upper)
{
    __shared__ unsigned red[4];
    const double tl = log1p(stats[3]);
    const int64_t b0 = (int64_t)blockIdx.x * seg, b1 = b0 + seg < n ? b0 + seg : n;
    unsigned cs = 0, cb = 0, ca = 0;
    for (int64_t i = b0 + threadIdx.x; i < b1; i += 256) {
        // the band |yhat - log1p(tau)| <= band, or with `upper` everything above its lower edge
        const double dv = (double)yhat[i] - tl;
        const bool in_band = upper ? !(dv < -band) : !(fabs(dv) > band);
        const bool audit = (uint32_t)(splitmix64_at(seed, (uint64_t)i) >> 32) < audit_cut;
        const unsigned f = (in_band ? 1u : 0u) | (audit ? 2u : 0u);
        flags[i] = (uint8_t)f;
        cs += f != 0u;
        cb += f & 1u;
        ca += f >> 1;
    }
    cs = block_sum_u32(cs, red);
    cb = block_sum_u32(cb, red);
    ca = block_sum_u32(ca, red);
    if (threadIdx.x == 0) {
        bcnt[3 * blockIdx.x] = cs;
        bcnt[3 * blockIdx.x + 1] = cb;
        bcnt[3 * blockIdx.x + 2] = ca;
    }
}

// one block of 1024 threads; nb <= 4096 (four per thread)
__global__ __launch_bounds__(1024) void select_scan_kernel(const unsigned *__restrict__ bcnt, int nb,
                                                           unsigned *__restrict__ boff, unsigned *__restrict__ counts)
{
    __shared__ unsigned sc[1024];
    __shared__ unsigned wtot[2][16];
    const int t = threadIdx.x;
    unsigned v[4], loc = 0, lb = 0, la = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int b = 4 * t + q;
        v[q] = b < nb ? bcnt[3 * b] : 0u;
        lb += b < nb ? bcnt[3 * b + 1] : 0u;
        la += b < nb ? bcnt[3 * b + 2] : 0u;
        loc += v[q];
    }
    // band and audit totals: wave sums, then the 16 wave totals (integer sums, any order)
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        lb += __shfl_down(lb, o, 64);
        la += __shfl_down(la, o, 64);
    }
    if ((t & 63) == 0) {
        wtot[0][t >> 6] = lb;
        wtot[1][t >> 6] = la;
    }
    sc[t] = loc;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {   // inclusive Hillis-Steele scan
        const unsigned add = t >= o ? sc[t - o] : 0u;
        __syncthreads();
        sc[t] += add;
        __syncthreads();
    }
    unsigned run = sc[t] - loc;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int b = 4 * t + q;
        if (b < nb) boff[b] = run;
        run += v[q];
    }
    if (t == 0) {
        unsigned tb = 0, ta = 0;
        for (int w = 0; w < 16; ++w) {
            tb += wtot[0][w];
            ta += wtot[1][w];
        }
        counts[0] = sc[1023];
        counts[1] = tb;
        counts[2] = ta;
    }
}

__global__ __launch_bounds__(256) void select_write_kernel(const uint8_t *__restrict__ flags, int64_t n, int64_t seg,
                                                           const unsigned *__restrict__ boff, int32_t *__restrict__ idx)
{
    __shared__ unsigned wsum[4];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t b0 = (int64_t)blockIdx.x * seg, b1 = b0 + seg < n ? b0 + seg : n;
    unsigned base = boff[blockIdx.x];
    for (int64_t s0 = b0; s0 < b1; s0 += 256) {
        const int64_t i = s0 + threadIdx.x;
        const bool f = i < b1 && flags[i] != 0;
        const uint64_t m = __ballot(f);
        if (lane == 0) wsum[wv] = (unsigned)__popcll(m);
        __syncthreads();
        unsigned pre = 0;
        for (int q = 0; q < wv; ++q) pre += wsum[q];
        if (f) idx[base + pre + (unsigned)__popcll(m & ((1ull << lane) - 1ull))] = (int32_t)i;
        base += (wsum[0] + wsum[1]) + (wsum[2] + wsum[3]);
        __syncthreads();
    }
}

__global__ void fill_u32_kernel(unsigned *p, int n, unsigned v)
{
    for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = v;
}

__global__ __launch_bounds__(256) void expm1_kernel(const float *__restrict__ y, int64_t n, float *__restrict__ s)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        s[i] = (float)expm1((double)y[i]);
}

// error e_i = yhat_i - r_i with r_i = log1p(ref_i) (ref_is_score) or ref_i, over the rows
// with (flags[i] & mask) != 0 (all rows when flags is NULL) and finite e: per block
// {count, sum e^2, max |e|}, merged by one thread in block order -> out {count, rmse, max}
__global__ __launch_bounds__(256) void err_partial_kernel(const float *__restrict__ yhat, const float *__restrict__ ref,
                                                          int ref_is_score, const uint8_t *__restrict__ flags,
                                                          int mask, int64_t n, double *__restrict__ part)
{
    __shared__ double r0[4], r1[4], r2[4];
    double c = 0.0, s = 0.0, mx = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        if (flags && !(flags[i] & mask)) continue;
        const double r = ref_is_score ? log1p((double)ref[i]) : (double)ref[i];
        const double e = (double)yhat[i] - r;
        if (!isfinite(e)) continue;
        c += 1.0;
        s += e * e;
        mx = fmax(mx, fabs(e));
    }
    for (int o = 32; o > 0; o >>= 1) {
        c += __shfl_xor(c, o);
        s += __shfl_xor(s, o);
        mx = fmax(mx, __shfl_xor(mx, o));
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        r0[w] = c;
        r1[w] = s;
        r2[w] = mx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        part[3 * blockIdx.x] = (r0[0] + r0[1]) + (r0[2] + r0[3]);
        part[3 * blockIdx.x + 1] = (r1[0] + r1[1]) + (r1[2] + r1[3]);
        part[3 * blockIdx.x + 2] = fmax(fmax(r2[0], r2[1]), fmax(r2[2], r2[3]));
    }
}

// one block of 256 threads: strided partial sums per thread, then a fixed tree (the same
// order on every run)
__global__ __launch_bounds__(256) void err_final_kernel(const double *__restrict__ part, int nb,
                                                        double *__restrict__ out)
{
    __shared__ double red[3][256];
    const int t = threadIdx.x;
    double c = 0.0, s = 0.0, mx = 0.0;
    for (int b = t; b < nb; b += 256) {
        c += part[3 * b];
        s += part[3 * b + 1];
        mx = fmax(mx, part[3 * b + 2]);
    }
    red[0][t] = c;
    red[1][t] = s;
    red[2][t] = mx;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (t < o) {
            red[0][t] += red[0][t + o];
            red[1][t] += red[1][t + o];
            red[2][t] = fmax(red[2][t], red[2][t + o]);
        }
        __syncthreads();
    }
    if (t == 0) {
        c = red[0][0];
        out[0] = c;
        out[1] = c > 0.0 ? sqrt(red[1][0] / c) : 0.0;
        out[2] = red[2][0];
    }
}

// Histogram of the audit's absolute prediction errors |yhat - log1p(score)| (log1p space) in
// kAuditBins bins of width 1 / kAuditBinsPerUnit (the last bin also takes everything beyond),
// and in hist[kAuditBins] the audited pixels whose predicted score and exact score fall on
// different sides of the predicted map's eq. (12) threshold (stats[3]).  Integer atomics,
// so the counts do not depend on the order.
static constexpr int kAuditBins = 4096;
static constexpr double kAuditBinsPerUnit = 256.0;

__global__ __launch_bounds__(256) void audit_hist_kernel(const float *__restrict__ yhat,
                                                         const float *__restrict__ scores,
                                                         const uint8_t *__restrict__ flags, int64_t n,
                                                         const double *__restrict__ stats, unsigned *__restrict__ hist)
{
    const double tau = stats[3], ltau = log1p(tau);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        if (!(flags[i] & 2)) continue;
        const double y = (double)yhat[i], sc = (double)scores[i];
        const double e = y - log1p(sc);
        if (!isfinite(e)) continue;
        const double b = fabs(e) * kAuditBinsPerUnit;
        const int bin = b >= (double)(kAuditBins - 1) ? kAuditBins - 1 : (int)b;
        atomicAdd(&hist[bin], 1u);
        if ((y > ltau) != (sc > tau)) atomicAdd(&hist[kAuditBins], 1u);
    }
}

// number of audited pixels (flags & 2) outside the second selection (flags2 == 0)
__global__ __launch_bounds__(256) void audit_outside_kernel(const uint8_t *__restrict__ flags,
                                                            const uint8_t *__restrict__ flags2, int64_t n,
                                                            unsigned *__restrict__ count)
{
    unsigned c = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        c += ((flags[i] & 2) && !flags2[i]) ? 1u : 0u;
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
    if ((threadIdx.x & 63) == 0 && c) atomicAdd(count, c);
}

int grid_for(int64_t n, int cap = 8192)
{
    int64_t g = (n + 255) / 256;
    return (int)(g < 1 ? 1 : g > cap ? cap : g);
}

bool bad_dp(int Dp) { return Dp < 32 || Dp % 32 != 0 || Dp > MAX_DP; }

int check_feature_windows(const char *fn, const hsad_window_params *p, int64_t H, int64_t W)
{
    if (!p) return fail(HSAD_EINVAL, std::string(fn) + ": params is NULL");
    if (p->outer < 1 || (p->outer & 1) == 0 || p->outer > HSAD_MAX_WINDOW || p->inner < 0 ||
        (p->inner > 0 && (p->inner & 1) == 0) || p->inner >= p->outer ||
        (p->inner > 0 && H <= p->inner && W <= p->inner))
        return fail(HSAD_EINVAL, std::string(fn) + ": bad windows (odd sizes, inner < outer, non-empty annulus)");
    return HSAD_OK;
}

int err_stats_launch(const float *yhat, const float *ref, int ref_is_score, const uint8_t *flags, int mask,
                     int64_t n, double *out, void *ws, hipStream_t s)
{
    const int nb = grid_for(n, 1024);
    hipLaunchKernelGGL(err_partial_kernel, dim3(nb), dim3(256), 0, s, yhat, ref, ref_is_score, flags, mask, n,
                       (double *)ws);
    hipLaunchKernelGGL(err_final_kernel, dim3(1), dim3(256), 0, s, (const double *)ws, nb, out);
    return check_launch("err_stats");
}

static int g_feat_cfg = 0;   // 0: 32-wide tiles where they fit; 1: 16-wide tiles (tests)

template <int FCC, int FTX>
static int features_go(const float *x, int64_t H, int64_t W, int64_t Lp, int R, int RI, int hi, const float *norm,
                       int Dp, float *feat, uint16_t *packed, hipStream_t s)
{
    const size_t sh = features_smem<FCC, FTX>(R);
    if (int rc = allow_lds((const void *)surr_features_kernel<FCC, FTX>, sh, "surr_features_kernel")) return rc;
    dim3 grid((unsigned)((W + FTX - 1) / FTX), (unsigned)((H + FTY - 1) / FTY));
    hipLaunchKernelGGL((surr_features_kernel<FCC, FTX>), grid, dim3(FTX * FTY), sh, s, x, (int)H, (int)W, (int)Lp, R,
                       RI, hi, norm, Dp, feat, packed);
    return check_launch("surr_features_kernel");
}

int features_launch(const float *x, int64_t H, int64_t W, int64_t Lp, const hsad_window_params *p,
                    const float *norm, int Dp, float *feat, uint16_t *packed, hipStream_t s)
{
    const int R = p->outer / 2, RI = p->inner / 2;
    const int hi = p->inner > 0 ? 1 : 0;
    // 32 x 16 tiles, four bands per chunk: fewer halo columns per pixel (measured at 2048^2,
    // 15 x 15 windows: L' = 56 7.8 -> 7.1 ms, L' = 14 unchanged; two-band chunks were slower)
    if (g_feat_cfg != 1 && Lp >= 4 && features_smem<4, 32>(R) <= 150 * 1024)
        return features_go<4, 32>(x, H, W, Lp, R, RI, hi, norm, Dp, feat, packed, s);
    if (features_smem<4, 16>(R) <= 64 * 1024 && Lp >= 4)
        return features_go<4, 16>(x, H, W, Lp, R, RI, hi, norm, Dp, feat, packed, s);
    if (features_smem<2, 16>(R) <= 64 * 1024 && Lp >= 2)
        return features_go<2, 16>(x, H, W, Lp, R, RI, hi, norm, Dp, feat, packed, s);
    return features_go<1, 16>(x, H, W, Lp, R, RI, hi, norm, Dp, feat, packed, s);
}

int infer_launch(const uint16_t *X, int64_t n, int Dp, const float *params, const uint16_t *wbf, float *yhat,
                 hipStream_t s)
{
    const size_t sh = infer_smem(Dp);
    if (int rc = allow_lds((const void *)mlp_infer_kernel, sh, "mlp_infer_kernel")) return rc;
    const int64_t tiles = (n + 15) / 16;
    int64_t grid = (tiles + 3) / 4;
    if (grid > 256 * 4) grid = 256 * 4;
    hipLaunchKernelGGL(mlp_infer_kernel, dim3((unsigned)grid), dim3(256), sh, s, X, n, Dp, wbf, params, yhat);
    return check_launch("mlp_infer_kernel");
}

struct RunLayout {
    size_t X, yhat, flags, idx, small, gen, total;
};

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

RunLayout run_layout(int64_t H, int64_t W, int64_t Lp, int Dp, const hsad_window_params *p)
{
    const int64_t n = H * W;
    RunLayout L{};
    size_t o = 0;
    L.X = o;
    o = align256(o + (size_t)n * Dp * sizeof(uint16_t));
    L.yhat = o;
    o = align256(o + (size_t)n * sizeof(float));
    L.flags = o;
    o = align256(o + (size_t)n);
    L.idx = o;
    o = align256(o + (size_t)n * sizeof(int32_t));
    // counts (4 u32, 64 B) | predicted-map stats (4) | final stats (4) | audit (4) doubles,
    // then the threshold / error-statistics workspace
    L.small = o;
    o = align256(o + 256 + std::max({hsad_threshold_workspace_bytes(n), (size_t)3 * 1024 * sizeof(double),
                                     (size_t)kSelMaxBlocks * 4 * sizeof(unsigned),
                                     (size_t)(kAuditBins + 1) * sizeof(unsigned)}));
    L.gen = o;
    size_t g = hsad_workspace_bytes(HSAD_OP_LRX, H, W, Lp, p);
    g = std::max(g, generic_ws_per_pixel(Lp, GRAM_LRX) * (size_t)std::min<int64_t>(n, 8192));
    L.total = align256(o + g);
    return L;
}

}  // namespace

}  // namespace hsad

using namespace hsad;

extern "C" {

int hsad_mlp_dims(int64_t Lp, int32_t *D, int32_t *Dp, int64_t *nparams, int64_t *nbf16)
{
    clear_error();
    if (Lp < 1 || 3 * Lp > MAX_DP) return fail(HSAD_EINVAL, "hsad_mlp_dims: L' must be 1..85");
    const int d = (int)(3 * Lp), dp = (d + 31) / 32 * 32;
    if (D) *D = d;
    if (Dp) *Dp = dp;
    if (nparams) *nparams = mlp_nparams(dp);
    if (nbf16) *nbf16 = mlp_nbf16(dp);
    return HSAD_OK;
}

int hsad_surrogate_features(const float *x, int64_t H, int64_t W, int64_t Lp, const hsad_window_params *p,
                            const float *norm, int32_t Dp, float *feat, uint16_t *packed, hipStream_t stream)
{
    clear_error();
    if (!x || H < 1 || W < 1 || Lp < 1 || 3 * Lp > MAX_DP || H * W > ((int64_t)1 << 31) - 1)
        return fail(HSAD_EINVAL, "hsad_surrogate_features: bad cube");
    if (int rc = check_feature_windows("hsad_surrogate_features", p, H, W)) return rc;
    if (norm ? (!packed || bad_dp(Dp) || Dp < 3 * Lp) : !feat)
        return fail(HSAD_EINVAL, "hsad_surrogate_features: need feat (norm NULL) or packed with Dp >= 3 L'");
    return features_launch(x, H, W, Lp, p, norm, Dp, feat, packed, stream);
}

int hsad_mlp_norm_stats(const float *feat, int64_t n, int32_t D, float *norm, hipStream_t stream)
{
    clear_error();
    if (!feat || !norm || n < 1 || D < 1 || D > MAX_DP) return fail(HSAD_EINVAL, "hsad_mlp_norm_stats: bad arguments");
    hipLaunchKernelGGL(norm_stats_kernel, dim3(D), dim3(256), 0, stream, feat, n, D, norm);
    return check_launch("norm_stats_kernel");
}

int hsad_mlp_pack(const float *feat, int64_t n, int32_t D, int32_t Dp, const float *norm, uint16_t *out,
                  hipStream_t stream)
{
    clear_error();
    if (!feat || !norm || !out || n < 1 || D < 1 || bad_dp(Dp) || Dp < D)
        return fail(HSAD_EINVAL, "hsad_mlp_pack: bad arguments");
    hipLaunchKernelGGL(mlp_pack_kernel, dim3(grid_for(n * Dp)), dim3(256), 0, stream, feat, n, D, Dp, norm, out);
    return check_launch("mlp_pack_kernel");
}

int hsad_surrogate_targets(const float *scores, int64_t n, float *tgt, hipStream_t stream)
{
    clear_error();
    if (!scores || !tgt || n < 1) return fail(HSAD_EINVAL, "hsad_surrogate_targets: bad arguments");
    hipLaunchKernelGGL(targets_kernel, dim3(grid_for(n)), dim3(256), 0, stream, scores, n, tgt);
    return check_launch("targets_kernel");
}

int hsad_mlp_sync(const float *params, int32_t Dp, uint16_t *wbf, hipStream_t stream)
{
    clear_error();
    if (!params || !wbf || bad_dp(Dp)) return fail(HSAD_EINVAL, "hsad_mlp_sync: bad arguments");
    hipLaunchKernelGGL(mlp_sync_kernel, dim3(grid_for(off_b2(Dp))), dim3(256), 0, stream, params, Dp, wbf);
    return check_launch("mlp_sync_kernel");
}

int hsad_mlp_infer(const uint16_t *X, int64_t n, int32_t Dp, const float *params, const uint16_t *wbf,
                   float *yhat, hipStream_t stream)
{
    clear_error();
    if (!X || !params || !wbf || !yhat || n < 1 || bad_dp(Dp)) return fail(HSAD_EINVAL, "hsad_mlp_infer: bad arguments");
    return infer_launch(X, n, Dp, params, wbf, yhat, stream);
}

size_t hsad_mlp_train_workspace_bytes(int64_t batch, int32_t Dp)
{
    if (batch < 1 || bad_dp(Dp)) return 0;
    return (size_t)((batch + 63) / 64) * (size_t)(mlp_nparams(Dp) + 4) * sizeof(float);
}

static int grad_common(const char *fn, const uint16_t *X, int64_t nX, const float *tgt, const int32_t *rows,
                       int64_t batch, int32_t Dp, const float *params, const uint16_t *wbf, void *ws,
                       size_t ws_bytes, hipStream_t s)
{
    if (!X || nX < 1 || !tgt || !rows || !params || !wbf || batch < 1 || batch > ((int64_t)1 << 30) || bad_dp(Dp))
        return fail(HSAD_EINVAL, std::string(fn) + ": bad arguments");
    if (!ws || ws_bytes < hsad_mlp_train_workspace_bytes(batch, Dp))
        return fail(HSAD_ENOMEM, std::string(fn) + ": workspace too small (see hsad_mlp_train_workspace_bytes)");
    const size_t sh = grad_smem(Dp);
    if (int rc = allow_lds((const void *)mlp_grad_kernel, sh, "mlp_grad_kernel")) return rc;
    hipLaunchKernelGGL(mlp_grad_kernel, dim3((unsigned)((batch + 63) / 64)), dim3(256), sh, s, X, nX, tgt, rows,
                       batch, Dp, wbf, params, 1.0f / (float)batch, (float *)ws);
    return check_launch("mlp_grad_kernel");
}

int hsad_mlp_gradient(const uint16_t *X, int64_t nX, const float *tgt, const int32_t *rows, int64_t batch,
                      int32_t Dp, const float *params, const uint16_t *wbf, float *grad, void *ws, size_t ws_bytes,
                      hipStream_t stream)
{
    clear_error();
    if (!grad) return fail(HSAD_EINVAL, "hsad_mlp_gradient: grad is NULL");
    if (int rc = grad_common("hsad_mlp_gradient", X, nX, tgt, rows, batch, Dp, params, wbf, ws, ws_bytes, stream))
        return rc;
    const int nwg = (int)((batch + 63) / 64);
    hipLaunchKernelGGL(grad_sum_kernel, dim3((unsigned)((mlp_nparams(Dp) + 64) / 64)), dim3(256), 0, stream,
                       (const float *)ws, nwg, Dp, 1.0f / (float)batch, grad);
    return check_launch("grad_sum_kernel");
}

int hsad_mlp_train_step(const uint16_t *X, int64_t nX, const float *tgt, const int32_t *rows, int64_t batch,
                        int32_t Dp, float *params, uint16_t *wbf, float *adam_m, float *adam_v, int64_t step,
                        float lr, float *loss, void *ws, size_t ws_bytes, hipStream_t stream)
{
    clear_error();
    if (!adam_m || !adam_v || step < 1 || !(lr >= 0.f)) return fail(HSAD_EINVAL, "hsad_mlp_train_step: bad arguments");
    if (int rc = grad_common("hsad_mlp_train_step", X, nX, tgt, rows, batch, Dp, params, wbf, ws, ws_bytes, stream))
        return rc;
    const int nwg = (int)((batch + 63) / 64);
    const float b1c = (float)(1.0 - std::pow(0.9, (double)step)), b2c = (float)(1.0 - std::pow(0.999, (double)step));
    hipLaunchKernelGGL(mlp_adam_kernel, dim3((unsigned)((mlp_nparams(Dp) + 64) / 64)), dim3(256), 0, stream,
                       (const float *)ws, nwg, Dp, params, adam_m, adam_v, wbf, lr, b1c, b2c,
                       1.0f / (float)batch, loss);
    return check_launch("mlp_adam_kernel");
}

size_t hsad_error_stats_workspace_bytes(int64_t n)
{
    (void)n;
    return 3 * 1024 * sizeof(double);
}

int hsad_error_stats(const float *yhat, const float *ref, int32_t ref_is_score, const uint8_t *flags,
                     int32_t flag_mask, int64_t n, double *out, void *ws, size_t ws_bytes, hipStream_t stream)
{
    clear_error();
    if (!yhat || !ref || !out || n < 1) return fail(HSAD_EINVAL, "hsad_error_stats: bad arguments");
    if (!ws || ws_bytes < hsad_error_stats_workspace_bytes(n)) return fail(HSAD_ENOMEM, "hsad_error_stats: workspace");
    return err_stats_launch(yhat, ref, ref_is_score, flags, flag_mask, n, out, ws, stream);
}

size_t hsad_surrogate_select_workspace_bytes(int64_t n)
{
    (void)n;
    return (size_t)kSelMaxBlocks * 4 * sizeof(unsigned);
}

static int select_common(const float *yhat, int64_t n, const double *stats, double band, uint64_t seed,
                         double audit_frac, uint8_t *flags, int32_t *idx, uint32_t *counts, void *ws,
                         size_t ws_bytes, hipStream_t stream, int upper);

int hsad_surrogate_select(const float *yhat, int64_t n, const double *stats, double band, uint64_t seed,
                          double audit_frac, uint8_t *flags, int32_t *idx, uint32_t *counts, void *ws,
                          size_t ws_bytes, hipStream_t stream)
{
    return select_common(yhat, n, stats, band, seed, audit_frac, flags, idx, counts, ws, ws_bytes, stream, 0);
}

static int select_common(const float *yhat, int64_t n, const double *stats, double band, uint64_t seed,
                         double audit_frac, uint8_t *flags, int32_t *idx, uint32_t *counts, void *ws,
                         size_t ws_bytes, hipStream_t stream, int upper)
{
    clear_error();
    if (!yhat || !stats || !flags || !idx || !counts || n < 1 || n > ((int64_t)1 << 31) - 1 || !(band >= 0.0) ||
        !(audit_frac >= 0.0 && audit_frac <= 1.0))
        return fail(HSAD_EINVAL, "hsad_surrogate_select: bad arguments");
    if (!ws || ws_bytes < hsad_surrogate_select_workspace_bytes(n))
        return fail(HSAD_ENOMEM, "hsad_surrogate_select: workspace too small");
    const double cut = std::ldexp(audit_frac, 32);
    const uint32_t audit_cut = cut >= 4294967295.0 ? 0xffffffffu : (uint32_t)cut;
    int64_t nb = (n + 255) / 256;
    if (nb > kSelMaxBlocks) nb = kSelMaxBlocks;
    int64_t seg = (n + nb - 1) / nb;
    seg = (seg + 255) / 256 * 256;
    nb = (n + seg - 1) / seg;
    unsigned *bcnt = (unsigned *)ws, *boff = bcnt + 3 * kSelMaxBlocks;
    hipLaunchKernelGGL(select_flags_kernel, dim3((unsigned)nb), dim3(256), 0, stream, yhat, n, stats, band, seed,
                       audit_cut, seg, flags, bcnt, upper);
    hipLaunchKernelGGL(select_scan_kernel, dim3(1), dim3(1024), 0, stream, (const unsigned *)bcnt, (int)nb, boff,
                       (unsigned *)counts);
    hipLaunchKernelGGL(select_write_kernel, dim3((unsigned)nb), dim3(256), 0, stream, flags, n, seg,
                       (const unsigned *)boff, idx);
    return check_launch("hsad_surrogate_select");
}

int hsad_lrx_dwrx_at(const float *x, int64_t H, int64_t W, int64_t Lp, const hsad_window_params *p,
                     const int32_t *idx, int64_t nidx, float *lrx, float *dwrx, void *ws, size_t ws_bytes,
                     hipStream_t stream)
{
    clear_error();
    if (!x || !idx || nidx < 0 || (!lrx && !dwrx) || H < 1 || W < 1 || Lp < 1 || Lp > HSAD_MAX_LP ||
        H * W > ((int64_t)1 << 31) - 1)
        return fail(HSAD_EINVAL, "hsad_lrx_dwrx_at: bad arguments");
    if (int rc = check_feature_windows("hsad_lrx_dwrx_at", p, H, W)) return rc;
    if (!(p->load_rel >= 0.0) || (dwrx && p->inner < 1) ||
        (p->precision != HSAD_PREC_AUTO && p->precision != HSAD_PREC_FP64))
        return fail(HSAD_EINVAL, "hsad_lrx_dwrx_at: load_rel >= 0, DWRX needs inner >= 1, precision AUTO/FP64");
    if (nidx == 0) return HSAD_OK;
    if (!ws || ws_bytes < generic_ws_per_pixel(Lp, GRAM_LRX))
        return fail(HSAD_ENOMEM, "hsad_lrx_dwrx_at: workspace too small (one pixel needs (L'+2) L' doubles)");
    Windows w{p->inner, p->outer, p->inner / 2, p->outer / 2};
    return generic_lrx_dwrx_at(x, H, W, Lp, w, p->load_rel, GP_FP64, idx, nidx, lrx, dwrx, ws, ws_bytes, stream);
}

size_t hsad_surrogate_workspace_bytes(int64_t H, int64_t W, int64_t Lp, int32_t Dp, const hsad_window_params *p)
{
    if (H < 1 || W < 1 || Lp < 1 || bad_dp(Dp) || !p) return 0;
    return run_layout(H, W, Lp, Dp, p).total;
}

int hsad_surrogate_run(const float *x, int64_t H, int64_t W, int64_t Lp, const hsad_window_params *p,
                       const hsad_mlp_model *model, const hsad_surrogate_options *opt, float *scores,
                       uint8_t *mask, hsad_surrogate_report *rep, void *ws, size_t ws_bytes, hipStream_t stream)
{
    clear_error();
    if (!x || !model || !opt || !scores || !rep || H < 1 || W < 1 || Lp < 1 || H * W > ((int64_t)1 << 31) - 1)
        return fail(HSAD_EINVAL, "hsad_surrogate_run: bad arguments");
    if (int rc = check_feature_windows("hsad_surrogate_run", p, H, W)) return rc;
    if (!model->params || !model->wbf || !model->norm || model->Lp != Lp || bad_dp(model->Dp) ||
        model->Dp < 3 * Lp || !(model->rmse_val >= 0.0))
        return fail(HSAD_EINVAL, "hsad_surrogate_run: model does not match the cube (L', Dp, pointers, rmse_val)");
    if (!(opt->band_k >= 0.0) || !(opt->audit_frac >= 0.0 && opt->audit_frac <= 1.0) ||
        !std::isfinite(opt->z_alpha) || !(opt->fallback_factor > 0.0) ||
        !(opt->band_quantile >= 0.0 && opt->band_quantile < 1.0) ||
        !(opt->max_exact_frac > 0.0 && opt->max_exact_frac <= 1.0) || opt->reserved != 0)
        return fail(HSAD_EINVAL, "hsad_surrogate_run: bad options");
    if (p->precision != HSAD_PREC_AUTO && p->precision != HSAD_PREC_FP64)
        return fail(HSAD_EINVAL, "hsad_surrogate_run: exact recomputation needs precision AUTO/FP64");
    const RunLayout L = run_layout(H, W, Lp, model->Dp, p);
    if (!ws || ws_bytes < L.total)
        return fail(HSAD_ENOMEM, "hsad_surrogate_run: workspace too small (see hsad_surrogate_workspace_bytes)");
    const int64_t n = H * W;
    char *b = (char *)ws;
    uint16_t *X = (uint16_t *)(b + L.X);
    float *yhat = (float *)(b + L.yhat);
    uint8_t *flags = (uint8_t *)(b + L.flags);
    int32_t *idx = (int32_t *)(b + L.idx);
    uint32_t *counts = (uint32_t *)(b + L.small);
    double *dev_stats = (double *)(b + L.small + 64);   // pred[4] | final[4] | audit[4]
    void *ws_small = b + L.small + 256;
    const size_t ws_small_bytes = L.gen - L.small - 256;
    void *ws_gen = b + L.gen;
    const size_t ws_gen_bytes = L.total - L.gen;
    int rc;
    // features -> normalised BF16 rows -> predictions; predicted scores and their eq. (12) tau
    if ((rc = features_launch(x, H, W, Lp, p, model->norm, model->Dp, nullptr, X, stream))) return rc;
    if ((rc = infer_launch(X, n, model->Dp, model->params, model->wbf, yhat, stream))) return rc;
    hipLaunchKernelGGL(expm1_kernel, dim3(grid_for(n)), dim3(256), 0, stream, yhat, n, scores);
    if ((rc = hsad_threshold(scores, n, opt->z_alpha, dev_stats, nullptr, ws_small, ws_small_bytes, stream)))
        return rc;
    // near-threshold band + audit sample, then exact LRX there (overwrites those pixels)
    if ((rc = select_common(yhat, n, dev_stats, opt->band_k * model->rmse_val, opt->seed, opt->audit_frac, flags, idx,
                            counts, ws_small, ws_small_bytes, stream, opt->exact_above ? 1 : 0)))
        return rc;
    uint32_t hc[3] = {0, 0, 0};
    if (hipMemcpyAsync(hc, counts, sizeof(hc), hipMemcpyDeviceToHost, stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess)
        return fail(HSAD_EHIP, "hsad_surrogate_run: reading the selection counts failed");
    if (hc[0] > 0 &&
        (rc = hsad_lrx_dwrx_at(x, H, W, Lp, p, idx, hc[0], scores, nullptr, ws_gen, ws_gen_bytes, stream)))
        return rc;
    // audit: prediction error against the exact score on the audited pixels (log1p space)
    if ((rc = err_stats_launch(yhat, scores, 1, flags, 2, n, dev_stats + 8, ws_small, stream))) return rc;
    double hs[12];
    if (hipMemcpyAsync(hs, dev_stats, 12 * sizeof(double), hipMemcpyDeviceToHost, stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess)
        return fail(HSAD_EHIP, "hsad_surrogate_run: reading the audit failed");
    const double *audit = hs + 8;
    int fallback = (audit[0] > 0.0 && !(audit[1] <= opt->fallback_factor * model->rmse_val)) ? 1 : 0;
    // the audit's error tail and mask flips: the band widens to the band_quantile quantile of
    // the audited |error| (when that exceeds band_k * rmse_val), and the pixels of the wider
    // band are recomputed exactly as well
    double band = opt->band_k * model->rmse_val;
    int64_t flips = 0, band_count = hc[1], selected = hc[0];
    if (!fallback && hc[2] > 0) {
        unsigned *hist = (unsigned *)ws_small;
        hipLaunchKernelGGL(fill_u32_kernel, dim3(1), dim3(256), 0, stream, hist, kAuditBins + 1, 0u);
        hipLaunchKernelGGL(audit_hist_kernel, dim3(grid_for(n)), dim3(256), 0, stream, yhat, scores, flags, n,
                           (const double *)dev_stats, hist);
        if ((rc = check_launch("audit_hist_kernel"))) return rc;
        std::vector<unsigned> hh(kAuditBins + 1);
        if (hipMemcpyAsync(hh.data(), hist, hh.size() * sizeof(unsigned), hipMemcpyDeviceToHost, stream) !=
                hipSuccess ||
            hipStreamSynchronize(stream) != hipSuccess)
            return fail(HSAD_EHIP, "hsad_surrogate_run: reading the audit histogram failed");
        flips = hh[kAuditBins];
        if (opt->band_quantile > 0.0) {
            uint64_t tot = 0;
            for (int b = 0; b < kAuditBins; ++b) tot += hh[b];
            const double want = opt->band_quantile * (double)tot;
            uint64_t cum = 0;
            int qb = kAuditBins - 1;
            for (int b = 0; b < kAuditBins; ++b) {
                cum += hh[b];
                if ((double)cum >= want) {
                    qb = b;
                    break;
                }
            }
            const double qw = (double)(qb + 1) / kAuditBinsPerUnit;   // upper edge of the quantile's bin
            if (qw > band) {
                band = qw;
                // the feature rows are no longer needed: their space holds the second
                // selection's flags and indices
                uint8_t *flags2 = (uint8_t *)X;
                int32_t *idx2 = (int32_t *)((char *)X + align256((size_t)n));
                if ((rc = select_common(yhat, n, dev_stats, band, opt->seed, 0.0, flags2, idx2, counts, ws_small,
                                        ws_small_bytes, stream, opt->exact_above ? 1 : 0)))
                    return rc;
                hipLaunchKernelGGL(fill_u32_kernel, dim3(1), dim3(64), 0, stream, counts + 3, 1, 0u);
                hipLaunchKernelGGL(audit_outside_kernel, dim3(grid_for(n, 1024)), dim3(256), 0, stream,
                                   (const uint8_t *)flags, (const uint8_t *)flags2, n, counts + 3);
                if ((rc = check_launch("audit_outside_kernel"))) return rc;
                uint32_t h2[4] = {0, 0, 0, 0};
                if (hipMemcpyAsync(h2, counts, sizeof(h2), hipMemcpyDeviceToHost, stream) != hipSuccess ||
                    hipStreamSynchronize(stream) != hipSuccess)
                    return fail(HSAD_EHIP, "hsad_surrogate_run: reading the selection counts failed");
                band_count = h2[1];
                selected = (int64_t)h2[0] + (int64_t)h2[3];   // the wider band, plus the audit outside it
                if ((double)selected > opt->max_exact_frac * (double)n) {
                    fallback = 1;
                } else if (h2[0] > 0 && (rc = hsad_lrx_dwrx_at(x, H, W, Lp, p, idx2, h2[0], scores, nullptr, ws_gen,
                                                               ws_gen_bytes, stream))) {
                    return rc;
                }
            }
        }
    }
    if (fallback && (rc = hsad_lrx(x, H, W, Lp, p, scores, ws_gen, ws_gen_bytes, stream))) return rc;
    // eq. (12) threshold and mask of the final map
    if ((rc = hsad_threshold(scores, n, opt->z_alpha, dev_stats + 4, mask, ws_small, ws_small_bytes, stream)))
        return rc;
    double tf[4];
    if (hipMemcpyAsync(tf, dev_stats + 4, sizeof(tf), hipMemcpyDeviceToHost, stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess)
        return fail(HSAD_EHIP, "hsad_surrogate_run: reading the threshold failed");
    rep->pixels = n;
    rep->selected = fallback ? n : selected;
    rep->band = band_count;
    rep->audit = hc[2];
    rep->audit_rmse = audit[1];
    rep->audit_max = audit[2];
    rep->tau_pred = hs[3];
    rep->tau = tf[3];
    rep->fallback = fallback;
    rep->reserved = 0;
    rep->band_width = band;
    rep->audit_flips = flips;
    return HSAD_OK;
}

}  // extern "C"

extern "C" int hsad_internal_feat_cfg(int cfg)
{
    hsad::g_feat_cfg = cfg;
    return 0;
}
