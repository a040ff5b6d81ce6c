// dev_box.hpp -- device body of the fused box-sum LRX/DWRX tile (window statistics,
// loading, Cholesky and scores for L' <= 8), shared by the per-cube kernel and the
// persistent batch kernel.  See box.hip for the method notes.
#pragma once
#include <hip/hip_runtime.h>

namespace hsad {

// Tiles are TXW x 16 output pixels (TXW = 16 or 32), one thread per pixel.  A wider tile
// spends fewer halo columns per pixel (TXW + 2R columns of vertical sums for TXW outputs).
constexpr int TY = 16;
// largest inner half-width summed directly per pixel (box_tile)
constexpr int kBoxDirectRI = 3;
constexpr int RB = 4;                 // output rows per vertical-sum job
constexpr int NRB = TY / RB;

template <int LP, int GCMAX = 15> struct BoxCfg {
    static constexpr int G = LP + LP * (LP + 1) / 2;   // moment features
    static constexpr int GT = G + 1;                   // + non-finite indicator
    static constexpr int GC = GT < GCMAX ? GT : GCMAX; // features per LDS chunk
    static constexpr int GCP = GC | 1;                 // odd stride (bank spread)
    static constexpr int NCH = (GT + GC - 1) / GC;
};

// Feature g of a pixel with centred values f[] and flag b (g is a compile-time constant
// after unrolling).
template <int LP> __device__ __forceinline__ double feat(const double *f, double b, int g)
{
    if (g < LP) return f[g];
    if (g >= BoxCfg<LP>::G) return b;
    // product feature r = g - LP enumerates the upper triangle row by row; row k starts at
    // k LP - k (k - 1) / 2.  A fixed-trip-count search keeps every index a compile-time
    // constant once g is (a data-dependent loop here sends f[] to scratch memory).
    const int r = g - LP;
    int i = 0;
#pragma unroll
    for (int k = 1; k < LP; ++k)
        if (r >= k * LP - k * (k - 1) / 2) i = k;
    const int j = i + (r - (i * LP - i * (i - 1) / 2));
    return f[i] * f[j];
}

// Centred values of tile pixel t (FP64, exact).
template <int LP>
__device__ __forceinline__ void centred(const float *xs, size_t t, const double *ref, double *f)
{
    if constexpr (LP % 4 == 0) {
        const float4 *q = reinterpret_cast<const float4 *>(xs + t * LP);
#pragma unroll
        for (int k = 0; k < LP / 4; ++k) {
            const float4 v = q[k];
            f[4 * k] = (double)v.x - ref[4 * k];
            f[4 * k + 1] = (double)v.y - ref[4 * k + 1];
            f[4 * k + 2] = (double)v.z - ref[4 * k + 2];
            f[4 * k + 3] = (double)v.w - ref[4 * k + 3];
        }
    } else {
#pragma unroll
        for (int i = 0; i < LP; ++i) f[i] = (double)xs[t * LP + i] - ref[i];
    }
}

__device__ __forceinline__ int clip_count(int c, int r, int n)
{
    const int lo = c - r < 0 ? 0 : c - r;
    const int hi = c + r > n - 1 ? n - 1 : c + r;
    return hi - lo + 1;
}

// Step 3 of the tile: statistics of the annulus from its sums S (features in the order of
// feat(): L' linear, the upper triangle of products, the non-finite count), loading,
// Cholesky and both scores for output pixel (py, px).
template <int LP, int GT>
// Returns the LRX score it wrote (NaN when lrx is NULL).
__device__ __forceinline__ float box_score(const float *__restrict__ x, int H, int W, int R, int RI,
                                           int has_inner, double load_rel, const double *ref,
                                           const double *S, double *sin_lin, double in_bad, int py,
                                           int px, float *__restrict__ lrx, float *__restrict__ dwrx)
{
    constexpr int G = GT - 1;
    // 3. statistics of the annulus, loading, Cholesky, scores
    const int n_o = clip_count(py, R, H) * clip_count(px, R, W);
    const int n_i = has_inner ? clip_count(py, RI, H) * clip_count(px, RI, W) : 0;
    const double inv_na = 1.0 / (double)(n_o - n_i);
    const bool ann_bad = S[G] > 0.5;      // exact small integers in FP64
    double mu[LP];
#pragma unroll
    for (int i = 0; i < LP; ++i) mu[i] = S[i] * inv_na;
    double Lm[LP][LP];
    double tr = 0.0;
    {
        int g = LP;
#pragma unroll
        for (int i = 0; i < LP; ++i)
#pragma unroll
            for (int j = i; j < LP; ++j) {
                const double c = S[g++] * inv_na - mu[i] * mu[j];
                Lm[j][i] = c;
                if (i == j) tr += c;
            }
    }
    double lam = load_rel * tr / (double)LP;
    lam = lam < 1e-30 ? 1e-30 : lam;
    // Cholesky with reciprocal pivots: Lm[j][j] holds 1/L_jj
    bool pd = true;
#pragma unroll
    for (int j = 0; j < LP; ++j) {
        double d = Lm[j][j] + lam;
#pragma unroll
        for (int k = 0; k < j; ++k) d -= Lm[j][k] * Lm[j][k];
        pd = pd && (d > 0.0);
        const double inv = rsqrt(d);
        Lm[j][j] = inv;
#pragma unroll
        for (int i = j + 1; i < LP; ++i) {
            double t = Lm[i][j];
#pragma unroll
            for (int k = 0; k < j; ++k) t -= Lm[i][k] * Lm[j][k];
            Lm[i][j] = t * inv;
        }
    }
    const size_t o = (size_t)py * W + px;
    float lrx_v = NAN;
    if (lrx) {
        const float *pc = x + o * LP;            // raw centre pixel
        double z[LP], s = 0.0;
#pragma unroll
        for (int i = 0; i < LP; ++i) {
            double t = ((double)pc[i] - ref[i]) - mu[i];
#pragma unroll
            for (int k = 0; k < i; ++k) t -= Lm[i][k] * z[k];
            z[i] = t * Lm[i][i];
            s += z[i] * z[i];
        }
        lrx_v = (pd && !ann_bad) ? (float)s : INFINITY;
        lrx[o] = lrx_v;
    }
    if (dwrx) {
        if (in_bad > 0.5) {
            // rare: a non-finite inner sample; take the mean from the raw values so that
            // NaN / Inf propagate exactly as in the definition
#pragma unroll
            for (int i = 0; i < LP; ++i) sin_lin[i] = 0.0;
            for (int dy = -RI; dy <= RI; ++dy)
                for (int dx = -RI; dx <= RI; ++dx) {
                    const int gy = py + dy, gx = px + dx;
                    if (gy < 0 || gy >= H || gx < 0 || gx >= W) continue;
                    const float *raw = x + ((size_t)gy * W + gx) * LP;
#pragma unroll
                    for (int i = 0; i < LP; ++i) sin_lin[i] += (double)raw[i] - ref[i];
                }
        }
        const double inv_ni = 1.0 / (double)n_i;
        double z[LP], s = 0.0;
#pragma unroll
        for (int i = 0; i < LP; ++i) {
            double t = sin_lin[i] * inv_ni - mu[i];
#pragma unroll
            for (int k = 0; k < i; ++k) t -= Lm[i][k] * z[k];
            z[i] = t * Lm[i][i];
            s += z[i] * z[i];
        }
        dwrx[o] = (pd && !ann_bad) ? (float)s : INFINITY;
    }
    return lrx_v;
}

// Deterministic block sum of NW wavefronts (fixed shuffle tree per wavefront, then the
// wavefront sums pairwise: (0+1) + (2+3), ...); red holds NW doubles of LDS; the result is
// valid in every thread.
template <int NW> __device__ __forceinline__ double box_block_sum(double v, double *red)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double t[NW];
#pragma unroll
    for (int i = 0; i < NW; ++i) t[i] = red[i];
#pragma unroll
    for (int w = NW / 2; w >= 1; w /= 2)
#pragma unroll
        for (int i = 0; i < w; ++i) t[i] = t[2 * i] + t[2 * i + 1];
    __syncthreads();
    return t[0];
}

// Two block sums in one round (each in the order of box_block_sum, so the results are the
// same); red holds 2 NW doubles.
template <int NW> __device__ __forceinline__ void box_block_sum2(double &a, double &b, double *red)
{
    for (int o = 32; o > 0; o >>= 1) {
        const double xa = __shfl_xor(a, o), xb = __shfl_xor(b, o);
        a += xa;
        b += xb;
    }
    if ((threadIdx.x & 63) == 0) {
        red[threadIdx.x >> 6] = a;
        red[NW + (threadIdx.x >> 6)] = b;
    }
    __syncthreads();
    double t[NW], u[NW];
#pragma unroll
    for (int i = 0; i < NW; ++i) {
        t[i] = red[i];
        u[i] = red[NW + i];
    }
#pragma unroll
    for (int w = NW / 2; w >= 1; w /= 2)
#pragma unroll
        for (int i = 0; i < w; ++i) {
            t[i] = t[2 * i] + t[2 * i + 1];
            u[i] = u[2 * i] + u[2 * i + 1];
        }
    __syncthreads();
    a = t[0];
    b = u[0];
}

// (count, mean, centred sum of squares) of the finite values v of a tile's threads, two
// passes in FP64 -> out[0..2].  The partial statistics of eq. (12) for one tile.
template <int NW> __device__ __forceinline__ void box_tile_stats(float v, bool valid, double *out, double *red)
{
    const bool fin = valid && isfinite(v);
    double c = fin ? 1.0 : 0.0, sum = fin ? (double)v : 0.0;
    box_block_sum2<NW>(c, sum, red);
    const double mean = c > 0.0 ? sum / c : 0.0;
    const double d = fin ? (double)v - mean : 0.0;
    const double m2 = box_block_sum<NW>(d * d, red);
    if (threadIdx.x == 0) {
        out[0] = c;
        out[1] = mean;
        out[2] = m2;
    }
}

// FEATLANES: the horizontal jobs take the feature fastest over the lanes (fewer LDS bank
// conflicts; faster on its own), else the segment (faster beside the DWT in the shared
// launch).  Either order gives the same sums.
template <int LP, int GCMAX, int TXW = 16, bool FEATLANES = true>
__device__ __forceinline__ void box_tile(const float *__restrict__ x, int H, int W, int R, int RI,
                                int has_inner, double load_rel, float *__restrict__ lrx,
                                float *__restrict__ dwrx, int by, int bx, double *smem,
                                double *__restrict__ part = nullptr, int ntx = -1)
{
    using C = BoxCfg<LP, GCMAX>;
    constexpr int TX = TXW, NT = TXW * TY;
    const int EX = TX + 2 * R, EY = TY + 2 * R;
    double *V = smem;                                                    // TY*EX*GCP
    float *xs = reinterpret_cast<float *>(smem + (size_t)TY * EX * C::GCP);   // EY*EX*LP
    float *bad = xs + (size_t)EY * EX * LP;                              // EY*EX

    const int tid = threadIdx.x;
    const int y0 = by * TY, x0 = bx * TX;

    double ref[LP];
    {
        const int ry = min(y0 + TY / 2, H - 1), rx = min(x0 + TX / 2, W - 1);
        const float *rp = x + ((size_t)ry * W + rx) * LP;
#pragma unroll
        for (int i = 0; i < LP; ++i) {
            const float v = rp[i];
            ref[i] = isfinite(v) ? (double)v : 0.0;
        }
    }

    // 1. halo tile.  The loads are unconditional, from coordinates clamped into the image,
    //    and the outside samples are dropped by selects afterwards: a load under a
    //    lane-dependent branch whose value is used inside it waits for its round trip
    //    before the next iteration's loads are issued.
#pragma unroll 4
    for (int t = tid; t < EY * EX; t += NT) {
        const int ey = t / EX, ex = t - ey * EX;
        const int gy = y0 - R + ey, gx = x0 - R + ex;
        const bool ok = gy >= 0 && gy < H && gx >= 0 && gx < W;
        const int cy = gy < 0 ? 0 : gy >= H ? H - 1 : gy, cx = gx < 0 ? 0 : gx >= W ? W - 1 : gx;
        const float *src = x + ((size_t)cy * W + cx) * LP;
        float v[LP];
        bool fin = true;
#pragma unroll
        for (int i = 0; i < LP; ++i) {
            v[i] = src[i];
            fin = fin && isfinite(v[i]);
        }
        float *dst = xs + (size_t)t * LP;
#pragma unroll
        for (int i = 0; i < LP; ++i) dst[i] = (ok && fin) ? v[i] : (float)ref[i];
        bad[t] = (ok && !fin) ? 1.0f : 0.0f;
    }
    __syncthreads();

    const int ty = tid / TX, tx = tid - ty * TX;
    const int py = y0 + ty, px = x0 + tx;

    // a small inner window (up to 7 x 7) is summed directly per output pixel from the staged
    // tile after the outer window's box sums, instead of by two more rounds of box sums
    const bool direct_inner = has_inner && RI <= kBoxDirectRI;
    double S[C::GT];        // annulus sums (outer minus inner)
    double sin_lin[LP];     // inner-window linear sums (DWRX mean)
    double in_bad = 0.0;
#pragma unroll
    for (int g = 0; g < C::GT; ++g) S[g] = 0.0;
#pragma unroll
    for (int i = 0; i < LP; ++i) sin_lin[i] = 0.0;

#pragma unroll
    for (int ch = 0; ch < C::NCH; ++ch) {
        const int g0 = ch * C::GC;
        for (int win = has_inner && !direct_inner ? 0 : 1; win < 2; ++win) {
            // win 0: inner window (half RI), win 1: outer window (half R)
            const int h = win == 0 ? RI : R;
            const int eoff = R - h;            // first extended row/col of the window
            // 2a. vertical sums: job = (column c, row block rb), for the TX + 2h columns the
            //     window's horizontal sums read (eoff .. eoff + TX + 2h - 1)
            const int EW = TX + 2 * h;
            for (int job = tid; job < EW * NRB; job += NT) {
                const int rb = job / EW, c = eoff + (job - rb * EW);
                const int r0 = rb * RB;
                double acc[C::GC];
#pragma unroll
                for (int gg = 0; gg < C::GC; ++gg) acc[gg] = 0.0;
                // uniform trip count (2h+1) and counter: the loop is unrolled and its LDS
                // reads overlap (a per-lane bound would wait for each read in turn)
#pragma unroll 4
                for (int k = 0; k <= 2 * h; ++k) {
                    const int ey = r0 + eoff + k;
                    const size_t t = (size_t)ey * EX + c;
                    double f[LP];
                    centred<LP>(xs, t, ref, f);
                    const double b = (double)bad[t];
#pragma unroll
                    for (int gg = 0; gg < C::GC; ++gg)
                        if (g0 + gg < C::GT) acc[gg] += feat<LP>(f, b, g0 + gg);
                }
                double *vr = V + ((size_t)r0 * EX + c) * C::GCP;
#pragma unroll
                for (int gg = 0; gg < C::GC; ++gg) vr[gg] = acc[gg];
#pragma unroll
                for (int r = 1; r < RB; ++r) {
                    const size_t ta = (size_t)(r0 + r + eoff + 2 * h) * EX + c;
                    const size_t tb = (size_t)(r0 + r - 1 + eoff) * EX + c;
                    double fa[LP], fb[LP];
                    centred<LP>(xs, ta, ref, fa);
                    centred<LP>(xs, tb, ref, fb);
                    const double ba = (double)bad[ta], bb = (double)bad[tb];
#pragma unroll
                    for (int gg = 0; gg < C::GC; ++gg)
                        if (g0 + gg < C::GT)
                            acc[gg] += feat<LP>(fa, ba, g0 + gg) - feat<LP>(fb, bb, g0 + gg);
                    double *vq = V + ((size_t)(r0 + r) * EX + c) * C::GCP;
#pragma unroll
                    for (int gg = 0; gg < C::GC; ++gg) vq[gg] = acc[gg];
                }
            }
            __syncthreads();
            // 2b. horizontal window sums: one job per (row, feature, segment of HS outputs).
            //     The segment's first sum is taken directly (2h+1 terms, four chains), the
            //     rest slide by one column; the results wait in registers for a barrier and
            //     then overwrite the row's first TX columns.  A dependency chain of about
            //     HS + 4 adds per job where a running sum along the row was EX long.
            constexpr int HS = TY * C::GC * (TX / 8) <= NT ? 8 : TY * C::GC * (TX / 16) <= NT ? 16 : 32;
            constexpr int NSEG = TX / HS;
            static_assert(TY * C::GC * NSEG <= NT, "one horizontal job per thread");
            double hv[HS];
            const bool hjob = tid < TY * C::GC * NSEG;
            // FEATLANES: the feature varies fastest over the lanes, then the segment, so the
            // lanes of a 16-lane group read 16 different LDS bank pairs (feature stride 2
            // banks, segment stride 8 GCP = 72 doubles, 16 banks mod 32)
            const int hr = tid / (C::GC * NSEG), hrem = tid - hr * (C::GC * NSEG);
            const int hseg = FEATLANES ? hrem / C::GC : hrem % NSEG;
            const int hg = FEATLANES ? hrem - hseg * C::GC : hrem / NSEG, hx0 = hseg * HS;
            if (hjob) {
                const double *v = V + ((size_t)hr * EX + hx0 + eoff) * C::GCP + hg;
                double r0 = 0.0, r1 = 0.0, r2 = 0.0, r3 = 0.0;
                int k = 0;
                for (; k + 3 <= 2 * h; k += 4) {
                    r0 += v[(size_t)k * C::GCP];
                    r1 += v[(size_t)(k + 1) * C::GCP];
                    r2 += v[(size_t)(k + 2) * C::GCP];
                    r3 += v[(size_t)(k + 3) * C::GCP];
                }
                for (; k <= 2 * h; ++k) r0 += v[(size_t)k * C::GCP];
                double run = (r0 + r1) + (r2 + r3);
                hv[0] = run;
#pragma unroll
                for (int q = 1; q < HS; ++q) {
                    run += v[(size_t)(q + 2 * h) * C::GCP] - v[(size_t)(q - 1) * C::GCP];
                    hv[q] = run;
                }
            }
            __syncthreads();
            if (hjob) {
                double *o = V + ((size_t)hr * EX + hx0) * C::GCP + hg;
#pragma unroll
                for (int q = 0; q < HS; ++q) o[(size_t)q * C::GCP] = hv[q];
            }
            __syncthreads();
            // 2c. this thread's pixel: its window sums are now at column tx of row ty
            const double *vh = V + ((size_t)ty * EX + tx) * C::GCP;
            double hsum[C::GC];
#pragma unroll
            for (int gg = 0; gg < C::GC; ++gg) hsum[gg] = vh[gg];
#pragma unroll
            for (int gg = 0; gg < C::GC; ++gg) {
                const int g = g0 + gg;
                if (g < C::GT) {
                    if (win == 0) {
                        S[g] -= hsum[gg];
                        if (g < LP) sin_lin[g] = hsum[gg];
                        if (g == C::G) in_bad = hsum[gg];
                    } else {
                        S[g] += hsum[gg];
                    }
                }
            }
            __syncthreads();
        }
    }

    if (direct_inner) {
        for (int dy = -RI; dy <= RI; ++dy) {
#pragma unroll 1
            for (int dx = -RI; dx <= RI; ++dx) {
                const size_t t = (size_t)(ty + R + dy) * EX + (tx + R + dx);
                double f[LP];
                centred<LP>(xs, t, ref, f);
                const double b = (double)bad[t];
#pragma unroll
                for (int g = 0; g < C::GT; ++g) S[g] -= feat<LP>(f, b, g);
#pragma unroll
                for (int i = 0; i < LP; ++i) sin_lin[i] += f[i];
                in_bad += b;
            }
        }
    }
    const bool inside = py < H && px < W;
    float v = NAN;
    if (inside)
        v = box_score<LP, C::GT>(x, H, W, R, RI, has_inner, load_rel, ref, S, sin_lin, in_bad, py, px, lrx,
                                 dwrx);
    // eq. (12) partials of this tile's LRX scores (the LDS tile is free again here)
    // partial of tile (by, bx) at by * ntx + bx (ntx: tiles per row, the grid's x extent by
    // default)
    if (part)
        box_tile_stats<NT / 64>(v, inside, part + 3 * ((size_t)by * (ntx < 0 ? (int)gridDim.x : ntx) + bx), smem);
}


template <int LP, int GCMAX = 15, int TXW = 16> __host__ __device__ inline size_t box_smem(int R)
{
    using C = BoxCfg<LP, GCMAX>;
    const size_t EX = TXW + 2 * R, EY = TY + 2 * R;
    return (size_t)TY * EX * C::GCP * sizeof(double) + EY * EX * (LP + 1) * sizeof(float);
}

}  // namespace hsad
