// dev_boxg.hpp -- window statistics by sliding box sums for mid-size L' (any L' up to 128),
// the producer of the raw per-pixel records that the FP64 Cholesky kernel finalises.
//
// The annulus statistics of Sec. 2.2 (outer window minus inner window, clipped to the
// image) are sums over the window of f = x - ref and of the products f_i f_j, where ref is
// one pixel of the tile (it keeps the FP64 sums small; the covariance does not depend on
// it).  Window sums are separable: vertical running sums per (column, 2-row block), then
// running sums along each tile row, then a difference of two prefixes per pixel.  The
// work per pixel is a few operations per feature, against 2 n_a per feature for a direct
// Gram over the window.
//
// A 16 x 16 pixel tile per workgroup of 256 threads (thread = pixel in the last phase).
// Features are processed in chunks so that only the bands a chunk needs sit in LDS:
//   linear chunks: bands 4c .. 4c+3 (and, in the last one, the non-finite indicator);
//   product chunks: f_i f_j for i in a pair of bands, j in a block of 4 bands, j >= i.
// Non-finite samples: each non-finite value is replaced by ref (f = 0) and the sample is
// flagged; a flagged sample in the annulus makes the covariance NaN (score +inf), one in
// the inner window makes m_in NaN (DWRX NaN), and a non-finite centre pixel propagates
// through d = x_p - mu (the definitions of eqs. 1 and 5 on such data).
//
// Raw record per pixel ((L'+3) x L' doubles, row-major):
//   rows 0..L'-1, upper triangle j >= i : R_ij = (1/n_a) sum_annulus f_i f_j  (diagonal NaN
//                                          when the annulus holds a flagged sample)
//   row L'   : d = (x_p - ref) - mu_f          (mu_f = annulus mean of f)
//   row L'+1 : m = (inner mean of f) - mu_f    (NaN when the inner window holds a flagged
//                                               sample; unused without an inner window)
//   row L'+2 : mu_f
// The Cholesky kernel forms C = R - mu_f mu_f^T in the lower triangle, adds the loading and
// factorises (dev_chol.hpp).
#pragma once
#include <hip/hip_runtime.h>

namespace hsad {

constexpr int BG_TX = 16, BG_TY = 16, BG_NT = 256, BG_RB = 4;   // RB: output rows per vertical job
constexpr int BG_VS = 9;                 // odd LDS stride of the vertical-sum rows (>= 8 features)
// odd LDS stride of a pixel's horizontal window sums (>= 8 features): a 16-lane group reading
// its 16 pixels' sums, or writing a row's, then touches 16 different bank pairs (a stride of
// 8 doubles put every pixel of a row on the same two banks)
constexpr int BG_HS = 9;
constexpr int BG_MAX_LP = 128, BG_MAX_R = 15;

__host__ __device__ inline int bg_lpad(int Lp) { return (Lp + 3) & ~3; }

// LDS bytes of a tile for halo R and L' when the bands are staged per chunk (2 + 4 bands).
__host__ __device__ inline size_t bg_smem_chunked(int Lp, int R)
{
    const size_t EX = BG_TX + 2 * R, EY = BG_TY + 2 * R;
    return (size_t)bg_lpad(Lp) * 8            // ref
           + (size_t)BG_TY * EX * BG_VS * 8     // V (vertical sums)
           + (size_t)BG_TY * BG_TX * BG_HS * 8  // horizontal window sums
           + EY * EX * 4                        // bad flags
           + EY * EX * 6 * 4;                   // xi (2 bands) + xj (4 bands)
}
// ... and when every band of the extended tile stays resident in LDS (staged once).
__host__ __device__ inline size_t bg_smem_resident(int Lp, int R)
{
    const size_t EX = BG_TX + 2 * R, EY = BG_TY + 2 * R;
    return (size_t)bg_lpad(Lp) * 8 + (size_t)BG_TY * EX * BG_VS * 8 + (size_t)BG_TY * BG_TX * BG_HS * 8 + EY * EX * 4 +
           EY * EX * (size_t)bg_lpad(Lp) * 4;
}
// resident staging when the whole extended tile fits this many KiB of LDS (kernel argument,
// chosen on the host; 0 disables it)
__host__ __device__ inline bool bg_resident_at(int Lp, int R, int max_kb)
{
    // measured at 512^2 and 2048^2: per-chunk staging is faster up to L' = 16 (two tiles
    // per CU), resident bands beyond
    return Lp > 16 && bg_smem_resident(Lp, R) <= (size_t)max_kb * 1024;
}
__host__ __device__ inline size_t bg_smem_bytes(int Lp, int R, int max_kb)
{
    return bg_resident_at(Lp, R, max_kb) ? bg_smem_resident(Lp, R) : bg_smem_chunked(Lp, R);
}

__device__ __forceinline__ int bg_clip(int c, int r, int n)
{
    const int lo = c - r < 0 ? 0 : c - r, hi = c + r > n - 1 ? n - 1 : c + r;
    return hi - lo + 1;
}

// Window sums of NF features for the thread's pixel: S_in (inner window, when has_inner)
// and S_out (outer window).  feat(t, f) evaluates the NF features of extended-tile sample t.
// Vertical running sums per (column, block of RB rows) into V; then one job per (tile row,
// feature) slides the horizontal window along the row in registers and stores the 16
// window sums of that row in Hs; each thread finally reads its pixel's NF sums.
template <int NF, int RB, class Feat>
__device__ inline void bg_window_sums(const Feat &feat, int EX, int R, int RI, int has_inner, double *V,
                                      double *Hs, double *S_in, double *S_out)
{
    const int tid = threadIdx.x, ty = tid / BG_TX, tx = tid - ty * BG_TX;
#pragma unroll
    for (int g = 0; g < NF; ++g) S_in[g] = 0.0;
    for (int win = has_inner ? 0 : 1; win < 2; ++win) {
        const int h = win == 0 ? RI : R, eoff = R - h;
        // vertical: only the BG_TX + 2h columns this window's horizontal sums read
        const int EW = BG_TX + 2 * h;
        for (int job = tid; job < EW * (BG_TY / RB); job += BG_NT) {
            const int rb = job / EW, c = eoff + (job - rb * EW), r0 = rb * RB;
            double acc[NF];
#pragma unroll
            for (int g = 0; g < NF; ++g) acc[g] = 0.0;
            // uniform trip count (2h+1) and counter: the loop is unrolled and its LDS
            // reads overlap (a per-lane bound would wait for each read in turn)
#pragma unroll 4
            for (int k = 0; k <= 2 * h; ++k) {
                const int ey = r0 + eoff + k;
                double f[NF];
                feat(ey * EX + c, f);
#pragma unroll
                for (int g = 0; g < NF; ++g) acc[g] += f[g];
            }
            double *vr = V + ((size_t)r0 * EX + c) * BG_VS;
#pragma unroll
            for (int g = 0; g < NF; ++g) vr[g] = acc[g];
#pragma unroll
            for (int r = 1; r < RB; ++r) {
                double fa[NF], fb[NF];
                feat((r0 + r + eoff + 2 * h) * EX + c, fa);
                feat((r0 + r - 1 + eoff) * EX + c, fb);
#pragma unroll
                for (int g = 0; g < NF; ++g) acc[g] += fa[g] - fb[g];
                double *vq = V + ((size_t)(r0 + r) * EX + c) * BG_VS;
#pragma unroll
                for (int g = 0; g < NF; ++g) vq[g] = acc[g];
            }
        }
        __syncthreads();
        // horizontal: one job per (row, feature, HSG outputs); the segment's first sum
        // directly (four chains), the rest sliding
        constexpr int HSG = BG_TY * NF * (BG_TX / 8) <= BG_NT ? 8 : 16;
        constexpr int NSG = BG_TX / HSG;
        for (int job = tid; job < BG_TY * NF * NSG; job += BG_NT) {
            const int r = job / (NF * NSG), rem = job - r * (NF * NSG);
            const int g = rem / NSG, x0 = (rem - g * NSG) * HSG;
            const double *v = V + ((size_t)r * EX + x0 + eoff) * BG_VS + g;
            double r0 = 0.0, r1 = 0.0, r2 = 0.0, r3 = 0.0;
            int k = 0;
            for (; k + 3 <= 2 * h; k += 4) {
                r0 += v[(size_t)k * BG_VS];
                r1 += v[(size_t)(k + 1) * BG_VS];
                r2 += v[(size_t)(k + 2) * BG_VS];
                r3 += v[(size_t)(k + 3) * BG_VS];
            }
            for (; k <= 2 * h; ++k) r0 += v[(size_t)k * BG_VS];
            double run = (r0 + r1) + (r2 + r3);
            double *hs = Hs + ((size_t)r * BG_TX + x0) * BG_HS + g;
            hs[0] = run;
#pragma unroll
            for (int q = 1; q < HSG; ++q) {
                run += v[(size_t)(q + 2 * h) * BG_VS] - v[(size_t)(q - 1) * BG_VS];
                hs[(size_t)q * BG_HS] = run;
            }
        }
        __syncthreads();
        double *S = win == 0 ? S_in : S_out;
        const double *hp = Hs + ((size_t)ty * BG_TX + tx) * BG_HS;
#pragma unroll
        for (int g = 0; g < NF; ++g) S[g] = hp[g];
        __syncthreads();
    }
}

// Stage NB consecutive bands b0.. of the extended tile into dst[t * stride + q] (bands
// >= L' and samples outside the image stage as ref: f = 0).  One element per thread and
// step, so many independent loads are in flight.  Non-finite values stage as ref; if mark,
// their sample is flagged in bad[] (several threads may store the same 1.0f).
template <int NB>
__device__ inline void bg_stage(const float *__restrict__ x, int H, int W, int Lp, int R, int EX, int EY,
                                int y0, int x0, int b0, int stride, const double *ref, float *dst, float *bad,
                                bool mark)
{
    // Eight elements per thread and pass: the eight loads are issued unconditionally (from
    // coordinates clamped into the image) before any of their values is used, so their
    // round trips overlap; flags are OR-ed in with LDS atomics, which need no branch.
    constexpr int K = 8;
    const int n = EY * EX * NB;
    for (int e0 = threadIdx.x; e0 < n; e0 += K * BG_NT) {
        float u[K];
        bool ok[K];
        int tt[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int e = e0 + k * BG_NT, ec = e < n ? e : n - 1;
            const int t = ec / NB, q = ec - t * NB;     // NB is 2 or 4: shifts
            const int ey = t / EX, ex = t - ey * EX;
            const int gy = y0 - R + ey, gx = x0 - R + ex, b = b0 + q;
            ok[k] = e < n && gy >= 0 && gy < H && gx >= 0 && gx < W && b < Lp;
            const int cy = gy < 0 ? 0 : gy >= H ? H - 1 : gy, cx = gx < 0 ? 0 : gx >= W ? W - 1 : gx;
            u[k] = x[((size_t)cy * W + cx) * Lp + (b < Lp ? b : Lp - 1)];
            tt[k] = ec;
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
            if (e0 + k * BG_NT < n) {
                const int t = tt[k] / NB, q = tt[k] - t * NB;
                const bool fin = isfinite(u[k]);
                if (mark) atomicOr(reinterpret_cast<unsigned *>(bad + t), ok[k] && !fin ? 0x3f800000u : 0u);
                dst[t * stride + q] = ok[k] && fin ? u[k] : (float)ref[b0 + q];
            }
        }
    }
}

// All Lpad bands of the extended tile into xs[t * Lpad + b], row segment by row segment
// (a segment of the tile row is contiguous in the cube: coalesced loads).  Flags samples
// with a non-finite band.  magic_lp = ceil(2^32 / Lpad).
__device__ inline void bg_stage_all(const float *__restrict__ x, int H, int W, int Lp, int Lpad, int R, int EX,
                                    int EY, int y0, int x0, const double *ref, float *xs, float *bad)
{
    const int per_row = EX * Lpad, n = EY * per_row;
    const uint32_t m_row = (uint32_t)((((uint64_t)1 << 32) + (uint64_t)per_row - 1) / (uint64_t)per_row);
    const uint32_t m_lp = (uint32_t)((((uint64_t)1 << 32) + (uint64_t)Lpad - 1) / (uint64_t)Lpad);
    // eight elements per thread and pass, loads first (as bg_stage)
    constexpr int K = 8;
    for (int e0 = threadIdx.x; e0 < n; e0 += K * BG_NT) {
        float u[K];
        bool ok[K];
        int tb[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int e = e0 + k * BG_NT, ec = e < n ? e : n - 1;
            const int ey = (int)__umulhi((uint32_t)ec, m_row), rem = ec - ey * per_row;
            const int ex = (int)__umulhi((uint32_t)rem, m_lp), b = rem - ex * Lpad;
            const int gy = y0 - R + ey, gx = x0 - R + ex;
            ok[k] = e < n && gy >= 0 && gy < H && gx >= 0 && gx < W && b < Lp;
            const int cy = gy < 0 ? 0 : gy >= H ? H - 1 : gy, cx = gx < 0 ? 0 : gx >= W ? W - 1 : gx;
            u[k] = x[((size_t)cy * W + cx) * Lp + (b < Lp ? b : Lp - 1)];
            tb[k] = (ey * EX + ex) * 256 + b;        // sample index and band (Lpad <= 128)
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int e = e0 + k * BG_NT;
            if (e < n) {
                const int t = tb[k] >> 8, b = tb[k] & 255;
                const bool fin = isfinite(u[k]);
                atomicOr(reinterpret_cast<unsigned *>(bad + t), ok[k] && !fin ? 0x3f800000u : 0u);
                xs[e] = ok[k] && fin ? u[k] : (float)ref[b];
            }
        }
    }
}

// One tile: writes the raw records of its pixels (rows y0.., columns x0..) to
// rec + (pixel - pix0) * rec_stride, or, with pix0 < 0, to rec + (ty * 16 + tx) * rec_stride
// (tile-local records, as the batch engine allocates them).
// With inner_rec set (DWEST), rows L'+3 .. 2L'+2 of the record also take the inner-window
// second moments R_in,ij = (1/n_i) sum_inner f_i f_j (j >= i; diagonal NaN when the inner
// window holds a flagged sample), so the record holds both covariances of eqs. 2-3.
template <int RB = BG_RB>
__device__ inline void boxg_tile(const float *__restrict__ x, int H, int W, int Lp, int R, int RI, int has_inner,
                                 double *__restrict__ rec, int64_t pix0, int64_t rec_stride, int by, int bx,
                                 unsigned char *smem, int resident_kb, int inner_rec = 0)
{
    const int EX = BG_TX + 2 * R, EY = BG_TY + 2 * R;
    const int Lpad = bg_lpad(Lp);
    const bool resident = bg_resident_at(Lp, R, resident_kb);
    double *ref = reinterpret_cast<double *>(smem);
    double *V = ref + Lpad;
    double *Hs = V + (size_t)BG_TY * EX * BG_VS;
    float *bad = reinterpret_cast<float *>(Hs + (size_t)BG_TY * BG_TX * BG_HS);
    float *xs = bad + EY * EX;                  // resident: all bands, stride Lpad
    float *xi = xs, *xj = xs + EY * EX * 2;     // chunked: 2 + 4 bands
    const int tid = threadIdx.x, ty = tid / BG_TX, tx = tid - ty * BG_TX;
    const int y0 = by * BG_TY, x0 = bx * BG_TX;
    const int py = y0 + ty, px = x0 + tx;
    const bool valid = py < H && px < W;

    {
        const int ry = min(y0 + BG_TY / 2, H - 1), rx = min(x0 + BG_TX / 2, W - 1);
        const float *rp = x + ((size_t)ry * W + rx) * Lp;
        for (int b = tid; b < Lpad; b += BG_NT) {
            const float v = b < Lp ? rp[b] : 0.f;
            ref[b] = isfinite(v) ? (double)v : 0.0;
        }
        for (int t = tid; t < EY * EX; t += BG_NT) bad[t] = 0.0f;
    }
    __syncthreads();

    int n_a = 1, n_i = 1;
    if (valid) {
        const int n_o = bg_clip(py, R, H) * bg_clip(px, R, W);
        n_i = has_inner ? bg_clip(py, RI, H) * bg_clip(px, RI, W) : 0;
        n_a = n_o - n_i;
        if (n_i < 1) n_i = 1;
    }
    const double inv_na = 1.0 / (double)n_a, inv_ni = 1.0 / (double)n_i;
    const size_t pix = (size_t)py * W + px;
    double *r = !valid ? nullptr
                : pix0 < 0 ? rec + (int64_t)tid * rec_stride
                           : rec + (int64_t)(pix - (size_t)pix0) * rec_stride;
    const float *xc = x + pix * Lp;

    if (resident) {
        // every band of the extended tile, once
        __syncthreads();     // bad[] cleared above
        bg_stage_all(x, H, W, Lp, Lpad, R, EX, EY, y0, x0, ref, xs, bad);
    }
    const int sI = resident ? Lpad : 2, sJ = resident ? Lpad : 4;

    // ---- linear chunks (mu_f, d, m) and the indicator --------------------------------
    const int nlin = Lpad / 4;
    bool ann_bad = false, in_bad = false;
    for (int c = 0; c < nlin; ++c) {
        const int b0 = 4 * c;
        const bool last = c == nlin - 1;
        if (!resident) bg_stage<4>(x, H, W, Lp, R, EX, EY, y0, x0, b0, 4, ref, xj, bad, true);
        __syncthreads();
        double rf[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) rf[q] = ref[b0 + q];
        const float *xl = resident ? xs + b0 : xj;
        auto feat = [&](int t, double *f) {
            const float *s = xl + t * sJ;
#pragma unroll
            for (int q = 0; q < 4; ++q) f[q] = (double)s[q] - rf[q];
            f[4] = last ? (double)bad[t] : 0.0;
        };
        double S_in[5], S_out[5];
        bg_window_sums<5, RB>(feat, EX, R, RI, has_inner, V, Hs, S_in, S_out);
        if (valid) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int b = b0 + q;
                if (b < Lp) {
                    const double mu = (S_out[q] - S_in[q]) * inv_na;
                    r[(size_t)(Lp + 2) * Lp + b] = mu;
                    r[(size_t)Lp * Lp + b] = ((double)xc[b] - rf[q]) - mu;
                    r[(size_t)(Lp + 1) * Lp + b] = S_in[q] * inv_ni - mu;
                }
            }
            if (last) {
                ann_bad = (S_out[4] - S_in[4]) > 0.5;
                in_bad = has_inner && S_in[4] > 0.5;
            }
        }
    }
    if (valid && in_bad)
        for (int b = 0; b < Lp; ++b) r[(size_t)(Lp + 1) * Lp + b] = __builtin_nan("");

    // ---- product chunks: i in {i0, i0+1}, j in {j0..j0+3}, j >= i --------------------
    for (int i0 = 0; i0 < Lp; i0 += 2) {
        if (!resident) bg_stage<2>(x, H, W, Lp, R, EX, EY, y0, x0, i0, 2, ref, xi, bad, false);
        for (int j0 = i0 & ~3; j0 < Lp; j0 += 4) {
            if (!resident) bg_stage<4>(x, H, W, Lp, R, EX, EY, y0, x0, j0, 4, ref, xj, bad, false);
            __syncthreads();
            const double ri0 = ref[i0], ri1 = ref[i0 + 1];
            double rj[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) rj[q] = ref[j0 + q];
            const float *xa = resident ? xs + i0 : xi, *xb = resident ? xs + j0 : xj;
            auto feat = [&](int t, double *f) {
                const double a0 = (double)xa[t * sI] - ri0, a1 = (double)xa[t * sI + 1] - ri1;
                const float *s = xb + t * sJ;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const double bq = (double)s[q] - rj[q];
                    f[q] = a0 * bq;
                    f[4 + q] = a1 * bq;
                }
            };
            double S_in[8], S_out[8];
            bg_window_sums<8, RB>(feat, EX, R, RI, has_inner, V, Hs, S_in, S_out);
            if (valid) {
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int i = i0 + a, j = j0 + q;
                        if (i < Lp && j < Lp && j >= i) {
                            double v = (S_out[4 * a + q] - S_in[4 * a + q]) * inv_na;
                            if (i == j && ann_bad) v = __builtin_nan("");
                            r[(size_t)i * Lp + j] = v;
                            if (inner_rec) {
                                double u = S_in[4 * a + q] * inv_ni;
                                if (i == j && in_bad) u = __builtin_nan("");
                                r[(size_t)(Lp + 3 + i) * Lp + j] = u;
                            }
                        }
                    }
            }
        }
    }
}

}  // namespace hsad
