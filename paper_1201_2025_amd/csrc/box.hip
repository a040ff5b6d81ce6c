// box.hip -- fused window statistics + loading + Cholesky + LRX/DWRX for short spectra
// (L' <= 8), the regime of the paper's DWT-reduced detectors (Sec. 4: four samples).
//
// Statistics (Sec. 2.1 local background; Sec. 2.2 inner/outer windows).  For pixel p the
// annulus A = outer window \ inner window, both clipped to the image.  Its mean and 1/n
// covariance come from box sums of the features
//     f_i = x_i - ref_i          (L' linear features)
//     q_ij = f_i f_j, i <= j     (L'(L'+1)/2 quadratic features)
//     b = [pixel has a non-finite component]
// where ref is one pixel of the tile.  Every feature is exact in FP64: the difference of
// two FP32 values and the product of two such differences both fit in 53 bits.  The sums
// are FP64, so C = Q/n - mu_f mu_f^T keeps about 12 significant digits even when |mu_f|^2
// is 1e4 times the smallest eigenvalue of C.  This data-dependent cancellation rules
// out FP32 sums here.
//
// Per 16 x 16 output tile (256 threads, one output pixel each):
//   1. stage the (16+2R)^2 halo tile of the reduced cube in LDS (coalesced).  Pixels
//      outside the image or with a non-finite component take the reference value, and
//      the second kind is flagged;
//   2. for each feature chunk and each window (inner, then outer): vertical box sums,
//      one job per (column, pair of output rows) with every feature of the chunk in
//      registers; then horizontal sums of those columns by each output thread.
//      S = outer - inner gives the annulus sums directly;
//   3. mu, C, diagonal loading lambda = load_rel tr(C)/L' (floor 1e-30), Cholesky in
//      registers (FP64), z = L^-1 d and score = |z|^2 for d = x_p - mu (LRX, eq. 1)
//      and d = m_in - mu (DWRX, eq. 5).
//   A non-finite sample in the annulus makes the covariance non-finite, and the score
//   is +inf as in the definition.  A non-finite centre or inner-window value propagates
//   through d, from the raw values (a rare path that re-reads the inner window).
// HBM traffic is the reduced cube once (the halo re-reads hit L2) and the score maps.
#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace hsad {

namespace {
constexpr int TX = 16, TY = 16, NT = TX * TY;
constexpr int RB = 2;                 // output rows per vertical-sum job
constexpr int NRB = TY / RB;

template <int LP> struct BoxCfg {
    static constexpr int G = LP + LP * (LP + 1) / 2;   // moment features
    static constexpr int GT = G + 1;                   // + non-finite indicator
    static constexpr int GC = GT < 15 ? GT : 15;       // features per LDS chunk
    static constexpr int GCP = GC | 1;                 // odd stride (bank spread)
    static constexpr int NCH = (GT + GC - 1) / GC;
};

// Feature g of a pixel with centred values f[] and flag b (g is a compile-time constant
// after unrolling).
template <int LP> __device__ __forceinline__ double feat(const double *f, double b, int g)
{
    if (g < LP) return f[g];
    if (g >= BoxCfg<LP>::G) return b;
    int r = g - LP, i = 0, len = LP;
    while (r >= len) {
        r -= len;
        --len;
        ++i;
    }
    return f[i] * f[i + r];
}

__device__ __forceinline__ int clip_count(int c, int r, int n)
{
    const int lo = c - r < 0 ? 0 : c - r;
    const int hi = c + r > n - 1 ? n - 1 : c + r;
    return hi - lo + 1;
}
}  // namespace

template <int LP>
__global__ __launch_bounds__(NT) void box_lrx_dwrx_kernel(const float *__restrict__ x, int H,
                                                          int W, int R, int RI, int has_inner,
                                                          double load_rel,
                                                          float *__restrict__ lrx,
                                                          float *__restrict__ dwrx)
{
    using C = BoxCfg<LP>;
    extern __shared__ double smem[];
    const int EX = TX + 2 * R, EY = TY + 2 * R;
    double *V = smem;                                                    // TY*EX*GCP
    float *xs = reinterpret_cast<float *>(smem + (size_t)TY * EX * C::GCP);   // EY*EX*LP
    float *bad = xs + (size_t)EY * EX * LP;                              // EY*EX

    const int tid = threadIdx.x;
    const int y0 = blockIdx.y * TY, x0 = blockIdx.x * TX;

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

    // 1. halo tile
    for (int t = tid; t < EY * EX; t += NT) {
        const int ey = t / EX, ex = t - ey * EX;
        const int gy = y0 - R + ey, gx = x0 - R + ex;
        float v[LP];
        bool ok = false, fin = true;
        if (gy >= 0 && gy < H && gx >= 0 && gx < W) {
            const float *src = x + ((size_t)gy * W + gx) * LP;
            ok = true;
#pragma unroll
            for (int i = 0; i < LP; ++i) {
                v[i] = src[i];
                fin = fin && isfinite(v[i]);
            }
        }
        float *dst = xs + (size_t)t * LP;
#pragma unroll
        for (int i = 0; i < LP; ++i) dst[i] = (ok && fin) ? v[i] : (float)ref[i];
        bad[t] = (ok && !fin) ? 1.0f : 0.0f;
    }
    __syncthreads();

    const int ty = tid / TX, tx = tid - ty * TX;
    const int py = y0 + ty, px = x0 + tx;

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
        for (int win = has_inner ? 0 : 1; win < 2; ++win) {
            // win 0: inner window (half RI), win 1: outer window (half R)
            const int h = win == 0 ? RI : R;
            const int eoff = R - h;            // first extended row/col of the window
            // 2a. vertical sums: job = (column c, row block rb)
            for (int job = tid; job < EX * NRB; job += NT) {
                const int rb = job / EX, c = job - rb * EX;
                const int r0 = rb * RB;
                double acc[C::GC];
#pragma unroll
                for (int gg = 0; gg < C::GC; ++gg) acc[gg] = 0.0;
                for (int ey = r0 + eoff; ey <= r0 + eoff + 2 * h; ++ey) {
                    const size_t t = (size_t)ey * EX + c;
                    double f[LP];
#pragma unroll
                    for (int i = 0; i < LP; ++i) f[i] = (double)xs[t * LP + i] - ref[i];
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
#pragma unroll
                    for (int i = 0; i < LP; ++i) {
                        fa[i] = (double)xs[ta * LP + i] - ref[i];
                        fb[i] = (double)xs[tb * LP + i] - ref[i];
                    }
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
            // 2b. horizontal sums for this thread's pixel
            const double *vrow = V + ((size_t)ty * EX + tx + eoff) * C::GCP;
            double hsum[C::GC];
#pragma unroll
            for (int gg = 0; gg < C::GC; ++gg) hsum[gg] = 0.0;
            for (int dx = 0; dx <= 2 * h; ++dx) {
                const double *v = vrow + (size_t)dx * C::GCP;
#pragma unroll
                for (int gg = 0; gg < C::GC; ++gg) hsum[gg] += v[gg];
            }
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

    if (py >= H || px >= W) return;

    // 3. statistics of the annulus, loading, Cholesky, scores
    const int n_o = clip_count(py, R, H) * clip_count(px, R, W);
    const int n_i = has_inner ? clip_count(py, RI, H) * clip_count(px, RI, W) : 0;
    const double inv_na = 1.0 / (double)(n_o - n_i);
    const bool ann_bad = S[C::G] > 0.5;      // exact small integers in FP64
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
    bool pd = true;
#pragma unroll
    for (int j = 0; j < LP; ++j) {
        double d = Lm[j][j] + lam;
#pragma unroll
        for (int k = 0; k < j; ++k) d -= Lm[j][k] * Lm[j][k];
        pd = pd && (d > 0.0);
        const double ljj = sqrt(d);
        Lm[j][j] = ljj;
        const double inv = 1.0 / ljj;
#pragma unroll
        for (int i = j + 1; i < LP; ++i) {
            double t = Lm[i][j];
#pragma unroll
            for (int k = 0; k < j; ++k) t -= Lm[i][k] * Lm[j][k];
            Lm[i][j] = t * inv;
        }
    }
    const size_t o = (size_t)py * W + px;
    if (lrx) {
        const float *pc = x + o * LP;            // raw centre pixel
        double z[LP], s = 0.0;
#pragma unroll
        for (int i = 0; i < LP; ++i) {
            double t = ((double)pc[i] - ref[i]) - mu[i];
#pragma unroll
            for (int k = 0; k < i; ++k) t -= Lm[i][k] * z[k];
            z[i] = t / Lm[i][i];
            s += z[i] * z[i];
        }
        lrx[o] = (pd && !ann_bad) ? (float)s : INFINITY;
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
            z[i] = t / Lm[i][i];
            s += z[i] * z[i];
        }
        dwrx[o] = (pd && !ann_bad) ? (float)s : INFINITY;
    }
}

template <int LP> static size_t box_smem(int R)
{
    using C = BoxCfg<LP>;
    const size_t EX = TX + 2 * R, EY = TY + 2 * R;
    return (size_t)TY * EX * C::GCP * sizeof(double) + EY * EX * (LP + 1) * sizeof(float);
}

static size_t box_smem_lp(int64_t Lp, int R)
{
    switch (Lp) {
    case 1: return box_smem<1>(R);
    case 2: return box_smem<2>(R);
    case 3: return box_smem<3>(R);
    case 4: return box_smem<4>(R);
    case 5: return box_smem<5>(R);
    case 6: return box_smem<6>(R);
    case 7: return box_smem<7>(R);
    case 8: return box_smem<8>(R);
    default: return (size_t)-1;
    }
}

static constexpr size_t kBoxMaxSmem = 144 * 1024;

bool box_supported(int64_t Lp, const Windows &w)
{
    return Lp >= 1 && Lp <= 8 && box_smem_lp(Lp, w.ro) <= kBoxMaxSmem;
}

template <int LP>
static int box_launch(const float *x, int64_t H, int64_t W, const Windows &w, double load_rel,
                      float *lrx, float *dwrx, hipStream_t s)
{
    const size_t sh = box_smem<LP>(w.ro);
    if (int rc = allow_lds((const void *)box_lrx_dwrx_kernel<LP>, sh, "box_lrx_dwrx_kernel")) return rc;
    dim3 grid((unsigned)((W + TX - 1) / TX), (unsigned)((H + TY - 1) / TY)), block(NT);
    hipLaunchKernelGGL(box_lrx_dwrx_kernel<LP>, grid, block, sh, s, x, (int)H, (int)W, w.ro, w.ri,
                       w.inner > 0 ? 1 : 0, load_rel, lrx, dwrx);
    return check_launch("box_lrx_dwrx_kernel");
}

int box_lrx_dwrx_launch(const float *x, int64_t H, int64_t W, int64_t Lp, const Windows &w,
                        double load_rel, float *lrx, float *dwrx, hipStream_t s)
{
    if (H > (1 << 24) || W > (1 << 24)) return fail(HSAD_EUNSUPPORTED, "box path: image too large");
    switch (Lp) {
    case 1: return box_launch<1>(x, H, W, w, load_rel, lrx, dwrx, s);
    case 2: return box_launch<2>(x, H, W, w, load_rel, lrx, dwrx, s);
    case 3: return box_launch<3>(x, H, W, w, load_rel, lrx, dwrx, s);
    case 4: return box_launch<4>(x, H, W, w, load_rel, lrx, dwrx, s);
    case 5: return box_launch<5>(x, H, W, w, load_rel, lrx, dwrx, s);
    case 6: return box_launch<6>(x, H, W, w, load_rel, lrx, dwrx, s);
    case 7: return box_launch<7>(x, H, W, w, load_rel, lrx, dwrx, s);
    case 8: return box_launch<8>(x, H, W, w, load_rel, lrx, dwrx, s);
    default: return fail(HSAD_EUNSUPPORTED, "box path: L' > 8");
    }
}

}  // namespace hsad
