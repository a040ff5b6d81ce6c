// box.hip -- fused window statistics + loading + Cholesky + LRX/DWRX for short spectra
// (L' <= 8), the regime of the paper's DWT-reduced detectors (Sec. 4: four samples).
//
// Statistics (Sec. 2.1 local background; Sec. 2.2 inner/outer windows).  For pixel p the
// annulus A = outer window \ inner window, both clipped to the image.  Its mean and 1/n
// covariance come from box sums of the features
//     f_i = x_i - ref_i          (L' linear features)
//     q_ij = f_i f_j, i <= j     (L'(L'+1)/2 quadratic features)
// where ref is one pixel of the tile.  Every feature is exact in FP64: the difference of
// two FP32 values and the product of two such differences both fit in 53 bits.  The sums
// are FP64, so C = Q/n - mu_f mu_f^T keeps about 12 significant digits even when |mu_f|^2
// is 1e4 times the smallest eigenvalue of C.  This is the data-dependent cancellation
// that rules out FP32 sums here.
//
// Per 16 x 16 output tile (256 threads, one per output pixel):
//   1. stage the (16+2R)^2 halo tile of the reduced cube in LDS (coalesced);
//   2. for each chunk of up to 16 features: vertical box sums over 2R+1 rows, one
//      (column, feature) job per thread sliding down the tile; then horizontal sums of
//      2R+1 columns by each output thread into registers;
//   3. subtract the inner window (direct, (2RI+1)^2 pixels) to get the annulus sums;
//      keep the inner mean for DWRX;
//   4. mu, C, diagonal loading lambda = load_rel tr(C)/L' (floor 1e-30), Cholesky in
//      registers (FP64), then z = L^-1 d and score = |z|^2 for d = x_p - mu (LRX, eq. 1)
//      and d = m_in - mu (DWRX, eq. 5).
// HBM traffic is the reduced cube once (the halo re-reads hit L2) and the score maps.
#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace hsad {

namespace {
constexpr int TX = 16, TY = 16, NT = TX * TY;

template <int LP> struct BoxCfg {
    static constexpr int G = LP + LP * (LP + 1) / 2;   // moment features
    static constexpr int GT = G + 1;                   // + non-finite-sample indicator
    static constexpr int GC = GT < 16 ? GT : 16;
    static constexpr int GCP = GC | 1;
    static constexpr int NCH = (GT + GC - 1) / GC;
};

// quadratic feature r (0-based, row-major over i <= j) -> (i, j)
template <int LP> __device__ __forceinline__ void quad_ij(int r, int &i, int &j)
{
    i = 0;
    int len = LP;
#pragma unroll
    for (int t = 0; t < LP; ++t) {
        if (r >= len) {
            r -= len;
            len -= 1;
            i += 1;
        }
    }
    j = i + r;
}

// px points at a sanitised tile pixel (non-finite pixels hold the reference value, so
// their moment features are 0); g == G is the non-finite indicator.
template <int LP>
__device__ __forceinline__ double feature(const float *px, float badf, const double *ref, int g)
{
    if (g < LP) return (double)px[g] - ref[g];
    if (g >= BoxCfg<LP>::G) return (double)badf;
    int i, j;
    quad_ij<LP>(g - LP, i, j);
    return ((double)px[i] - ref[i]) * ((double)px[j] - ref[j]);
}

__device__ __forceinline__ int clip_count(int c, int r, int n)
{
    int lo = c - r < 0 ? 0 : c - r;
    int hi = c + r > n - 1 ? n - 1 : c + r;
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
    double *V = smem;                                          // TY * EX * GCP
    float *xs = reinterpret_cast<float *>(smem + (size_t)TY * EX * C::GCP);   // EY*EX*LP
    float *bad = xs + (size_t)EY * EX * LP;                    // EY*EX (0/1)

    const int tid = threadIdx.x;
    const int y0 = blockIdx.y * TY, x0 = blockIdx.x * TX;

    // tile reference pixel (a finite value keeps NaN/Inf confined to their windows)
    double ref[LP];
    {
        const int ry = min(y0 + TY / 2, H - 1), rx = min(x0 + TX / 2, W - 1);
        const float *rp = x + ((size_t)ry * W + rx) * LP;
#pragma unroll
        for (int i = 0; i < LP; ++i) {
            float v = rp[i];
            ref[i] = isfinite(v) ? (double)v : 0.0;
        }
    }

    // 1. halo tile.  Pixels outside the image, and pixels with a non-finite component,
    //    take the reference value (zero features); the latter are flagged in bad[] so that
    //    a window containing one scores like the definition (see step 4).
    for (int t = tid; t < EY * EX; t += NT) {
        const int ey = t / EX, ex = t - ey * EX;
        const int gy = y0 - R + ey, gx = x0 - R + ex;
        float *dst = xs + (size_t)t * LP;
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
#pragma unroll
        for (int i = 0; i < LP; ++i) dst[i] = (ok && fin) ? v[i] : (float)ref[i];
        bad[t] = (ok && !fin) ? 1.0f : 0.0f;
    }
    __syncthreads();

    const int ty = tid / TX, tx = tid - ty * TX;
    const int py = y0 + ty, px = x0 + tx;

    // 3a. inner window, subtracted up front: S = -sum_inner (sanitised features), and
    //     the inner mean for DWRX from the raw values (non-finite values propagate)
    double S[C::GT];
    double min_sum[LP];
#pragma unroll
    for (int g = 0; g < C::GT; ++g) S[g] = 0.0;
#pragma unroll
    for (int i = 0; i < LP; ++i) min_sum[i] = 0.0;
    if (has_inner) {
        for (int dy = -RI; dy <= RI; ++dy)
            for (int dx = -RI; dx <= RI; ++dx) {
                const size_t t = (size_t)(ty + R + dy) * EX + (tx + R + dx);
                const float *pp = xs + t * LP;
                double f[LP];
#pragma unroll
                for (int i = 0; i < LP; ++i) f[i] = (double)pp[i] - ref[i];
                int g = LP;
#pragma unroll
                for (int i = 0; i < LP; ++i) {
                    S[i] -= f[i];
#pragma unroll
                    for (int j = i; j < LP; ++j) S[g++] -= f[i] * f[j];
                }
                S[C::G] -= (double)bad[t];
                const int gy = py + dy, gx = px + dx;
                if (gy >= 0 && gy < H && gx >= 0 && gx < W) {
                    const float *raw = x + ((size_t)gy * W + gx) * LP;
#pragma unroll
                    for (int i = 0; i < LP; ++i) min_sum[i] += (double)raw[i] - ref[i];
                }
            }
    }

    // 2. outer box sums, feature chunk by feature chunk
#pragma unroll
    for (int ch = 0; ch < C::NCH; ++ch) {
        const int g0 = ch * C::GC;
        const int ng = (C::GT - g0) < C::GC ? (C::GT - g0) : C::GC;
        for (int job = tid; job < EX * ng; job += NT) {
            const int gg = job / EX, c = job - gg * EX;
            const int g = g0 + gg;
            double s = 0.0;
            for (int ey = 0; ey <= 2 * R; ++ey) {
                const size_t t = (size_t)ey * EX + c;
                s += feature<LP>(xs + t * LP, bad[t], ref, g);
            }
            V[((size_t)0 * EX + c) * C::GCP + gg] = s;
            for (int r = 1; r < TY; ++r) {
                const size_t ta = (size_t)(r + 2 * R) * EX + c, tb = (size_t)(r - 1) * EX + c;
                s += feature<LP>(xs + ta * LP, bad[ta], ref, g) - feature<LP>(xs + tb * LP, bad[tb], ref, g);
                V[((size_t)r * EX + c) * C::GCP + gg] = s;
            }
        }
        __syncthreads();
        const double *vrow = V + ((size_t)ty * EX + tx) * C::GCP;
#pragma unroll
        for (int gg = 0; gg < C::GC; ++gg) {
            if (g0 + gg < C::GT) {
                double s = 0.0;
                for (int dx = 0; dx <= 2 * R; ++dx) s += vrow[(size_t)dx * C::GCP + gg];
                S[g0 + gg] += s;
            }
        }
        __syncthreads();
    }

    if (py >= H || px >= W) return;

    // 4. statistics of the annulus, loading, Cholesky, scores
    const int n_o = clip_count(py, R, H) * clip_count(px, R, W);
    const int n_i = has_inner ? clip_count(py, RI, H) * clip_count(px, RI, W) : 0;
    const double inv_na = 1.0 / (double)(n_o - n_i);
    // a non-finite sample in the annulus makes C non-finite: not positive definite (+inf),
    // as in the definition; the counts are exact integers held in FP64
    const bool ann_bad = S[C::G] > 0.5;
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
        const double inv_ni = 1.0 / (double)n_i;
        double z[LP], s = 0.0;
#pragma unroll
        for (int i = 0; i < LP; ++i) {
            double t = min_sum[i] * inv_ni - mu[i];
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
