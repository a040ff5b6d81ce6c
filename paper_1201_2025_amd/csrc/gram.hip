// gram.hip -- per-pixel window statistics on matrix cores, for any L' (up to 512).
//
// One wavefront owns one pixel.  Its background is the annulus A = outer \ inner (Sec. 2.1,
// Sec. 2.2), clipped to the image.  Two passes follow the exact two-pass definition:
//   pass 1: mu_a = mean over A, m_in = mean over the inner window (FP64 accumulation);
//   pass 2: C = sum_A (x - mu_a)(x - mu_a)^T as an MFMA Gram, C_a = C / n_a.
// In DWEST mode the inner samples enter the same accumulator with weight 1/n_in and the
// annulus samples with weight -1/n_a.  The accumulator then holds C_diff = C_inner -
// C_outer (eq. 2) directly.
//
// MFMA mapping (16 x 16 output tiles, K = samples): for a group of samples the lane
// (c = lane & 15, g = lane >> 4) supplies component 16*b + c of sample g (FP64/FP32,
// K = 4) or of samples 8g..8g+7 (BF16/FP16, K = 32).  This is the same value for the
// A (= X^T) and B (= X) operand of a tile, so any k-ordering the hardware uses gives
// the same sum.  Output element e of lane l is row 4*(l>>4)+e, column l&15 for the
// FP32/BF16/FP16 instructions and row 4*e+(l>>4) for the FP64 one (measured on gfx950).
//
// The per-lane centred samples are staged in LDS, which serves as a runtime-indexed
// register file; each lane reads only its own slots, so no synchronisation is needed.
// Output per pixel into the chunk workspace (double, row-major, (L'+2) rows x L'):
//   LRX mode  : rows 0..L'-1 = C_a, row L' = x_p - mu_a, row L'+1 = m_in - mu_a
//   DWEST mode: rows 0..L'-1 = C_diff, row L' = m_in - mu_a (eq. 3)
#include <hip/hip_runtime.h>

#include "dev_gram.hpp"

namespace hsad {

// smallest tile count T = ceil(L'/16) that takes the workgroup-per-pixel FP64 Gram, and its
// most accumulator tiles per wavefront and pass: 9, three waves per SIMD (at L' = 224 three
// passes: 285.5 ms per full band against 298.8 with two passes of 14 at two waves per SIMD;
// tests choose through hsad_internal_gram_wg)
static int g_gram_wg_min_t = 6;
// contiguous chunks take their means from gram_means_kernel (0: the kernel's own first pass)
static int g_gram_means = 1;
static int g_gram_wg_tiles = 9;

template <int PREC, int kMaxTilesPerPass>
__global__ __launch_bounds__(256) void gram_kernel(GramArgs a, int waves_per_block)
{
    extern __shared__ double lds[];
    const int wv = threadIdx.x >> 6;
    const int local = blockIdx.x * waves_per_block + wv;
    if (local >= a.npix) return;
    gram_pixel<PREC, kMaxTilesPerPass>(a, local, lds + wv * gram_wave_doubles(a.Lp, PREC));
}

// ------------------------------------------------------------------------------------
// Workgroup per pixel (FP64, LRX mode, 81 <= L' <= 256).  A pixel's annulus Gram has
// T(T+1)/2 tiles of 16 x 16 (105 at L' = 224), more than one wavefront can keep in
// registers, so the per-wavefront kernel above re-reads every window sample once per pass
// of 16 tiles.  Here the four wavefronts of a workgroup share each group of 4 centred
// samples through LDS (staged once per group for all bands) and split the tiles, MT
// accumulators per wavefront and pass.  Groups are staged two at a time (one barrier per
// pair), each pair fetched into registers two pairs ahead of use (two LDS buffers).  Definitions as in
// gram_pixel: FP64 means first (all threads, band-parallel partial sums), then the Gram
// of the exactly centred annulus samples, scaled by 1/n_a.
// The tiles are written through an LDS transpose so that both triangles are stored in
// rows of 16 consecutive doubles.
// LDS: mu, m_in [256] doubles; two staging buffers [2][4][Lpad + 16] doubles (also the
// partial sums of the means and the transposes); sample table [4 ceil(K/4)] ints (annulus:
// pixel index, inner window: -2 - pixel index, outside the image or past K: -1).
// ------------------------------------------------------------------------------------
static constexpr int kWgMaxLpad = 256;
// row stride of a staged group (doubles): Lpad + 16 puts the four sample rows a matrix-core
// operand read spans 32 banks apart, so each half-wavefront reads 64 distinct banks
static constexpr int kWgStageLd = kWgMaxLpad + 16;

// groups of 4 samples staged per barrier
static constexpr int kWgGroups = 2;

__host__ __device__ inline size_t gram_wg_lds_bytes(int K)
{
    const size_t nsg = ((size_t)(K + 3) / 4 + kWgGroups - 1) / kWgGroups;
    return ((size_t)2 * kWgMaxLpad + 8 * (size_t)kWgGroups * kWgStageLd) * sizeof(double) +
           (size_t)4 * kWgGroups * nsg * sizeof(int);
}

// FP64 annulus and inner-window means of the chunk's pixels pix0 .. pix0 + npix - 1, into
// rows L' and L'+1 of each pixel's record (what the workgroup kernel's first pass computes,
// as the plain sums of the definition: FP32 samples added in FP64).  One thread per (pixel,
// band), bands fastest, so a wavefront's loads of a window sample are consecutive floats.
__global__ __launch_bounds__(256) void gram_means_kernel(GramArgs a)
{
    const int64_t gt = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int Lp = a.Lp;
    if (gt >= (int64_t)a.npix * Lp) return;
    const int local = (int)(gt / Lp), b = (int)(gt - (int64_t)local * Lp);
    const int64_t pix = a.pix0 + local;
    const int py = (int)(pix / a.W), px = (int)(pix - (int64_t)py * a.W);
    const int y0 = py - a.R < 0 ? 0 : py - a.R, y1 = py + a.R > a.H - 1 ? a.H - 1 : py + a.R;
    const int x0 = px - a.R < 0 ? 0 : px - a.R, x1 = px + a.R > a.W - 1 ? a.W - 1 : px + a.R;
    double sa = 0.0, si = 0.0;
    for (int y = y0; y <= y1; ++y) {
        const bool iny = a.has_inner && y - py <= a.RI && py - y <= a.RI;
        const float *row = a.x + (size_t)y * a.W * Lp + b;
#pragma unroll 4
        for (int xx = x0; xx <= x1; ++xx) {
            const double v = (double)row[(size_t)xx * Lp];
            const bool inn = iny && xx - px <= a.RI && px - xx <= a.RI;
            sa += inn ? 0.0 : v;
            si += inn ? v : 0.0;
        }
    }
    const int n_o = clipn(py, a.R, a.H) * clipn(px, a.R, a.W);
    const int n_i = a.has_inner ? clipn(py, a.RI, a.H) * clipn(px, a.RI, a.W) : 0;
    double *out = a.ws + (size_t)local * (Lp + 2) * Lp;
    out[(size_t)Lp * Lp + b] = sa / (double)(n_o - n_i);
    out[(size_t)(Lp + 1) * Lp + b] = n_i > 0 ? si / (double)n_i : 0.0;
}

template <int MT, int WPE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WPE, WPE))) void gram_wg_kernel(GramArgs a)
{
    extern __shared__ double sm[];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int Lp = a.Lp, T = (Lp + 15) >> 4, Lpad = 16 * T, LS = Lpad + 16;
    double *mu = sm, *mi = sm + kWgMaxLpad, *buf = sm + 2 * kWgMaxLpad;
    const int local = blockIdx.x;
    if (local >= a.npix) return;
    const int64_t pix = a.idx ? (int64_t)a.idx[a.pix0 + local] : a.pix0 + local;
    if (pix < 0 || pix >= (int64_t)a.H * a.W) return;   // uniform over the workgroup
    const int py = (int)(pix / a.W), px = (int)(pix - (int64_t)py * a.W);
    const int K = (2 * a.R + 1) * (2 * a.R + 1);
    const int ng = (K + 3) / 4;
    constexpr int GPB = kWgGroups;
    const int nsg = (ng + GPB - 1) / GPB;   // staged units of GPB groups
    const int n_o = clipn(py, a.R, a.H) * clipn(px, a.R, a.W);
    const int n_i = a.has_inner ? clipn(py, a.RI, a.H) * clipn(px, a.RI, a.W) : 0;
    const int n_a = n_o - n_i;
    int *sof = reinterpret_cast<int *>(sm + 2 * kWgMaxLpad + 8 * GPB * kWgStageLd);
    for (int k = tid; k < 4 * GPB * nsg; k += 256) {
        int v = -1;
        if (k < K) {
            int sy, sx;
            bool inn;
            if (sample_pos(a, py, px, k, sy, sx, inn)) {
                const int q = sy * a.W + sx;
                v = inn ? -2 - q : q;
            }
        }
        sof[k] = v;
    }
    // the thread's staged elements e = tid + 256 i: sample e / Lpad of the group, band e % Lpad
    constexpr int NE = 4 * kWgMaxLpad / 256;
    const int nel = 4 * Lpad;
    int es[NE], eb[NE], eo[NE];
    bool ev[NE];
#pragma unroll
    for (int i = 0; i < NE; ++i) {
        const int e = tid + 256 * i;
        es[i] = e < nel ? e / Lpad : 0;
        eb[i] = e < nel ? e - es[i] * Lpad : 0;
        eo[i] = es[i] * LS + eb[i];   // staging offset (padding bands keep their own cell)
        ev[i] = e < nel && eb[i] < Lp;
        if (eb[i] >= Lp) eb[i] = Lp - 1;   // clamped band: loads stay in the row, value dropped
    }
    __syncthreads();

    double *out = a.ws + (size_t)local * (Lp + 2) * Lp;
    if (a.means_ready) {
        // the means were written into rows L' (annulus) and L'+1 (inner window) beforehand
        for (int b = tid; b < Lpad; b += 256) {
            mu[b] = b < Lp ? out[(size_t)Lp * Lp + b] : 0.0;
            mi[b] = b < Lp ? out[(size_t)(Lp + 1) * Lp + b] : 0.0;
        }
    } else {
    // pass 1: FP64 sums over the annulus and the inner window
    {
        double sa[NE], si[NE];
#pragma unroll
        for (int i = 0; i < NE; ++i) sa[i] = si[i] = 0.0;
#pragma unroll 8
        for (int g = 0; g < ng; ++g) {
#pragma unroll
            for (int i = 0; i < NE; ++i) {
                const int o = sof[4 * g + es[i]];
                const int q = o >= 0 ? o : o <= -2 ? -2 - o : 0;
                const double v = (double)a.x[(size_t)q * Lp + eb[i]];
                sa[i] += ev[i] && o >= 0 ? v : 0.0;
                si[i] += ev[i] && o <= -2 ? v : 0.0;
            }
        }
#pragma unroll
        for (int i = 0; i < NE; ++i) {
            const int e = tid + 256 * i;
            if (e < nel) {
                buf[e] = sa[i];
                buf[4 * kWgMaxLpad + e] = si[i];
            }
        }
    }
    __syncthreads();
    for (int b = tid; b < Lpad; b += 256) {
        const double sa = (buf[b] + buf[Lpad + b]) + (buf[2 * Lpad + b] + buf[3 * Lpad + b]);
        const double *bi = buf + 4 * kWgMaxLpad;
        const double si = (bi[b] + bi[Lpad + b]) + (bi[2 * Lpad + b] + bi[3 * Lpad + b]);
        mu[b] = b < Lp ? sa / (double)n_a : 0.0;
        mi[b] = (b < Lp && n_i > 0) ? si / (double)n_i : 0.0;
    }
    }
    __syncthreads();
    for (int b = tid; b < Lp; b += 256) {
        out[(size_t)Lp * Lp + b] = (double)a.x[(size_t)pix * Lp + b] - mu[b];
        out[(size_t)(Lp + 1) * Lp + b] = mi[b] - mu[b];
    }
    double emu[NE];
#pragma unroll
    for (int i = 0; i < NE; ++i) emu[i] = mu[eb[i]];

    // pass 2: the Gram, MT tiles per wavefront per pass (tile t = wv + 4 m, row-major over
    // the upper triangle bi <= bj)
    const int ntiles = T * (T + 1) / 2;
    const int nper = (ntiles + 3) / 4;
    const int c16 = lane & 15, g4 = lane >> 4;
    const double scale = 1.0 / (double)n_a;
    double *tw = buf + wv * (16 * 17);   // this wavefront's transpose tile (after the loop)
    for (int m0 = 0; m0 < nper; m0 += MT) {
        int tb[MT];   // 16 bi | (16 bj) << 16, wave-uniform
#pragma unroll
        for (int m = 0; m < MT; ++m) {
            int t = wv + 4 * (m0 + m), bi = 0;
            t = t < ntiles ? t : 0;
            while (t >= T - bi) {
                t -= T - bi;
                ++bi;
            }
            tb[m] = 16 * bi | (16 * (bi + t)) << 16;
        }
        f64x4 acc[MT];
#pragma unroll
        for (int m = 0; m < MT; ++m)
            for (int e = 0; e < 4; ++e) acc[m][e] = 0.0;
        // unit u (groups GPB u .. GPB u + GPB - 1): fetched into registers two units before
        // it is staged, so that each load has two units of matrix-core work to arrive
        float xa[GPB * NE], xb[GPB * NE];
        bool ka[GPB * NE], kb[GPB * NE];
        auto fetch = [&](int u, float *xv, bool *xok) {
#pragma unroll
            for (int gi = 0; gi < GPB; ++gi)
#pragma unroll
                for (int i = 0; i < NE; ++i) {
                    const int o = sof[4 * (GPB * u + gi) + es[i]];
                    xv[gi * NE + i] = a.x[(size_t)(o >= 0 ? o : 0) * Lp + eb[i]];
                    xok[gi * NE + i] = ev[i] && o >= 0;
                }
        };
        auto stage = [&](double *dst, const float *xv, const bool *xok) {
#pragma unroll
            for (int gi = 0; gi < GPB; ++gi)
#pragma unroll
                for (int i = 0; i < NE; ++i) {
                    const int e = tid + 256 * i;
                    if (e < nel)
                        dst[gi * 4 * LS + eo[i]] = xok[gi * NE + i] ? (double)xv[gi * NE + i] - emu[i] : 0.0;
                }
        };
        auto mfma_unit = [&](const double *b) {
#pragma unroll
            for (int gi = 0; gi < GPB; ++gi) {
                const double *cur = b + gi * 4 * LS + g4 * LS + c16;
#pragma unroll
                for (int m = 0; m < MT; ++m)
                    if (m0 + m < nper && wv + 4 * (m0 + m) < ntiles)
                        acc[m] = __builtin_amdgcn_mfma_f64_16x16x4f64(cur[tb[m] & 0xffff], cur[tb[m] >> 16], acc[m],
                                                                      0, 0, 0);
            }
        };
        double *buf0 = buf, *buf1 = buf + GPB * 4 * kWgStageLd;
        fetch(0, xa, ka);
        __syncthreads();   // readers of the buffers (means, previous pass) are done
        stage(buf0, xa, ka);
        if (1 < nsg) fetch(1, xb, kb);
        if (2 < nsg) fetch(2, xa, ka);
        __syncthreads();
        // even steps: unit u in buf0, unit u+1 (xb) staged to buf1, unit u+3 fetched to xb;
        // odd steps mirror with buf1 / xa
        for (int u = 0; u < nsg; u += 2) {
            mfma_unit(buf0);
            if (u + 1 < nsg) stage(buf1, xb, kb);
            if (u + 3 < nsg) fetch(u + 3, xb, kb);
            __syncthreads();
            if (u + 1 >= nsg) break;
            mfma_unit(buf1);
            if (u + 2 < nsg) stage(buf0, xa, ka);
            if (u + 4 < nsg) fetch(u + 4, xa, ka);
            __syncthreads();
        }
        // write the tiles: the upper triangle straight from the accumulators, the lower
        // through the transpose (diagonal tiles: one value per symmetric pair)
#pragma unroll
        for (int m = 0; m < MT; ++m) {
            if (!(m0 + m < nper && wv + 4 * (m0 + m) < ntiles)) continue;
            const int r0 = tb[m] & 0xffff, c0 = tb[m] >> 16;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                // FP64 16x16x4: element e of lane l sits at row 4e + (l >> 4), column l & 15
                const int rl = 4 * e + g4;
                const double v = acc[m][e] * scale;
                tw[rl * 17 + c16] = v;
                if (r0 + rl < Lp && c0 + c16 < Lp && (r0 < c0 || rl <= c16))
                    out[(size_t)(r0 + rl) * Lp + c0 + c16] = v;
            }
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                // row c0 + jl of the lower triangle, column r0 + c16
                const int jl = 4 * e + g4;
                const double v = tw[c16 * 17 + jl];
                if (c0 + jl < Lp && r0 + c16 < Lp && (r0 < c0 || c16 <= jl))
                    out[(size_t)(c0 + jl) * Lp + r0 + c16] = v;
            }
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        }
    }
}

size_t gram_lds_per_wave(int64_t Lp, int prec)
{
    const int64_t T = (Lp + 15) / 16;
    const int64_t stage = T * 64 * ((prec == GP_BF16 || prec == GP_FP16) ? 2 : 1);
    return (size_t)(stage + 2 * T * 16) * sizeof(double);
}

int gram_launch(const float *x, int64_t H, int64_t W, int64_t Lp, const Windows &w, int mode,
                int prec, int64_t pix0, int npix, double *ws, hipStream_t s, const int32_t *idx)
{
    GramArgs a;
    a.idx = idx;
    a.x = x;
    a.H = (int)H;
    a.W = (int)W;
    a.Lp = (int)Lp;
    a.R = w.ro;
    a.RI = w.ri;
    a.has_inner = w.inner > 0;
    a.mode = mode;
    a.pix0 = pix0;
    a.npix = npix;
    a.ws = ws;
    a.means_ready = 0;
    const uint32_t outer = (uint32_t)w.outer;
    a.outer_magic = (uint32_t)((((uint64_t)1 << 32) + outer - 1) / outer);
    const int T = (int)((Lp + 15) / 16);
    const int ntiles = T * (T + 1) / 2;
    if (prec == GP_FP64 && mode == GRAM_LRX && T >= g_gram_wg_min_t && 16 * T <= kWgMaxLpad) {
        // long spectra: one workgroup per pixel, samples staged once per pass for all tiles
        const size_t shw = gram_wg_lds_bytes(w.outer * w.outer);
        const int nper = (ntiles + 3) / 4;
        const int npass = (nper + g_gram_wg_tiles - 1) / g_gram_wg_tiles;
        const int need = (nper + npass - 1) / npass;
        const void *k = need <= 6    ? (const void *)gram_wg_kernel<6, 2>
                        : need <= 9  ? (const void *)gram_wg_kernel<9, 3>
                        : need <= 12 ? (const void *)gram_wg_kernel<12, 2>
                        : need <= 14 ? (const void *)gram_wg_kernel<14, 2>
                        : need <= 17 ? (const void *)gram_wg_kernel<17, 2>
                        : need <= 22 ? (const void *)gram_wg_kernel<22, 1>
                                     : (const void *)gram_wg_kernel<28, 1>;
        if (int rc = allow_lds(k, shw, "gram_wg_kernel")) return rc;
        if (!idx && g_gram_means) {
            // contiguous chunk: the means by their own kernel, one thread per (pixel, band)
            const int64_t nt = (int64_t)npix * Lp;
            hipLaunchKernelGGL(gram_means_kernel, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, s, a);
            if (int rc = check_launch("gram_means_kernel")) return rc;
            a.means_ready = 1;
        }
        void *args[] = {&a};
        if (hipLaunchKernel(k, dim3((unsigned)npix), dim3(256), args, shw, s) != hipSuccess)
            return fail(HSAD_EHIP, "gram_wg_kernel: launch failed");
        return check_launch("gram_wg_kernel");
    }
    const size_t per_wave = gram_lds_per_wave(Lp, prec);
    int wpb = 4;
    while (wpb > 1 && per_wave * wpb > 64 * 1024) wpb >>= 1;
    const size_t sh = per_wave * wpb;
    if (sh > 160 * 1024) return fail(HSAD_EUNSUPPORTED, "gram: L' too large for LDS staging");
    dim3 grid((unsigned)((npix + wpb - 1) / wpb)), block(64 * wpb);
    const int mt = ntiles <= 1 ? 1 : ntiles <= 3 ? 3 : ntiles <= 6 ? 6 : ntiles <= 10 ? 10 : 16;
    int rc = HSAD_OK;
#define HSAD_GRAM_LAUNCH(P, M)                                                                   \
    do {                                                                                         \
        if ((rc = allow_lds((const void *)gram_kernel<P, M>, sh, "gram_kernel"))) return rc;     \
        hipLaunchKernelGGL((gram_kernel<P, M>), grid, block, sh, s, a, wpb);                     \
    } while (0)
#define HSAD_GRAM_MT(P)                                                                          \
    switch (mt) {                                                                                \
    case 1: HSAD_GRAM_LAUNCH(P, 1); break;                                                       \
    case 3: HSAD_GRAM_LAUNCH(P, 3); break;                                                       \
    case 6: HSAD_GRAM_LAUNCH(P, 6); break;                                                       \
    case 10: HSAD_GRAM_LAUNCH(P, 10); break;                                                     \
    default: HSAD_GRAM_LAUNCH(P, 16); break;                                                     \
    }
    switch (prec) {
    case GP_FP64: HSAD_GRAM_MT(0); break;
    case GP_FP32: HSAD_GRAM_MT(1); break;
    case GP_BF16: HSAD_GRAM_MT(2); break;
    default: HSAD_GRAM_MT(3); break;
    }
#undef HSAD_GRAM_MT
#undef HSAD_GRAM_LAUNCH
    return check_launch("gram_kernel");
}

}  // namespace hsad

// min_t: smallest T = ceil(L'/16) taking the workgroup kernel (< 1: never); tiles: most
// accumulator tiles per wavefront and pass (6..28)
extern "C" int hsad_internal_gram_means(int on)
{
    hsad::g_gram_means = on != 0;
    return 0;
}

extern "C" int hsad_internal_gram_wg(int min_t, int tiles)
{
    if (tiles < 6 || tiles > 28) return HSAD_EINVAL;
    hsad::g_gram_wg_min_t = min_t < 1 ? 1 << 20 : min_t;
    hsad::g_gram_wg_tiles = tiles;
    return 0;
}
