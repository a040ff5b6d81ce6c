// chol.hip -- diagonal loading, FP64 Cholesky and the RX quadratic forms (eqs. 1 and 5)
// for the generic (matrix-core Gram) path.
//
// Each pixel's block in the chunk workspace is an (L'+2) x L' row-major FP64 matrix:
// rows 0..L'-1 hold the annulus covariance C_a and rows L', L'+1 hold the two RHS
// vectors d_lrx = x_p - mu_a and d_dwrx = m_in - mu_a.  The right-looking Cholesky is run
// over the L' columns of this trapezoid.  Its two extra rows are updated like any
// row below the diagonal, so they end as (L^-1 d)^T and the scores are their squared
// norms.  No separate triangular solve is needed.
//
// L' > 64 (chol_blk_kernel): one workgroup per pixel, columns in panels of NB = 32.  The
// panel's diagonal block is factored and inverted by one wavefront, the rows below are
// solved as a product with that inverse, and the trailing lower trapezoid is updated in
// place; both products run on the FP64 matrix cores (dev_chol.hpp, chol_pixel_blk).
// chol_rx_kernel keeps the earlier form (panel factored with one workgroup barrier per
// column, trailing update in 4 x 4 register blocks); with L' <= 32 it is a single panel in
// LDS.  Smaller L' use one wavefront per pixel (L' <= 64) or a lane group per pixel
// (L' + 2 <= 64), below.
#include <hip/hip_runtime.h>

#include "internal.hpp"
#include "dev_chol.hpp"

namespace hsad {

__global__ __launch_bounds__(256) void chol_rx_kernel(double *__restrict__ ws, int Lp, int npix,
                                                      int64_t pix0, double load_rel,
                                                      float *__restrict__ lrx,
                                                      float *__restrict__ dwrx,
                                                      const int32_t *__restrict__ idx, int64_t npix_img,
                                                      int raw, int64_t stride)
{
    extern __shared__ double sm[];
    const int local = blockIdx.x;
    if (local >= npix) return;
    const int64_t p = idx ? (int64_t)idx[pix0 + local] : pix0 + local;
    if (p < 0 || p >= npix_img) return;   // listed index outside the image: skipped
    chol_pixel(ws + (size_t)local * stride, Lp, load_rel, lrx ? lrx + p : nullptr, dwrx ? dwrx + p : nullptr, sm,
               raw);
}

// L' > 64: chol_pixel_blk (diagonal blocks by one wavefront, row solves in registers,
// trailing updates on the FP64 matrix cores)
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void chol_blk_kernel(double *__restrict__ ws, int Lp, int npix, int64_t pix0,
                                                       double load_rel, float *__restrict__ lrx,
                                                       float *__restrict__ dwrx, const int32_t *__restrict__ idx,
                                                       int64_t npix_img, int raw, int64_t stride)
{
    extern __shared__ double sm[];
    const int local = blockIdx.x;
    if (local >= npix) return;
    const int64_t p = idx ? (int64_t)idx[pix0 + local] : pix0 + local;
    if (p < 0 || p >= npix_img) return;   // listed index outside the image: skipped
    chol_pixel_blk(ws + (size_t)local * stride, Lp, load_rel, lrx ? lrx + p : nullptr, dwrx ? dwrx + p : nullptr,
                   sm, raw);
}

// one wavefront per pixel (L' <= 64), four pixels per workgroup
__global__ __launch_bounds__(256) void chol_wave_kernel(const double *__restrict__ ws, int Lp, int npix, int64_t pix0,
                                                        double load_rel, float *__restrict__ lrx,
                                                        float *__restrict__ dwrx, const int32_t *__restrict__ idx,
                                                        int64_t npix_img, int raw, int64_t stride)
{
    extern __shared__ double smw[];
    const int wv = threadIdx.x >> 6;
    const int local = blockIdx.x * 4 + wv;
    if (local >= npix) return;
    const int64_t p = idx ? (int64_t)idx[pix0 + local] : pix0 + local;
    if (p < 0 || p >= npix_img) return;   // listed index outside the image: skipped
    chol_wave_pixel(ws + (size_t)local * stride, Lp, raw, load_rel, lrx ? lrx + p : nullptr,
                    dwrx ? dwrx + p : nullptr, smw + (size_t)wv * chol_wave_lds_doubles(Lp));
}

// G lanes per pixel (register-resident rows), 256 / G pixels per workgroup
template <int G, int CB>
__global__ __launch_bounds__(256) void chol_group_kernel(const double *__restrict__ ws, int Lp, int npix, int64_t pix0,
                                                         double load_rel, float *__restrict__ lrx,
                                                         float *__restrict__ dwrx, const int32_t *__restrict__ idx,
                                                         int64_t npix_img, int raw, int64_t stride)
{
    const int local = (int)((blockIdx.x * 256 + threadIdx.x) / G);
    bool active = local < npix;
    int64_t p = 0;
    if (active) {
        p = idx ? (int64_t)idx[pix0 + local] : pix0 + local;
        active = p >= 0 && p < npix_img;    // listed index outside the image: skipped
    }
    __shared__ double colbuf[256];
    chol_group_pixel<G, CB>(ws + (size_t)(active ? local : 0) * stride, Lp, raw, load_rel, active,
                        lrx ? lrx + p : nullptr, dwrx ? dwrx + p : nullptr,
                        colbuf + (threadIdx.x & ~(G - 1)));
}

size_t chol_smem(int64_t Lp) { return chol_smem_doubles((int)Lp) * sizeof(double); }

// columns per unrolled block of the register-resident factorisation (64: fully unrolled)
static int g_chol_cb = 16;
// L' > 64: 2 = blocked factorisation (chol_pixel_blk) above kCholBlkMinLp, the panel form
// below (measured crossover at L' = 128: 29.0 ms either way at 256 x 256); 1 = blocked for every L' > 64;
// 0 = panel form only
static int g_chol_blk = 2;

int chol_launch(double *ws, int64_t Lp, int npix, int64_t pix0, double load_rel, float *lrx,
                float *dwrx, hipStream_t s, const int32_t *idx, int64_t npix_img, int raw)
{
    const int64_t stride = raw ? (Lp + 3) * Lp : (Lp + 2) * Lp;
    if (Lp + 2 <= 64) {
        const int G = Lp + 2 <= 16 ? 16 : Lp + 2 <= 32 ? 32 : 64;
        dim3 grid((unsigned)(((int64_t)npix * G + 255) / 256));
        const void *k = nullptr;
#define HSAD_CG(g, cb) \
    if (G == g && cb_sel == cb) k = (const void *)chol_group_kernel<g, cb>;
        const int cb_sel = g_chol_cb;
        HSAD_CG(16, 4) HSAD_CG(16, 8) HSAD_CG(16, 16) HSAD_CG(16, 64)
        HSAD_CG(32, 4) HSAD_CG(32, 8) HSAD_CG(32, 16) HSAD_CG(32, 64)
        HSAD_CG(64, 4) HSAD_CG(64, 8) HSAD_CG(64, 16) HSAD_CG(64, 64)
#undef HSAD_CG
        if (!k) return fail(HSAD_EINVAL, "chol_group_kernel: bad column block");
        int Lpi = (int)Lp;
        void *args[] = {&ws, &Lpi, &npix, &pix0, &load_rel, &lrx, &dwrx, (void *)&idx, &npix_img, &raw,
                        (void *)&stride};
        if (hipLaunchKernel(k, grid, dim3(256), args, 0, s) != hipSuccess)
            return fail(HSAD_EHIP, "chol_group_kernel: launch failed");
        return check_launch("chol_group_kernel");
    }
    if (Lp <= 64) {
        const size_t shw = 4 * chol_wave_lds_doubles((int)Lp) * sizeof(double);
        if (int rc = allow_lds((const void *)chol_wave_kernel, shw, "chol_wave_kernel")) return rc;
        hipLaunchKernelGGL(chol_wave_kernel, dim3((unsigned)((npix + 3) / 4)), dim3(256), shw, s, ws, (int)Lp, npix,
                           pix0, load_rel, lrx, dwrx, idx, npix_img, raw, stride);
        return check_launch("chol_wave_kernel");
    }
    const size_t sh = chol_smem(Lp);
    const int nt = Lp <= 32 ? 64 : 256;
    if (int rc = allow_lds((const void *)chol_rx_kernel, sh, "chol_rx_kernel")) return rc;
    if (g_chol_blk == 1 || (g_chol_blk == 2 && Lp >= kCholBlkMinLp)) {
        const size_t shb = chol_blk_smem_doubles((int)Lp) * sizeof(double);
        if (int rc = allow_lds((const void *)chol_blk_kernel, shb, "chol_blk_kernel")) return rc;
        hipLaunchKernelGGL(chol_blk_kernel, dim3((unsigned)npix), dim3(256), shb, s, ws, (int)Lp, npix, pix0, load_rel,
                           lrx, dwrx, idx, npix_img, raw, stride);
        return check_launch("chol_blk_kernel");
    }
    hipLaunchKernelGGL(chol_rx_kernel, dim3((unsigned)npix), dim3(nt), sh, s, ws, (int)Lp, npix,
                       pix0, load_rel, lrx, dwrx, idx, npix_img, raw, stride);
    return check_launch("chol_rx_kernel");
}

}  // namespace hsad

extern "C" int hsad_internal_chol_blk(int mode)
{
    if (mode < 0 || mode > 2) return HSAD_EINVAL;
    hsad::g_chol_blk = mode;
    return 0;
}

extern "C" int hsad_internal_chol_cb(int cb)
{
    if (cb != 4 && cb != 8 && cb != 16 && cb != 64) return HSAD_EINVAL;
    hsad::g_chol_cb = cb;
    return 0;
}
