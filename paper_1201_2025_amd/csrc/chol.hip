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
// One workgroup per pixel.  Columns are processed in panels of NB = 32.  A panel
// (all rows from the panel down) is factored in LDS, written back, and applied to the
// trailing lower trapezoid with 4 x 4 register blocks per thread.  The trailing part
// stays in the workspace, which is L2-resident for a chunk.  With L' <= 32 this is a
// single panel and the whole factorisation runs in LDS.
#include <hip/hip_runtime.h>

#include "internal.hpp"
#include "dev_chol.hpp"

namespace hsad {

__global__ __launch_bounds__(256) void chol_rx_kernel(double *__restrict__ ws, int Lp, int npix,
                                                      int64_t pix0, double load_rel,
                                                      float *__restrict__ lrx,
                                                      float *__restrict__ dwrx,
                                                      const int32_t *__restrict__ idx, int64_t npix_img)
{
    extern __shared__ double sm[];
    const int local = blockIdx.x;
    if (local >= npix) return;
    const int64_t p = idx ? (int64_t)idx[pix0 + local] : pix0 + local;
    if (p < 0 || p >= npix_img) return;   // listed index outside the image: skipped
    chol_pixel(ws + (size_t)local * (Lp + 2) * Lp, Lp, load_rel, lrx ? lrx + p : nullptr,
               dwrx ? dwrx + p : nullptr, sm);
}

size_t chol_smem(int64_t Lp) { return chol_smem_doubles((int)Lp) * sizeof(double); }

int chol_launch(double *ws, int64_t Lp, int npix, int64_t pix0, double load_rel, float *lrx,
                float *dwrx, hipStream_t s, const int32_t *idx, int64_t npix_img)
{
    const size_t sh = chol_smem(Lp);
    const int nt = Lp <= 32 ? 64 : 256;
    if (int rc = allow_lds((const void *)chol_rx_kernel, sh, "chol_rx_kernel")) return rc;
    hipLaunchKernelGGL(chol_rx_kernel, dim3((unsigned)npix), dim3(nt), sh, s, ws, (int)Lp, npix,
                       pix0, load_rel, lrx, dwrx, idx, npix_img);
    return check_launch("chol_rx_kernel");
}

}  // namespace hsad
