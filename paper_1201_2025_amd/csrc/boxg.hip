// boxg.hip -- launcher of the sliding-box window statistics for mid-size L' (dev_boxg.hpp):
// one workgroup per 16 x 16 tile of a band of tile rows, raw records into the chunk
// workspace, finalised and factorised by the Cholesky kernel.
#include <hip/hip_runtime.h>

#include "internal.hpp"
#include "dev_boxg.hpp"

namespace hsad {

template <int RB>
__global__ __launch_bounds__(BG_NT) void boxg_kernel(const float *__restrict__ x, int H, int W, int Lp, int R, int RI,
                                                     int has_inner, int tile_row0, double *__restrict__ rec,
                                                     int64_t pix0, int64_t rec_stride, int resident_kb,
                                                     int inner_rec)
{
    extern __shared__ unsigned char bg_smem[];
    boxg_tile<RB>(x, H, W, Lp, R, RI, has_inner, rec, pix0, rec_stride, tile_row0 + (int)blockIdx.y,
                  (int)blockIdx.x, bg_smem, resident_kb, inner_rec);
}

// LDS budget (KiB) under which a tile keeps all its bands resident; tunable for tests
static int g_boxg_resident_kb = 156;
static int g_boxg_rb = BG_RB;     // output rows per vertical job: 2, 4 or 8 (tuning switch)
int boxg_resident_kb() { return g_boxg_resident_kb; }

bool boxg_supported(int64_t Lp, const Windows &w)
{
    return Lp >= 2 && Lp <= BG_MAX_LP && w.ro <= BG_MAX_R &&
           bg_smem_bytes((int)Lp, w.ro, g_boxg_resident_kb) <= 160 * 1024;
}

size_t boxg_record_doubles(int64_t Lp, int inner_rec) { return (size_t)((inner_rec ? 2 * Lp + 3 : Lp + 3) * Lp); }

// Records for the tile rows [tile_row0, tile_row0 + ntile_rows) into rec; record of pixel p
// at rec + (p - tile_row0 * 16 * W) * boxg_record_doubles(L', inner_rec).
int boxg_launch(const float *x, int64_t H, int64_t W, int64_t Lp, const Windows &w, int tile_row0, int ntile_rows,
                double *rec, hipStream_t s, int inner_rec)
{
    const size_t sh = bg_smem_bytes((int)Lp, w.ro, g_boxg_resident_kb);
    const void *k = g_boxg_rb == 2   ? (const void *)boxg_kernel<2>
                    : g_boxg_rb == 8 ? (const void *)boxg_kernel<8>
                                     : (const void *)boxg_kernel<4>;
    if (int rc = allow_lds(k, sh, "boxg_kernel")) return rc;
    dim3 grid((unsigned)((W + BG_TX - 1) / BG_TX), (unsigned)ntile_rows);
    int64_t pix0 = (int64_t)tile_row0 * BG_TY * W, stride = (int64_t)boxg_record_doubles(Lp, inner_rec);
    int Hi = (int)H, Wi = (int)W, Lpi = (int)Lp, ro = w.ro, ri = w.ri, hi = w.inner > 0 ? 1 : 0,
        kb = g_boxg_resident_kb, ir = inner_rec;
    void *args[] = {(void *)&x, &Hi, &Wi, &Lpi, &ro, &ri, &hi, &tile_row0, &rec, &pix0, &stride, &kb, &ir};
    if (hipLaunchKernel(k, grid, dim3(BG_NT), args, sh, s) != hipSuccess)
        return fail(HSAD_EHIP, "boxg_kernel: launch failed");
    return check_launch("boxg_kernel");
}

}  // namespace hsad

extern "C" int hsad_internal_boxg_resident_kb(int kb)
{
    hsad::g_boxg_resident_kb = kb < 0 ? 0 : kb > 156 ? 156 : kb;
    return 0;
}

extern "C" int hsad_internal_boxg_rb(int rb)
{
    if (rb != 2 && rb != 4 && rb != 8) return HSAD_EINVAL;
    hsad::g_boxg_rb = rb;
    return 0;
}
