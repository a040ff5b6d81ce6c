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

template <int PREC, int kMaxTilesPerPass>
__global__ __launch_bounds__(256) void gram_kernel(GramArgs a, int waves_per_block)
{
    extern __shared__ double lds[];
    const int wv = threadIdx.x >> 6;
    const int local = blockIdx.x * waves_per_block + wv;
    if (local >= a.npix) return;
    gram_pixel<PREC, kMaxTilesPerPass>(a, local, lds + wv * gram_wave_doubles(a.Lp, PREC));
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
    const uint32_t outer = (uint32_t)w.outer;
    a.outer_magic = (uint32_t)((((uint64_t)1 << 32) + outer - 1) / outer);
    const size_t per_wave = gram_lds_per_wave(Lp, prec);
    int wpb = 4;
    while (wpb > 1 && per_wave * wpb > 64 * 1024) wpb >>= 1;
    const size_t sh = per_wave * wpb;
    if (sh > 160 * 1024) return fail(HSAD_EUNSUPPORTED, "gram: L' too large for LDS staging");
    dim3 grid((unsigned)((npix + wpb - 1) / wpb)), block(64 * wpb);
    const int T = (int)((Lp + 15) / 16);
    const int ntiles = T * (T + 1) / 2;
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
