// generic.hip -- chunked orchestration of the matrix-core path: Gram -> Cholesky (LRX,
// DWRX) or Gram -> Jacobi (DWEST).  Pixels are processed in chunks that fit the caller's
// workspace; each chunk is two launches on the caller's stream.
#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace hsad {

size_t gram_lds_per_wave(int64_t Lp, int prec);
int gram_launch(const float *x, int64_t H, int64_t W, int64_t Lp, const Windows &w, int mode,
                int prec, int64_t pix0, int npix, double *ws, hipStream_t s,
                const int32_t *idx = nullptr);
size_t chol_smem(int64_t Lp);
int chol_launch(double *ws, int64_t Lp, int npix, int64_t pix0, double load_rel, float *lrx,
                float *dwrx, hipStream_t s, const int32_t *idx, int64_t npix_img, int raw);
int boxg_launch(const float *x, int64_t H, int64_t W, int64_t Lp, const Windows &w, int tile_row0, int ntile_rows,
                double *rec, hipStream_t s, int inner_rec = 0);
size_t jacobi_smem(int64_t n);
size_t eig_smem(int64_t n);
int eig_dwest_launch(double *ws, int64_t n, int npix, int64_t pix0, float *score, float *literal,
                     int32_t *npos, hipStream_t s, int raw = 0);
int tridiag_dwest_launch(double *ws, int64_t n, int npix, double *dey, int64_t S, hipStream_t s, int raw = 0);
int ql_dwest_global_launch(double *dey, int64_t n, int64_t S, int64_t pix0, float *score, float *literal,
                           int32_t *npos, hipStream_t s);
int ql_lds_pixels(int64_t n);
// Householder + implicit QL, 0: per chunk with LDS columns or over runs of pixels with
// global columns, whichever suits L' and the chunk size; 2: per chunk (also the
// small-workspace fallback); 3: over runs.  1: cyclic Jacobi.
static int g_dwest_solver = 0;
int jacobi_launch(const double *ws, int64_t n, int npix, int64_t pix0, float *score,
                  float *literal, int32_t *npos, hipStream_t s);

size_t generic_ws_per_pixel(int64_t Lp, GramMode)
{
    return (size_t)((Lp + 2) * Lp) * sizeof(double);
}

// Pixels per chunk.  A chunk's workspace is written by the Gram kernel and read back by
// the factorisation right after.  Up to 192 MiB it stays in the 256 MB Infinity Cache,
// but a chunk also needs about 8192 pixels (one wavefront each) to fill the 256 CUs.
// The cap is the larger of the two.
static int64_t chunk_pixels(int64_t total, int64_t Lp, size_t ws_bytes)
{
    const int64_t per = (int64_t)generic_ws_per_pixel(Lp, GRAM_LRX);
    int64_t P = (int64_t)(ws_bytes / per);
    int64_t cap = ((int64_t)192 << 20) / per;
    if (cap < 8192) cap = 8192;
    if (P > cap) P = cap;
    if (P > total) P = total;
    if (P > (1 << 30)) P = 1 << 30;
    return P;
}

// Tile-row bands per chunk of the box-statistics path: as many as the workspace holds, at
// most what keeps ~4096 tiles (16 per CU) in flight, within 8 GiB of records.
int64_t boxg_chunk_bands(int64_t H, int64_t W, int64_t Lp, size_t ws_bytes, int inner_rec)
{
    const int64_t band_bytes = (int64_t)(boxg_record_doubles(Lp, inner_rec) * sizeof(double)) * 16 * W;
    const int64_t total = (H + 15) / 16, tiles_per_band = (W + 15) / 16;
    int64_t want = (4096 + tiles_per_band - 1) / tiles_per_band;
    const int64_t cap = ((int64_t)8 << 30) / band_bytes;
    if (want > cap) want = cap > 1 ? cap : 1;
    if (want > total) want = total;
    int64_t fit = (int64_t)(ws_bytes / (size_t)band_bytes);
    return fit < want ? fit : want;
}

// -1 automatic, 1 matrix-core Gram only (tests compare the two statistics paths)
static int g_generic_force = -1;

int generic_lrx_dwrx(const float *x, int64_t H, int64_t W, int64_t Lp, const Windows &w,
                     double load_rel, GramPrec prec, float *lrx, float *dwrx, void *ws,
                     size_t ws_bytes, hipStream_t s)
{
    // exact statistics by sliding box sums when they fit (raw records, finalised by the
    // Cholesky kernel); otherwise the per-pixel matrix-core Gram
    if (prec == GP_FP64 && g_generic_force != 1 && boxg_supported(Lp, w)) {
        const int64_t bands = boxg_chunk_bands(H, W, Lp, ws_bytes);
        if (bands >= 1) {
            double *recs = (double *)ws;
            const int64_t total = (H + 15) / 16;
            for (int64_t b0 = 0; b0 < total; b0 += bands) {
                const int64_t nb = total - b0 < bands ? total - b0 : bands;
                int rc = boxg_launch(x, H, W, Lp, w, (int)b0, (int)nb, recs, s);
                if (rc) return rc;
                const int64_t y1 = (b0 + nb) * 16 < H ? (b0 + nb) * 16 : H;
                const int64_t p0 = b0 * 16 * W, n = y1 * W - p0;
                rc = chol_launch(recs, Lp, (int)n, p0, load_rel, lrx, dwrx, s, nullptr, H * W, 1);
                if (rc) return rc;
            }
            return HSAD_OK;
        }
    }
    if (gram_lds_per_wave(Lp, prec) > 160 * 1024 || chol_smem(Lp) > 160 * 1024)
        return fail(HSAD_EUNSUPPORTED, "generic path: L' too large");
    const int64_t total = H * W;
    const int64_t P = chunk_pixels(total, Lp, ws_bytes);
    if (P < 1) return fail(HSAD_ENOMEM, "generic path: workspace below one pixel");
    for (int64_t p0 = 0; p0 < total; p0 += P) {
        const int n = (int)((total - p0) < P ? (total - p0) : P);
        int rc = gram_launch(x, H, W, Lp, w, GRAM_LRX, prec, p0, n, (double *)ws, s);
        if (rc) return rc;
        rc = chol_launch((double *)ws, Lp, n, p0, load_rel, lrx, dwrx, s, nullptr, H * W, 0);
        if (rc) return rc;
    }
    return HSAD_OK;
}

// LRX / DWRX at a list of pixels (flat y * W + x); outputs written only there.
int generic_lrx_dwrx_at(const float *x, int64_t H, int64_t W, int64_t Lp, const Windows &w,
                        double load_rel, GramPrec prec, const int32_t *idx, int64_t nidx, float *lrx,
                        float *dwrx, void *ws, size_t ws_bytes, hipStream_t s)
{
    if (gram_lds_per_wave(Lp, prec) > 160 * 1024 || chol_smem(Lp) > 160 * 1024)
        return fail(HSAD_EUNSUPPORTED, "generic path: L' too large");
    const int64_t P = chunk_pixels(nidx, Lp, ws_bytes);
    if (P < 1) return fail(HSAD_ENOMEM, "generic path: workspace below one pixel");
    for (int64_t p0 = 0; p0 < nidx; p0 += P) {
        const int n = (int)((nidx - p0) < P ? (nidx - p0) : P);
        int rc = gram_launch(x, H, W, Lp, w, GRAM_LRX, prec, p0, n, (double *)ws, s, idx);
        if (rc) return rc;
        rc = chol_launch((double *)ws, Lp, n, p0, load_rel, lrx, dwrx, s, idx, H * W, 0);
        if (rc) return rc;
    }
    return HSAD_OK;
}

// DWEST runs: the tridiagonal form of every pixel of a run (up to kQlRun pixels) is kept in
// global columns (d, e, y: 3 L' doubles per pixel, pixel-minor) so that one QL launch holds
// the whole run, a lane per pixel.  Per chunk (8192 pixels at mid L') that launch would be
// one half-empty wavefront per CU.
static constexpr int64_t kQlRun = (int64_t)1 << 20;

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Pixels of a run the workspace allows beside the chunk records (0: too small, use the
// per-chunk path).  Records for a chunk are reserved first: 8192 pixels, or what 1 GiB
// holds for long spectra (the record cap of the reported workspace).  A run shorter than
// 8192 pixels is taken only when it covers the whole image.
static int64_t ql_run_pixels(int64_t total, int64_t Lp, size_t ws_bytes)
{
    const size_t col = (size_t)(3 * Lp) * sizeof(double), rec = generic_ws_per_pixel(Lp, GRAM_DWEST);
    const int64_t cap = total < kQlRun ? total : kQlRun;
    int64_t rp = 8192;
    const int64_t rcap = (int64_t)(((size_t)1 << 30) / rec);
    if (rp > rcap) rp = rcap > 0 ? rcap : 1;
    if (rp > total) rp = total;
    if (ws_bytes < 256 + rec * (size_t)rp + col) return 0;
    int64_t S = (int64_t)((ws_bytes - 256 - rec * (size_t)rp) / col);
    if (S > cap) S = cap;
    return S < cap && S < 8192 ? 0 : S;
}

// Tile rows per DWEST run on the box-statistics path (a run is a whole number of tile rows).
static int64_t dwest_run_rows(int64_t H, int64_t W)
{
    const int64_t ntr = (H + 15) / 16;
    int64_t rt = kQlRun / (16 * W);
    if (rt < 1) rt = 1;
    return rt < ntr ? rt : ntr;
}

size_t dwest_ws_bytes(int64_t H, int64_t W, int64_t Lp, const Windows &w)
{
    const int64_t total = H * W;
    const size_t rec = generic_ws_per_pixel(Lp, GRAM_DWEST);
    size_t want = rec * (size_t)total;
    const size_t cap = (size_t)1 << 30;
    if (want > cap) want = (cap / rec) * rec;
    const int64_t S = total < kQlRun ? total : kQlRun;
    size_t bytes = align256((size_t)(3 * Lp) * sizeof(double) * (size_t)S) + want;
    if (boxg_supported(Lp, w)) {
        // box statistics: the columns of one run of tile rows and records for the bands
        const int64_t rt = dwest_run_rows(H, W);
        int64_t bands = boxg_chunk_bands(H, W, Lp, (size_t)-1 / 2, 1);
        if (bands > rt) bands = rt;
        const int64_t rows = rt * 16 < H ? rt * 16 : H;
        const size_t b2 = align256((size_t)(3 * Lp) * sizeof(double) * (size_t)(rows * W)) +
                          (size_t)bands * 16 * (size_t)W * boxg_record_doubles(Lp, 1) * sizeof(double);
        if (b2 > bytes) bytes = b2;
    }
    return bytes;
}

static int g_dwest_stats = 0;   // 0: box statistics where supported, 1: matrix-core Gram (tests)

// DWEST from box statistics: the box kernel writes, per band of tile rows, records with the
// annulus and the inner-window moments; the tridiagonalisation forms C_diff from them.
// Returns 1 when the workspace is too small for this path (the caller takes the Gram path).
static int dwest_boxg(const float *x, int64_t H, int64_t W, int64_t Lp, const Windows &w, float *score,
                      float *literal, int32_t *npos, void *ws, size_t ws_bytes, hipStream_t s)
{
    const int64_t total = H * W, ntr = (H + 15) / 16;
    const int64_t all_bands = boxg_chunk_bands(H, W, Lp, ws_bytes, 1);
    const bool chunk_first = g_dwest_solver == 2 ||
                             (g_dwest_solver == 0 && ql_lds_pixels(Lp) == 64 &&
                              all_bands * 16 * W >= (total < 65536 ? total : 65536));
    if (chunk_first) {
        if (all_bands < 1) return 1;
        double *recs = (double *)ws;
        for (int64_t b0 = 0; b0 < ntr; b0 += all_bands) {
            const int64_t nb = ntr - b0 < all_bands ? ntr - b0 : all_bands;
            int rc = boxg_launch(x, H, W, Lp, w, (int)b0, (int)nb, recs, s, 1);
            if (rc) return rc;
            const int64_t y1 = (b0 + nb) * 16 < H ? (b0 + nb) * 16 : H;
            const int64_t p0 = b0 * 16 * W, n = y1 * W - p0;
            rc = eig_dwest_launch(recs, Lp, (int)n, p0, score, literal, npos, s, 1);
            if (rc) return rc;
        }
        return HSAD_OK;
    }
    const int64_t rt = dwest_run_rows(H, W);
    const int64_t rows = rt * 16 < H ? rt * 16 : H;
    const size_t colb = align256((size_t)(3 * Lp) * sizeof(double) * (size_t)(rows * W));
    if (ws_bytes <= colb) return 1;
    int64_t bands = boxg_chunk_bands(H, W, Lp, ws_bytes - colb, 1);
    if (bands > rt) bands = rt;
    if (bands < 1) return 1;
    double *dey = (double *)ws, *recs = (double *)((char *)ws + colb);
    for (int64_t tr0 = 0; tr0 < ntr; tr0 += rt) {
        const int64_t tr1 = tr0 + rt < ntr ? tr0 + rt : ntr;
        const int64_t s0 = tr0 * 16 * W, s1 = (tr1 * 16 < H ? tr1 * 16 : H) * W, sn = s1 - s0;
        for (int64_t b0 = tr0; b0 < tr1; b0 += bands) {
            const int64_t nb = tr1 - b0 < bands ? tr1 - b0 : bands;
            int rc = boxg_launch(x, H, W, Lp, w, (int)b0, (int)nb, recs, s, 1);
            if (rc) return rc;
            const int64_t y1 = (b0 + nb) * 16 < H ? (b0 + nb) * 16 : H;
            const int64_t p0 = b0 * 16 * W, n = y1 * W - p0;
            rc = tridiag_dwest_launch(recs, Lp, (int)n, dey + (p0 - s0), sn, s, 1);
            if (rc) return rc;
        }
        if (int rc = ql_dwest_global_launch(dey, Lp, sn, s0, score, literal, npos, s)) return rc;
    }
    return HSAD_OK;
}

int generic_dwest(const float *x, int64_t H, int64_t W, int64_t Lp, const Windows &w,
                  float *score, float *literal, int32_t *npos, void *ws, size_t ws_bytes,
                  hipStream_t s)
{
    const bool jac = g_dwest_solver == 1;
    if ((jac ? jacobi_smem(Lp) : eig_smem(Lp)) > 160 * 1024 || gram_lds_per_wave(Lp, GP_FP64) > 160 * 1024)
        return fail(HSAD_EUNSUPPORTED, "hsad_dwest: L' above the eigensolver's LDS limit");
    if (!jac && g_dwest_stats == 0 && boxg_supported(Lp, w)) {
        const int rc = dwest_boxg(x, H, W, Lp, w, score, literal, npos, ws, ws_bytes, s);
        if (rc != 1) return rc;
    }
    const int64_t total = H * W;
    // The LDS kernel is the faster one when its workgroups hold 64 pixels (L' <= 32) and a
    // chunk holds enough of them (measured at 512 x 512: L' = 14 per chunk 5.0 ms, in runs
    // 5.4 ms; L' = 28 and 56, 8192-30000-pixel chunks: runs 8 % and 43 % faster).
    const bool chunk_first = ql_lds_pixels(Lp) == 64 &&
                             chunk_pixels(total, Lp, ws_bytes) >= (total < 65536 ? total : 65536);
    const bool runs = !jac && (g_dwest_solver == 3 || (g_dwest_solver == 0 && !chunk_first));
    const int64_t S = runs ? ql_run_pixels(total, Lp, ws_bytes) : 0;
    if (S > 0) {
        double *dey = (double *)ws;
        const size_t colb = align256((size_t)(3 * Lp) * sizeof(double) * (size_t)S);
        double *rec = (double *)((char *)ws + colb);
        const int64_t P = chunk_pixels(S, Lp, ws_bytes - colb);
        if (P < 1) return fail(HSAD_ENOMEM, "hsad_dwest: workspace below one pixel");
        for (int64_t s0 = 0; s0 < total; s0 += S) {
            const int64_t sn = (total - s0) < S ? (total - s0) : S;
            for (int64_t p0 = s0; p0 < s0 + sn; p0 += P) {
                const int n = (int)((s0 + sn - p0) < P ? (s0 + sn - p0) : P);
                int rc = gram_launch(x, H, W, Lp, w, GRAM_DWEST, GP_FP64, p0, n, rec, s);
                if (rc) return rc;
                rc = tridiag_dwest_launch(rec, Lp, n, dey + (p0 - s0), sn, s);
                if (rc) return rc;
            }
            if (int rc = ql_dwest_global_launch(dey, Lp, sn, s0, score, literal, npos, s)) return rc;
        }
        return HSAD_OK;
    }
    const int64_t P = chunk_pixels(total, Lp, ws_bytes);
    if (P < 1) return fail(HSAD_ENOMEM, "hsad_dwest: workspace below one pixel");
    for (int64_t p0 = 0; p0 < total; p0 += P) {
        const int n = (int)((total - p0) < P ? (total - p0) : P);
        int rc = gram_launch(x, H, W, Lp, w, GRAM_DWEST, GP_FP64, p0, n, (double *)ws, s);
        if (rc) return rc;
        rc = jac ? jacobi_launch((const double *)ws, Lp, n, p0, score, literal, npos, s)
                 : eig_dwest_launch((double *)ws, Lp, n, p0, score, literal, npos, s);
        if (rc) return rc;
    }
    return HSAD_OK;
}

}  // namespace hsad

// ---- step-level entry points for tests (not part of the public header) ----
extern "C" int hsad_internal_gram(const float *x, int64_t H, int64_t W, int64_t Lp,
                                  const hsad_window_params *p, int mode, int prec, int64_t pix0,
                                  int npix, double *ws, hipStream_t s)
{
    using namespace hsad;
    if (!x || !p || !ws || H < 1 || W < 1 || Lp < 1 || Lp > HSAD_MAX_LP || npix < 1 ||
        pix0 < 0 || pix0 + npix > H * W || (p->outer & 1) == 0 || p->inner >= p->outer)
        return fail(HSAD_EINVAL, "hsad_internal_gram: bad arguments");
    Windows w{p->inner, p->outer, p->inner / 2, p->outer / 2};
    return gram_launch(x, H, W, Lp, w, mode, prec, pix0, npix, ws, s);
}

extern "C" int hsad_internal_generic_force(int mode)
{
    hsad::g_generic_force = mode;
    return 0;
}

extern "C" int hsad_internal_dwest_solver(int solver)
{
    hsad::g_dwest_solver = solver >= 1 && solver <= 3 ? solver : 0;
    return 0;
}

extern "C" int hsad_internal_dwest_stats(int gram)
{
    hsad::g_dwest_stats = gram ? 1 : 0;
    return 0;
}
