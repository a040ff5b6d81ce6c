// internal.hpp -- shared declarations of the libhsad translation units (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "../../include/hsad.h"

namespace hsad {

// ---- error reporting (thread-local message, see hsad_last_error) ----
void set_error(const std::string &msg);
void clear_error();
int fail(int code, const std::string &msg);
int check_launch(const char *what);
// Raises a kernel's dynamic-LDS limit when a launch needs more than the 64 KiB default.
int allow_lds(const void *kernel, size_t bytes, const char *what);

// ---- filter design (api.hip) ----
// 8-tap Daubechies low-pass, time order of eq. (9).
const double *db4_filter();

// ---- DWT (dwt.hip) ----
// Composite (equivalent-filter) matrix of `levels` levels applied to length L:
// Lp x L, row-major, double.  Pushes unit vectors through the cascade with the
// odd-length extension.
void dwt_composite_matrix(int64_t L, int levels, double *A /* Lp*L */);
// e0 / e1 (may be null): events that take the start and end of the transform's kernel
int dwt_launch(const float *cube, int64_t npix, int64_t L, int levels, int64_t Lp,
               float *approx, hipStream_t s, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
// Band-major [L][L'] composite matrix of the LDS-staged equivalent filter on the device, or
// nullptr when dwt_launch would use another kernel for (L, levels).
const double *dwt_lds_coefs(int64_t L, int levels, int64_t Lp, hipStream_t s);

// ---- window geometry ----
struct Windows {
    int inner, outer;
    int ri, ro;   // half sizes
};

// ---- small-L' fused box-sum detector (box.hip) ----
bool box_supported(int64_t Lp, const Windows &w);
// part (optional): 3 doubles per 16 x 16 tile, row-major over tiles, receive the
// (count, mean, M2) of the tile's finite LRX scores (eq. 12 partials; lrx must be set).
int box_lrx_dwrx_launch(const float *x, int64_t H, int64_t W, int64_t Lp, const Windows &w,
                        double load_rel, float *lrx, float *dwrx, hipStream_t s,
                        double *part = nullptr);
// The LDS-staged DWT of one cube (L bands, `levels` levels, into approx) and the box
// detector on another, already reduced cube x (as box_lrx_dwrx_launch with its tile
// partials; *nparts receives their number), in one launch whose workgroups take one role or
// the other.  The two must not
// overlap in memory.  Returns HSAD_EUNSUPPORTED, with nothing enqueued and no error set,
// when the pair cannot share a launch (the caller runs them one after the other).
// thr (optional): a third role in the same launch, eq. (12) of an earlier map s from its
// nblk <= 1024 tile partials, writing stats and mask (as threshold_from_partials).
struct FusedThr {
    const float *s;
    const double *part;
    int nblk;
    double z;
    double *stats;
    uint8_t *mask;
};
int dwt_box_fused_launch(const float *cube, int64_t L, int levels, float *approx, const float *x,
                         int64_t H, int64_t W, int64_t Lp, const Windows &w, double load_rel, float *lrx,
                         float *dwrx, double *part, int64_t *nparts, hipStream_t s, hipEvent_t e0,
                         hipEvent_t e1, const FusedThr *thr = nullptr);
size_t box_tiles(int64_t H, int64_t W);
// tiles of the box kernel as launched for these sizes (at most box_tiles(H, W))
size_t box_tiles_used(int64_t H, int64_t W, int64_t Lp, const Windows &w);

// ---- eq. (12) from partial statistics (eval.hip) ----
// Merges nblk (count, mean, M2) partials in a fixed order, writes stats {count, mu, sigma,
// tau = mu + z sigma} and, if mask is set, mask = scores > tau.  fold: device scratch of
// threshold_fold_doubles() doubles, used when nblk exceeds what one merge pass takes.
size_t threshold_fold_doubles();
int threshold_from_partials(const float *scores, int64_t n, const double *part, int64_t nblk, double z,
                            double *stats, uint8_t *mask, double *fold, hipStream_t s);

// ---- box-sum statistics for mid-size L' (boxg.hip) ----
bool boxg_supported(int64_t Lp, const Windows &w);
size_t boxg_record_doubles(int64_t Lp, int inner_rec = 0);
int64_t boxg_chunk_bands(int64_t H, int64_t W, int64_t Lp, size_t ws_bytes, int inner_rec = 0);
int boxg_resident_kb();

// ---- generic Gram + factorisation path (gram.hip, chol.hip, jacobi.hip) ----
enum GramMode { GRAM_LRX = 0, GRAM_DWEST = 1 };
enum GramPrec { GP_FP64 = 0, GP_FP32 = 1, GP_BF16 = 2, GP_FP16 = 3 };

// Bytes of workspace per pixel and the fixed part for the generic path.
size_t generic_ws_per_pixel(int64_t Lp, GramMode mode);
// workspace hsad_workspace_bytes reports for DWEST: the QL columns of one run of pixels and
// the chunk records
size_t dwest_ws_bytes(int64_t H, int64_t W, int64_t Lp, const Windows &w);
int generic_lrx_dwrx(const float *x, int64_t H, int64_t W, int64_t Lp, const Windows &w,
                     double load_rel, GramPrec prec, float *lrx, float *dwrx, void *ws,
                     size_t ws_bytes, hipStream_t s);
int generic_lrx_dwrx_at(const float *x, int64_t H, int64_t W, int64_t Lp, const Windows &w,
                        double load_rel, GramPrec prec, const int32_t *idx, int64_t nidx, float *lrx,
                        float *dwrx, void *ws, size_t ws_bytes, hipStream_t s);
// smallest workspace hsad_detect accepts (api.hip); 0 for invalid arguments
size_t detect_min_bytes(int64_t H, int64_t W, int64_t Lp, const hsad_window_params *p, bool with_dwrx);
int generic_dwest(const float *x, int64_t H, int64_t W, int64_t Lp, const Windows &w,
                  float *score, float *literal, int32_t *npos, void *ws, size_t ws_bytes,
                  hipStream_t s);

}  // namespace hsad
