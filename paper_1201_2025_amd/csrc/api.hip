// api.hip -- C ABI of libhsad: argument validation, filter design, dispatch.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>
#include <string>

#include "internal.hpp"

namespace hsad {

// ------------------------------------------------------------------------------------
// errors
// ------------------------------------------------------------------------------------
static thread_local std::string t_err;

void set_error(const std::string &msg) { t_err = msg; }
void clear_error() { t_err.clear(); }
int fail(int code, const std::string &msg)
{
    t_err = msg;
    return code;
}
int allow_lds(const void *kernel, size_t bytes, const char *what)
{
    if (bytes <= 64 * 1024) return HSAD_OK;
    hipError_t e = hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(HSAD_EUNSUPPORTED, std::string(what) + ": LDS request too large");
    }
    return HSAD_OK;
}

int check_launch(const char *what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(HSAD_EHIP, std::string(what) + ": " + hipGetErrorString(e));
    return HSAD_OK;
}

// ------------------------------------------------------------------------------------
// Daubechies-4 low-pass.  Seeded with the 12-decimal values of Daubechies, "Ten
// Lectures on Wavelets" (1992), Table 6.1, N = 4.  Gauss-Newton on the defining
// equations then refines them to double precision: sum h = sqrt 2, orthonormal even
// shifts, and four vanishing moments of the alternating sequence.
// ------------------------------------------------------------------------------------
static double g_h[8];
static std::once_flag g_h_once;

static void solve_spd(double *M, double *b, int n)   // in-place Gaussian elimination
{
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (std::fabs(M[r * n + c]) > std::fabs(M[piv * n + c])) piv = r;
        if (piv != c) {
            for (int k = 0; k < n; ++k) std::swap(M[c * n + k], M[piv * n + k]);
            std::swap(b[c], b[piv]);
        }
        for (int r = c + 1; r < n; ++r) {
            double f = M[r * n + c] / M[c * n + c];
            for (int k = c; k < n; ++k) M[r * n + k] -= f * M[c * n + k];
            b[r] -= f * b[c];
        }
    }
    for (int r = n - 1; r >= 0; --r) {
        double s = b[r];
        for (int k = r + 1; k < n; ++k) s -= M[r * n + k] * b[k];
        b[r] = s / M[r * n + r];
    }
}

static void design_db4()
{
    double h[8] = {0.230377813309, 0.714846570553, 0.630880767930, -0.027983769417,
                   -0.187034811719, 0.030841381836, 0.032883011667, -0.010597401785};
    constexpr int NE = 9, NU = 8;
    for (int it = 0; it < 6; ++it) {
        double F[NE], J[NE][NU];
        std::memset(J, 0, sizeof(J));
        double s = 0;
        for (int k = 0; k < 8; ++k) s += h[k];
        F[0] = s - std::sqrt(2.0);
        for (int k = 0; k < 8; ++k) J[0][k] = 1.0;
        for (int m = 0; m < 4; ++m) {
            double d = 0;
            for (int k = 0; k + 2 * m < 8; ++k) {
                d += h[k] * h[k + 2 * m];
                J[1 + m][k] += h[k + 2 * m];
                J[1 + m][k + 2 * m] += h[k];
            }
            F[1 + m] = d - (m == 0 ? 1.0 : 0.0);
        }
        for (int p = 0; p < 4; ++p) {
            double d = 0;
            for (int k = 0; k < 8; ++k) {
                double w = ((k & 1) ? -1.0 : 1.0) * std::pow((double)k, p);
                d += w * h[k];
                J[5 + p][k] = w;
            }
            F[5 + p] = d;
        }
        double M[NU * NU], b[NU];
        for (int a = 0; a < NU; ++a) {
            b[a] = 0;
            for (int e = 0; e < NE; ++e) b[a] += J[e][a] * F[e];
            for (int c = 0; c < NU; ++c) {
                double t = 0;
                for (int e = 0; e < NE; ++e) t += J[e][a] * J[e][c];
                M[a * NU + c] = t;
            }
        }
        solve_spd(M, b, NU);
        for (int k = 0; k < 8; ++k) h[k] -= b[k];
    }
    std::memcpy(g_h, h, sizeof(h));
}

const double *db4_filter()
{
    std::call_once(g_h_once, design_db4);
    return g_h;
}

// ------------------------------------------------------------------------------------
// validation helpers
// ------------------------------------------------------------------------------------
static int out_len(int64_t L, int levels, int64_t *Lp)
{
    if (L < 1 || levels < 0) return HSAD_EINVAL;
    int64_t n = L;
    for (int j = 0; j < levels; ++j) {
        if (n < 2) return HSAD_EINVAL;
        n = (n + 1) / 2;
    }
    *Lp = n;
    return HSAD_OK;
}

static int check_windows(const char *fn, const hsad_window_params *p, int64_t H, int64_t W,
                         int64_t Lp, bool need_inner, Windows *w)
{
    if (!p) return fail(HSAD_EINVAL, std::string(fn) + ": params is NULL");
    if (H < 1 || W < 1 || Lp < 1)
        return fail(HSAD_EINVAL, std::string(fn) + ": H, W and L' must be >= 1");
    if (Lp > HSAD_MAX_LP)
        return fail(HSAD_EUNSUPPORTED, std::string(fn) + ": L' above HSAD_MAX_LP");
    if (p->reserved != 0) return fail(HSAD_EINVAL, std::string(fn) + ": reserved must be 0");
    if (p->outer < 1 || (p->outer & 1) == 0 || p->outer > HSAD_MAX_WINDOW)
        return fail(HSAD_EINVAL, std::string(fn) + ": outer must be odd, 1..HSAD_MAX_WINDOW");
    if (p->inner < 0 || (p->inner != 0 && (p->inner & 1) == 0) || p->inner >= p->outer)
        return fail(HSAD_EINVAL, std::string(fn) + ": inner must be 0 or odd and < outer");
    if (need_inner && p->inner < 1)
        return fail(HSAD_EINVAL, std::string(fn) + ": this detector needs an inner window");
    if (!(p->load_rel >= 0.0) || !std::isfinite(p->load_rel))
        return fail(HSAD_EINVAL, std::string(fn) + ": load_rel must be finite and >= 0");
    if (p->precision < HSAD_PREC_AUTO || p->precision > HSAD_PREC_GRAM_FP16)
        return fail(HSAD_EINVAL, std::string(fn) + ": unknown precision");
    // the annulus is empty for some pixel iff the clipped inner window already covers
    // the whole image extent in both directions
    if (p->inner > 0 && H <= p->inner && W <= p->inner)
        return fail(HSAD_EINVAL, std::string(fn) + ": the annulus is empty for some pixel");
    w->inner = p->inner;
    w->outer = p->outer;
    w->ri = p->inner / 2;
    w->ro = p->outer / 2;
    return HSAD_OK;
}

static GramPrec gram_prec(int precision)
{
    switch (precision) {
    case HSAD_PREC_FP32: return GP_FP32;
    case HSAD_PREC_GRAM_BF16: return GP_BF16;
    case HSAD_PREC_GRAM_FP16: return GP_FP16;
    default: return GP_FP64;
    }
}

static bool exact(int precision)
{
    return precision == HSAD_PREC_AUTO || precision == HSAD_PREC_FP64;
}

}  // namespace hsad

using namespace hsad;

extern "C" {

const char *hsad_version(void) { return "hsad 0.1.0 gfx950"; }

const char *hsad_last_error(void) { return t_err.c_str(); }

int hsad_dwt_out_len(int64_t L, int levels, int64_t *Lp)
{
    if (!Lp) return fail(HSAD_EINVAL, "hsad_dwt_out_len: Lp is NULL");
    int rc = out_len(L, levels, Lp);
    if (rc) return fail(rc, "hsad_dwt_out_len: L < 1, levels < 0 or a level input below 2");
    return HSAD_OK;
}

int hsad_levels_for(int64_t L, int target)
{
    if (L < 1 || target < 1) return fail(HSAD_EINVAL, "hsad_levels_for: L and target must be >= 1");
    int J = 0;
    int64_t n = L;
    while (n >= 2 && (n + 1) / 2 >= target) {
        n = (n + 1) / 2;
        ++J;
    }
    return J;
}

int hsad_dwt(const float *cube, int64_t H, int64_t W, int64_t L, int levels, float *approx,
             hipStream_t stream)
{
    clear_error();
    if (!cube || !approx) return fail(HSAD_EINVAL, "hsad_dwt: NULL pointer");
    if (H < 1 || W < 1) return fail(HSAD_EINVAL, "hsad_dwt: H and W must be >= 1");
    int64_t Lp = 0;
    if (out_len(L, levels, &Lp))
        return fail(HSAD_EINVAL, "hsad_dwt: L < 1, levels < 0 or levels too deep for L");
    if (L > (1 << 20)) return fail(HSAD_EUNSUPPORTED, "hsad_dwt: L above 2^20");
    return dwt_launch(cube, H * W, L, levels, Lp, approx, stream);
}

int hsad_dwt_timed(const float *cube, int64_t H, int64_t W, int64_t L, int levels, float *approx,
                   hipStream_t stream, hipEvent_t start, hipEvent_t stop)
{
    clear_error();
    if (!cube || !approx) return fail(HSAD_EINVAL, "hsad_dwt_timed: NULL pointer");
    if (H < 1 || W < 1) return fail(HSAD_EINVAL, "hsad_dwt_timed: H and W must be >= 1");
    int64_t Lp = 0;
    if (out_len(L, levels, &Lp))
        return fail(HSAD_EINVAL, "hsad_dwt_timed: L < 1, levels < 0 or levels too deep for L");
    if (L > (1 << 20)) return fail(HSAD_EUNSUPPORTED, "hsad_dwt_timed: L above 2^20");
    return dwt_launch(cube, H * W, L, levels, Lp, approx, stream, start, stop);
}

size_t hsad_workspace_bytes(int op, int64_t H, int64_t W, int64_t Lp,
                            const hsad_window_params *p)
{
    Windows w;
    if (op < HSAD_OP_LRX || op > HSAD_OP_DWEST) return 0;
    std::string keep = t_err;
    int rc = check_windows("hsad_workspace_bytes", p, H, W, Lp, op != HSAD_OP_LRX, &w);
    t_err = keep;
    if (rc) return 0;
    if (op != HSAD_OP_DWEST && exact(p->precision) && box_supported(Lp, w)) return 0;
    if (op == HSAD_OP_DWEST) return dwest_ws_bytes(H, W, Lp, w);
    const GramMode mode = GRAM_LRX;
    const size_t per = generic_ws_per_pixel(Lp, mode);
    // enough for every pixel in one launch, capped at 1 GiB (larger chunks gain nothing)
    const size_t cap = (size_t)1 << 30;
    const size_t npix = (size_t)(H * W);
    size_t want = per * npix;
    if (want > cap) want = (cap / per) * per;
    if (want < per) want = per;
    if (op != HSAD_OP_DWEST && exact(p->precision) && boxg_supported(Lp, w)) {
        // box-statistics path: whole bands of 16 image rows, as many as its chunk rule uses
        const int64_t bands = boxg_chunk_bands(H, W, Lp, (size_t)-1 / 2);
        const size_t bw = (size_t)bands * 16 * (size_t)W * boxg_record_doubles(Lp) * sizeof(double);
        if (bw > want) want = bw;
    }
    return want;
}

static int lrx_dwrx_common(const char *fn, const float *x, int64_t H, int64_t W, int64_t Lp,
                           const hsad_window_params *p, float *lrx, float *dwrx, void *ws,
                           size_t ws_bytes, hipStream_t stream)
{
    clear_error();
    Windows w;
    int rc = check_windows(fn, p, H, W, Lp, dwrx != nullptr, &w);
    if (rc) return rc;
    if (!x) return fail(HSAD_EINVAL, std::string(fn) + ": x is NULL");
    if (!lrx && !dwrx) return fail(HSAD_EINVAL, std::string(fn) + ": no output requested");
    // A reduced-precision Gram is only offered where the annulus holds at least 2 L' samples:
    // with fewer the covariance is (nearly) rank-deficient, the loading alone sets its smallest
    // eigenvalues, and FP32/BF16/FP16 rounding of the samples moves those by more than the
    // loading (at L' = 224 with 200 samples the ROC AUC moved by 0.01-0.26).  Pixels whose
    // clipped annulus (image borders) is shorter than that take the FP64 Gram.
    if (!exact(p->precision)) {
        const int64_t n_a = (int64_t)p->outer * p->outer - (int64_t)p->inner * p->inner;
        if (n_a < 2 * Lp)
            return fail(HSAD_EUNSUPPORTED, std::string(fn) + ": a reduced-precision Gram needs an annulus of at "
                                                              "least 2 L' samples (outer^2 - inner^2 >= 2 L')");
    }
    if (exact(p->precision) && box_supported(Lp, w))
        return box_lrx_dwrx_launch(x, H, W, Lp, w, p->load_rel, lrx, dwrx, stream);
    const size_t per = generic_ws_per_pixel(Lp, GRAM_LRX);
    if (!ws || ws_bytes < per)
        return fail(HSAD_ENOMEM, std::string(fn) + ": workspace too small (see hsad_workspace_bytes)");
    return generic_lrx_dwrx(x, H, W, Lp, w, p->load_rel, gram_prec(p->precision), lrx, dwrx, ws,
                            ws_bytes, stream);
}

int hsad_lrx(const float *x, int64_t H, int64_t W, int64_t Lp, const hsad_window_params *p,
             float *scores, void *ws, size_t ws_bytes, hipStream_t stream)
{
    if (!scores) return fail(HSAD_EINVAL, "hsad_lrx: scores is NULL");
    return lrx_dwrx_common("hsad_lrx", x, H, W, Lp, p, scores, nullptr, ws, ws_bytes, stream);
}

int hsad_dwrx(const float *x, int64_t H, int64_t W, int64_t Lp, const hsad_window_params *p,
              float *scores, void *ws, size_t ws_bytes, hipStream_t stream)
{
    if (!scores) return fail(HSAD_EINVAL, "hsad_dwrx: scores is NULL");
    return lrx_dwrx_common("hsad_dwrx", x, H, W, Lp, p, nullptr, scores, ws, ws_bytes, stream);
}

int hsad_lrx_dwrx(const float *x, int64_t H, int64_t W, int64_t Lp,
                  const hsad_window_params *p, float *lrx, float *dwrx, void *ws,
                  size_t ws_bytes, hipStream_t stream)
{
    return lrx_dwrx_common("hsad_lrx_dwrx", x, H, W, Lp, p, lrx, dwrx, ws, ws_bytes, stream);
}

// Workspace of hsad_detect: eq. (12) partials (one per box tile, at most one per 16 x 16
// tiles, on the box path, else the threshold's blocks) and the fold buffer, 256-byte aligned, then what hsad_lrx_dwrx
// needs.
static size_t detect_head_bytes(int64_t H, int64_t W)
{
    size_t np = box_tiles(H, W);
    const size_t tb = hsad_threshold_workspace_bytes(H * W) / (3 * sizeof(double));
    if (np < tb) np = tb;
    const size_t b = (np + threshold_fold_doubles() / 3) * 3 * sizeof(double);
    return (b + 255) & ~(size_t)255;
}

}  // extern "C"

// Smallest workspace hsad_detect accepts for these arguments (0 when they are invalid; the
// calling thread's error message is left as it was).
size_t hsad::detect_min_bytes(int64_t H, int64_t W, int64_t Lp, const hsad_window_params *p, bool with_dwrx)
{
    Windows w;
    std::string keep = t_err;
    int rc = check_windows("hsad_detect", p, H, W, Lp, with_dwrx, &w);
    t_err = keep;
    if (rc) return 0;
    size_t b = detect_head_bytes(H, W);
    if (!(exact(p->precision) && box_supported(Lp, w))) b += generic_ws_per_pixel(Lp, GRAM_LRX);
    return b;
}

extern "C" {

size_t hsad_detect_workspace_bytes(int64_t H, int64_t W, int64_t Lp, const hsad_window_params *p)
{
    if (H < 1 || W < 1) return 0;
    const int op = p && p->inner > 0 ? HSAD_OP_LRX_DWRX : HSAD_OP_LRX;
    return detect_head_bytes(H, W) + hsad_workspace_bytes(op, H, W, Lp, p);
}

int hsad_detect(const float *x, int64_t H, int64_t W, int64_t Lp, const hsad_window_params *p,
                double z_alpha, float *lrx, float *dwrx, double *stats, uint8_t *mask, void *ws,
                size_t ws_bytes, hipStream_t stream)
{
    clear_error();
    Windows w;
    int rc = check_windows("hsad_detect", p, H, W, Lp, dwrx != nullptr, &w);
    if (rc) return rc;
    if (!x || !lrx || !stats) return fail(HSAD_EINVAL, "hsad_detect: x, lrx and stats are required");
    if (!std::isfinite(z_alpha)) return fail(HSAD_EINVAL, "hsad_detect: z_alpha not finite");
    const size_t head = detect_head_bytes(H, W);
    if (!ws || ws_bytes < head) return fail(HSAD_ENOMEM, "hsad_detect: workspace too small");
    double *part = (double *)ws;
    const size_t np = (head / (3 * sizeof(double))) - threshold_fold_doubles() / 3;
    double *fold = part + 3 * np;
    const int64_t n = H * W;
    if (exact(p->precision) && box_supported(Lp, w)) {
        // the box kernel leaves one partial per tile: no separate statistics pass
        rc = box_lrx_dwrx_launch(x, H, W, Lp, w, p->load_rel, lrx, dwrx, stream, part);
        if (rc) return rc;
        return threshold_from_partials(lrx, n, part, (int64_t)box_tiles_used(H, W, Lp, w), z_alpha, stats, mask,
                                       fold, stream);
    }
    rc = lrx_dwrx_common("hsad_detect", x, H, W, Lp, p, lrx, dwrx, (char *)ws + head, ws_bytes - head,
                         stream);
    if (rc) return rc;
    return hsad_threshold(lrx, n, z_alpha, stats, mask, part, head, stream);
}

int hsad_dwt_detect_fused(const float *cube_next, int64_t L, int levels, float *approx_next,
                          const float *x, int64_t H, int64_t W, int64_t Lp, const hsad_window_params *p,
                          double z_alpha, float *lrx, float *dwrx, double *stats, uint8_t *mask, void *ws,
                          size_t ws_bytes, hipStream_t stream, hipEvent_t start, hipEvent_t stop)
{
    static const char *fn = "hsad_dwt_detect_fused";
    clear_error();
    if (!cube_next && !x) return fail(HSAD_EINVAL, std::string(fn) + ": cube_next and x are both NULL");
    if (H < 1 || W < 1) return fail(HSAD_EINVAL, std::string(fn) + ": H and W must be >= 1");
    const int64_t n = H * W;
    int64_t Lpn = 0;
    if (cube_next) {
        if (!approx_next) return fail(HSAD_EINVAL, std::string(fn) + ": approx_next is NULL");
        if (out_len(L, levels, &Lpn))
            return fail(HSAD_EINVAL, std::string(fn) + ": L < 1, levels < 0 or levels too deep for L");
        if (L > (1 << 20)) return fail(HSAD_EUNSUPPORTED, std::string(fn) + ": L above 2^20");
        if (!x) return dwt_launch(cube_next, n, L, levels, Lpn, approx_next, stream, start, stop);
    }
    Windows w;
    int rc = check_windows(fn, p, H, W, Lp, dwrx != nullptr, &w);
    if (rc) return rc;
    if (!lrx || !stats) return fail(HSAD_EINVAL, std::string(fn) + ": lrx and stats are required");
    if (!std::isfinite(z_alpha)) return fail(HSAD_EINVAL, std::string(fn) + ": z_alpha not finite");
    const size_t head = detect_head_bytes(H, W);
    if (!ws || ws_bytes < head) return fail(HSAD_ENOMEM, std::string(fn) + ": workspace too small");
    if (!cube_next) return hsad_detect(x, H, W, Lp, p, z_alpha, lrx, dwrx, stats, mask, ws, ws_bytes, stream);
    if (Lpn != Lp)
        return fail(HSAD_EINVAL, std::string(fn) + ": L' of the cube to reduce differs from the L' of x");
    // the two halves run at the same time: what the DWT writes must not meet anything the
    // detector reads or writes, and what the detector writes must not meet the cube the DWT
    // reads
    const auto meets = [](const void *a, size_t na, const void *b, size_t nb) {
        if (!a || !b || !na || !nb) return false;
        const uintptr_t pa = (uintptr_t)a, pb = (uintptr_t)b;
        return pa < pb + nb && pb < pa + na;
    };
    const size_t red = (size_t)(n * Lp) * sizeof(float), raw = (size_t)(n * L) * sizeof(float);
    const size_t map = (size_t)n * sizeof(float);
    if (meets(approx_next, red, cube_next, raw) || meets(approx_next, red, x, red) ||
        meets(approx_next, red, lrx, map) || meets(approx_next, red, dwrx, map) ||
        meets(approx_next, red, mask, (size_t)n) || meets(approx_next, red, stats, 4 * sizeof(double)) ||
        meets(approx_next, red, ws, ws_bytes))
        return fail(HSAD_EINVAL, std::string(fn) + ": approx_next overlaps another argument");
    if (meets(cube_next, raw, lrx, map) || meets(cube_next, raw, dwrx, map) || meets(cube_next, raw, mask, (size_t)n) ||
        meets(cube_next, raw, stats, 4 * sizeof(double)) || meets(cube_next, raw, ws, ws_bytes))
        return fail(HSAD_EINVAL, std::string(fn) + ": cube_next overlaps an output of the detector");
    if (exact(p->precision) && box_supported(Lp, w)) {
        double *part = (double *)ws;
        const size_t np = (head / (3 * sizeof(double))) - threshold_fold_doubles() / 3;
        int64_t nparts = 0;
        rc = dwt_box_fused_launch(cube_next, L, levels, approx_next, x, H, W, Lp, w, p->load_rel, lrx, dwrx, part,
                                  &nparts, stream, start, stop);
        if (rc == HSAD_OK)
            return threshold_from_partials(lrx, n, part, nparts, z_alpha, stats, mask, part + 3 * np, stream);
        if (rc != HSAD_EUNSUPPORTED) return rc;
    }
    // the two cannot share a launch: one after the other
    rc = dwt_launch(cube_next, n, L, levels, Lp, approx_next, stream, start, stop);
    if (rc) return rc;
    return hsad_detect(x, H, W, Lp, p, z_alpha, lrx, dwrx, stats, mask, ws, ws_bytes, stream);
}

int hsad_detect_stream_step(const float *cube_next, int64_t L, int levels, float *approx_next, const float *x,
                            int64_t H, int64_t W, int64_t Lp, const hsad_window_params *p, float *lrx, float *dwrx,
                            void *ws, size_t ws_bytes, const float *prev_lrx, void *prev_ws, double z_alpha,
                            double *prev_stats, uint8_t *prev_mask, hipStream_t stream, hipEvent_t start,
                            hipEvent_t stop)
{
    static const char *fn = "hsad_detect_stream_step";
    clear_error();
    if (!cube_next && !x && !prev_lrx) return fail(HSAD_EINVAL, std::string(fn) + ": nothing to do");
    if (H < 1 || W < 1) return fail(HSAD_EINVAL, std::string(fn) + ": H and W must be >= 1");
    const int64_t n = H * W;
    int64_t Lpn = 0;
    if (cube_next) {
        if (!approx_next) return fail(HSAD_EINVAL, std::string(fn) + ": approx_next is NULL");
        if (out_len(L, levels, &Lpn))
            return fail(HSAD_EINVAL, std::string(fn) + ": L < 1, levels < 0 or levels too deep for L");
        if (L > (1 << 20)) return fail(HSAD_EUNSUPPORTED, std::string(fn) + ": L above 2^20");
        if (Lpn != Lp) return fail(HSAD_EINVAL, std::string(fn) + ": L' of the cube to reduce differs from Lp");
    }
    // the detector and the threshold work on the box path's tile partials
    Windows w;
    int rc = check_windows(fn, p, H, W, Lp, dwrx != nullptr, &w);
    if (rc) return rc;
    if (!exact(p->precision) || !box_supported(Lp, w))
        return fail(HSAD_EUNSUPPORTED, std::string(fn) + ": needs the exact box path (L' <= 8)");
    const size_t head = detect_head_bytes(H, W);
    if (x && (!lrx || !ws || ws_bytes < head))
        return fail(HSAD_EINVAL, std::string(fn) + ": x needs lrx and a workspace of hsad_detect's size");
    if (prev_lrx && (!prev_stats || !prev_ws))
        return fail(HSAD_EINVAL, std::string(fn) + ": prev_lrx needs prev_stats and prev_ws");
    if (prev_lrx && !std::isfinite(z_alpha)) return fail(HSAD_EINVAL, std::string(fn) + ": z_alpha not finite");
    // the stages run at the same time: nothing one writes may meet what another reads or writes
    const auto meets = [](const void *a, size_t na, const void *b, size_t nb) {
        if (!a || !b || !na || !nb) return false;
        const uintptr_t pa = (uintptr_t)a, pb = (uintptr_t)b;
        return pa < pb + nb && pb < pa + na;
    };
    const size_t red = (size_t)(n * Lp) * sizeof(float), map = (size_t)n * sizeof(float);
    struct Rg {
        const void *p;
        size_t n;
        bool written;
    } r[] = {{cube_next, cube_next ? (size_t)(n * L) * sizeof(float) : 0, false},
             {approx_next, cube_next ? red : 0, true},
             {x, x ? red : 0, false},
             {lrx, x ? map : 0, true},
             {dwrx, x ? map : 0, true},
             {ws, x ? ws_bytes : 0, true},
             {prev_lrx, prev_lrx ? map : 0, false},
             {prev_ws, prev_lrx ? head : 0, true},
             {prev_stats, prev_lrx ? 4 * sizeof(double) : 0, true},
             {prev_mask, prev_lrx ? (size_t)n : 0, true}};
    const int nr = (int)(sizeof(r) / sizeof(r[0]));
    for (int i = 0; i < nr; ++i)
        for (int j = i + 1; j < nr; ++j)
            if ((r[i].written || r[j].written) && meets(r[i].p, r[i].n, r[j].p, r[j].n))
                return fail(HSAD_EINVAL, std::string(fn) + ": two arguments overlap");
    const size_t np = (head / (3 * sizeof(double))) - threshold_fold_doubles() / 3;
    const int64_t ntiles = (int64_t)box_tiles_used(H, W, Lp, w);
    double *part = (double *)ws, *pprev = (double *)prev_ws;
    if (cube_next && x) {
        // the threshold joins the shared launch when its partials fit one merge tree
        const bool thr_in = prev_lrx && ntiles <= 1024;
        FusedThr thr{prev_lrx, pprev, (int)ntiles, z_alpha, prev_stats, prev_mask};
        int64_t nparts = 0;
        rc = dwt_box_fused_launch(cube_next, L, levels, approx_next, x, H, W, Lp, w, p->load_rel, lrx, dwrx, part,
                                  &nparts, stream, start, stop, thr_in ? &thr : nullptr);
        if (rc == HSAD_OK) {
            if (!prev_lrx || thr_in) return HSAD_OK;
            return threshold_from_partials(prev_lrx, n, pprev, ntiles, z_alpha, prev_stats, prev_mask,
                                           pprev + 3 * np, stream);
        }
        if (rc != HSAD_EUNSUPPORTED) return rc;
    }
    // the stages one after the other
    if (cube_next) {
        rc = dwt_launch(cube_next, n, L, levels, Lp, approx_next, stream, start, stop);
        if (rc) return rc;
    }
    if (x) {
        rc = box_lrx_dwrx_launch(x, H, W, Lp, w, p->load_rel, lrx, dwrx, stream, part);
        if (rc) return rc;
    }
    if (prev_lrx)
        return threshold_from_partials(prev_lrx, n, pprev, ntiles, z_alpha, prev_stats, prev_mask, pprev + 3 * np,
                                       stream);
    return HSAD_OK;
}

int hsad_dwest(const float *x, int64_t H, int64_t W, int64_t Lp, const hsad_window_params *p,
               float *scores, float *scores_literal, int32_t *npos, void *ws,
               size_t ws_bytes, hipStream_t stream)
{
    clear_error();
    Windows w;
    int rc = check_windows("hsad_dwest", p, H, W, Lp, true, &w);
    if (rc) return rc;
    if (!x || !scores) return fail(HSAD_EINVAL, "hsad_dwest: NULL pointer");
    const size_t per = generic_ws_per_pixel(Lp, GRAM_DWEST);
    if (!ws || ws_bytes < per)
        return fail(HSAD_ENOMEM, "hsad_dwest: workspace too small (see hsad_workspace_bytes)");
    return generic_dwest(x, H, W, Lp, w, scores, scores_literal, npos, ws, ws_bytes, stream);
}

// Filter taps as designed by the library (for tests of the design step).
int hsad_internal_filter(double *h8)
{
    if (!h8) return HSAD_EINVAL;
    std::memcpy(h8, db4_filter(), 8 * sizeof(double));
    return HSAD_OK;
}

}  // extern "C"
