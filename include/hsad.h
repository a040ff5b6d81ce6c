/*
 * hsad.h -- C ABI of libhsad, DWT-reduced local hyperspectral anomaly detection on
 * AMD Instinct MI355X (gfx950).
 *
 * Method: Zare Baghbidi, Jamshidi, Naghsh Nilchi, Homayouni, "Improvement of anomaly
 * detection algorithms in hyperspectral images using discrete wavelet transform",
 * SIPIJ 2(4), 2011.  Each pixel spectrum r (L bands, Sec. 2.1) is reduced by a
 * Daubechies-4 DWT to its approximation coefficients (Sec. 3 eqs. 8-9, Sec. 4).  Local
 * detectors then score the reduced cube: LRX (Sec. 2.1, eq. 1), DWRX (Sec. 2.3, eq. 5)
 * and DWEST (Sec. 2.2, eqs. 2-4).
 *
 * Conventions shared by every entry point
 *   - Layout: cubes are dense row-major [y][x][band] float32 (band fastest, "BIP").  The
 *     reduced cube is [y][x][k], k < L'.  Score maps are [y][x] float32.
 *   - Pointers named cube/x/approx/scores/mask/ws/... are DEVICE pointers owned by the
 *     caller.  The library never allocates or frees device memory in these calls.  A call
 *     validates its arguments on the host, enqueues kernels on `stream` and returns
 *     without synchronising.  Passing stream 0 means the null stream.
 *   - Return codes: HSAD_OK (0) or a negative HSAD_E*.  Argument errors are detected
 *     before any launch, and nothing is enqueued then.  hsad_last_error() gives a
 *     message for the calling thread.
 *   - Numerical events inside a pixel are not errors.  A non-finite input gives a
 *     non-finite score for every window that contains it.  A covariance that is not
 *     positive definite after loading gives +inf.
 *   - Windows: odd square windows centred on the pixel and clipped to the image
 *     (Sec. 2.2, Sec. 5.2).  The background of LRX/DWRX/DWEST is the outer window minus
 *     the inner window.  inner == 0 means no guard window, so the background
 *     includes the pixel itself.  inner == 1 excludes only the pixel.
 *   - Covariances are normalised by the sample count.  Diagonal loading (LRX/DWRX)
 *     adds lambda * I with lambda = load_rel * tr(C) / L', and lambda is at least 1e-30.
 */
#ifndef HSAD_H
#define HSAD_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* return codes */
#define HSAD_OK 0
#define HSAD_EINVAL (-1)       /* bad size, window, level, null pointer, n_a = 0 somewhere */
#define HSAD_ENOMEM (-2)       /* workspace smaller than hsad_workspace_bytes' minimum */
#define HSAD_EHIP (-3)         /* a HIP launch or runtime call failed */
#define HSAD_EUNSUPPORTED (-4) /* size or precision combination not built */

/* precision of the window covariance (Gram).  The reduced precisions (FP32, BF16, FP16)
 * need an annulus of at least 2 L' samples (outer^2 - inner^2 >= 2 L'); with fewer the
 * covariance is (nearly) singular and the call returns HSAD_EUNSUPPORTED.  Pixels near the
 * image borders whose clipped annulus holds fewer than 2 L' samples take the FP64 Gram. */
#define HSAD_PREC_AUTO 0       /* exact: FP64 sums / FP64 MFMA Gram, FP64 factorisation */
#define HSAD_PREC_FP32 1       /* FP32 MFMA Gram on exactly centred samples, FP64 factor */
#define HSAD_PREC_FP64 2       /* same as AUTO, requested explicitly */
#define HSAD_PREC_GRAM_BF16 3  /* BF16 MFMA Gram (FP32 accumulate), FP64 factorisation */
#define HSAD_PREC_GRAM_FP16 4  /* FP16 MFMA Gram (FP32 accumulate), FP64 factorisation */

/* operations (for hsad_workspace_bytes) */
#define HSAD_OP_LRX 1
#define HSAD_OP_DWRX 2
#define HSAD_OP_LRX_DWRX 3
#define HSAD_OP_DWEST 4

#define HSAD_MAX_LP 512        /* largest reduced band count the detectors accept */
#define HSAD_MAX_WINDOW 63     /* largest outer window side */

typedef struct hsad_window_params {
    int32_t inner;     /* odd inner (guard) window side, or 0 = none */
    int32_t outer;     /* odd outer window side, > inner, <= HSAD_MAX_WINDOW */
    double load_rel;   /* diagonal loading relative to tr(C)/L' (LRX, DWRX); >= 0 */
    int32_t precision; /* HSAD_PREC_* */
    int32_t reserved;  /* must be 0 */
} hsad_window_params;

/* Library version string, e.g. "hsad 0.1.0 gfx950". */
const char *hsad_version(void);

/* Message of the last failing call on this thread ("" if none). */
const char *hsad_last_error(void);

/* Approximation length after `levels` analysis levels (Sec. 3, eq. 9 iterated on the
 * low-pass branch, Fig. 1).  An odd level input of length n is extended to n+1 by
 * repeating its last sample, so every level maps n to ceil(n/2).  Host only.
 * Returns HSAD_EINVAL if L < 1, levels < 0 or a level input would be shorter than 2. */
int hsad_dwt_out_len(int64_t L, int levels, int64_t *Lp);

/* Level count of Sec. 4 ("until four samples are left"): the largest J whose
 * approximation keeps at least `target` samples (target = 4 in the paper).  Returns
 * the level count (0 if L < 2*target-1), or HSAD_EINVAL for L < 1 or target < 1. */
int hsad_levels_for(int64_t L, int target);

/* Periodised Daubechies-4 (8-tap, 4 vanishing moments) DWT of every pixel spectrum,
 * keeping only the approximation coefficients (Sec. 4 "approximation matrix").
 * Each level computes y[k] = sum_m h[m] x[(2k - m) mod n]  (eq. 9, periodic index),
 * after the odd-length extension above.
 *   cube   : device, H*W*L float32, [y][x][band]
 *   approx : device, H*W*L' float32, [y][x][k]; must not overlap cube
 *   levels : 0 copies the cube
 * The first call for an (L, levels) pair on a device computes its composite filter table on
 * the host and enqueues the table's copy into a library-owned device arena (4 MiB, from a
 * pinned host mirror allocated on the first call) on `stream`, ahead of the transform;
 * calls on other streams wait for that copy through an event, and nothing synchronises.
 * Under graph capture the copy is captured with the transform.  A first call of the process
 * made under capture (no pinned mirror yet), or one for which the arena is full, uses the
 * level-by-level kernel instead, with the same results to rounding.
 * Errors: HSAD_EINVAL (H, W, L < 1, bad levels, null pointers), HSAD_EHIP. */
int hsad_dwt(const float *cube, int64_t H, int64_t W, int64_t L, int levels, float *approx,
             hipStream_t stream);

/* hsad_dwt, and two caller-created events (hipEventCreate, timing enabled; either may be
 * NULL) that the transform's kernel dispatch records at its start and its end
 * (hipExtLaunchKernel), so that the kernel's own duration can be read with
 * hipEventElapsedTime without event records around the call, which wait for the work
 * before them.  For callers that time the transform, as a benchmark does.  levels = 0 (a
 * copy) leaves the events untouched.  Errors as hsad_dwt. */
int hsad_dwt_timed(const float *cube, int64_t H, int64_t W, int64_t L, int levels, float *approx,
                   hipStream_t stream, hipEvent_t start, hipEvent_t stop);

/* ---------------------------------------------------------------------------------------
 * Full transform: approximation and every detail band (Sec. 3, Fig. 1), its inverse, and
 * the Daubechies family of any order (Fig. 2 shows the db16 scaling function)
 * -------------------------------------------------------------------------------------*/
/* Host only.  h (2 * order doubles) receives the minimum-phase Daubechies scaling filter
 * with `order` vanishing moments (order 1 is Haar, 4 the db4 of hsad_dwt), in the time
 * order of eq. (9), sum h = sqrt 2.  The library designs it by a spectral factorisation of
 * Daubechies' polynomial polished on its defining equations (orthonormal even shifts and
 * `order` vanishing moments of the high-pass) in long double.
 * Errors: HSAD_EINVAL (order outside 1..16, NULL h). */
int hsad_wavelet_filter(int order, double *h);

/* Length of [a_J d_J d_{J-1} ... d_1] after `levels` levels of a length-L signal: level j
 * maps n_{j-1} samples to a_j and d_j of n_j = ceil(n_{j-1}/2) samples each (the odd-length
 * extension of hsad_dwt applied to both branches), so n = n_J + sum_j n_j; L for levels 0.
 * Errors: HSAD_EINVAL (L < 1, levels < 0, a level input shorter than 2). */
int hsad_dwt_full_len(int64_t L, int levels, int64_t *n);

/* Full periodised DWT of every pixel spectrum with the order-`order` Daubechies pair:
 * level by level a_j[k] = sum_t h_t x[(2k - t) mod n_e], d_j[k] = sum_t g_t x[(2k - t) mod n_e]
 * with g_t = (-1)^t h_{2 order - 1 - t} (eqs. 8-9) after the odd-length extension (n_e the
 * even, extended length).  FP64 arithmetic, FP32 storage.
 *   cube : device, npix * L float32, [p][band]
 *   coef : device, npix * n float32 (n from hsad_dwt_full_len), [p][a_J d_J ... d_1]
 * Errors: HSAD_EINVAL (NULL, npix < 1, order outside 1..16, bad levels), HSAD_EUNSUPPORTED
 * (L > 4096), HSAD_EHIP. */
int hsad_dwt_full(const float *cube, int64_t npix, int64_t L, int levels, int order, float *coef,
                  hipStream_t stream);

/* Inverse of hsad_dwt_full: from the coarsest level, each level's synthesis is the
 * transpose of its analysis on the even length n_e (an orthogonal matrix), and the repeated
 * sample of an odd level input is dropped, so hsad_idwt_full(hsad_dwt_full(x)) = x up to
 * rounding for every L.  Same arguments as hsad_dwt_full with the roles of the buffers
 * exchanged.  Errors as hsad_dwt_full. */
int hsad_idwt_full(const float *coef, int64_t npix, int64_t L, int levels, int order, float *cube,
                   hipStream_t stream);

/* Device workspace in bytes for `op` on an H x W x Lp reduced cube with these windows
 * (0 if none is needed).  Passing more lets the detectors process larger pixel chunks
 * per launch; passing less than this value but at least the minimum returned for a
 * 1 x 1 image is allowed and only costs launches.  Returns 0 on invalid arguments. */
size_t hsad_workspace_bytes(int op, int64_t H, int64_t W, int64_t Lp,
                            const hsad_window_params *p);

/* LRX: eq. (1) with a local background, the annulus of the pixel.  For pixel r:
 * mu, C = mean and 1/n covariance of the annulus samples,
 * score = (r - mu)^T (C + lambda I)^-1 (r - mu).
 * Exact precision (AUTO / FP64) computes the statistics in FP64: by sliding box sums for
 * L' <= 8 (fused with the factorisation) and for L' <= 128 with outer <= 31 (per-pixel
 * records in the workspace, then an FP64 Cholesky per pixel), otherwise by a per-pixel
 * matrix-core FP64 Gram.  The FP32 / BF16 / FP16 precisions always use the Gram.
 *   x      : device, H*W*Lp float32 reduced (or full-band) cube
 *   scores : device, H*W float32
 *   ws     : device workspace of ws_bytes (may be NULL when hsad_workspace_bytes is 0)
 * Errors: HSAD_EINVAL (sizes, windows, load_rel < 0, reserved != 0, Lp > HSAD_MAX_LP,
 * an empty annulus for some pixel), HSAD_ENOMEM, HSAD_EUNSUPPORTED, HSAD_EHIP. */
int hsad_lrx(const float *x, int64_t H, int64_t W, int64_t Lp, const hsad_window_params *p,
             float *scores, void *ws, size_t ws_bytes, hipStream_t stream);

/* DWRX: eq. (5), m_diff^T (C_outer + lambda I)^-1 m_diff with m_diff = inner-window mean
 * minus annulus mean (eq. 3) and C_outer the annulus covariance.  Needs inner >= 1.
 * Arguments and errors as hsad_lrx. */
int hsad_dwrx(const float *x, int64_t H, int64_t W, int64_t Lp, const hsad_window_params *p,
              float *scores, void *ws, size_t ws_bytes, hipStream_t stream);

/* LRX and DWRX from one pass (they share the annulus statistics and the factorisation).
 * Either output may be NULL (not both).  Arguments and errors as hsad_lrx. */
int hsad_lrx_dwrx(const float *x, int64_t H, int64_t W, int64_t Lp,
                  const hsad_window_params *p, float *lrx, float *dwrx, void *ws,
                  size_t ws_bytes, hipStream_t stream);

/* Device workspace for hsad_detect (bytes). */
size_t hsad_detect_workspace_bytes(int64_t H, int64_t W, int64_t Lp, const hsad_window_params *p);

/* The detection step in one call: LRX (eq. 1) and DWRX (eq. 5) as hsad_lrx_dwrx, then the
 * adaptive threshold of eq. (12) on the LRX map (Sec. 5.3.2) and its mask, as
 * hsad_threshold.  On the L' <= 8 box path the detector kernel also leaves the (count,
 * mean, M2) of each 16 x 16 tile's finite LRX scores, which replaces the threshold's own
 * statistics pass; the tiles are merged in a fixed order (deterministic).
 *   lrx    : device, H*W float32 (required); dwrx: device, H*W float32 or NULL
 *   stats  : device, 4 doubles written {count, mu_d, sigma_d, tau}
 *   mask   : device, H*W uint8 written (lrx > tau), or NULL
 *   ws     : device workspace of at least hsad_detect_workspace_bytes
 * Errors: as hsad_lrx_dwrx and hsad_threshold. */
int hsad_detect(const float *x, int64_t H, int64_t W, int64_t Lp, const hsad_window_params *p,
                double z_alpha, float *lrx, float *dwrx, double *stats, uint8_t *mask, void *ws,
                size_t ws_bytes, hipStream_t stream);

/* The DWT of one cube (Sec. 3, as hsad_dwt) and the detection step on another, already
 * reduced cube (as hsad_detect), with the same results as hsad_dwt followed by hsad_detect.
 * For a stream of cubes this is one step of a software pipeline: the call that scores cube
 * k reduces cube k + 1 into the other of two reduced buffers.  The two share one launch
 * when both halves are given, L' <= 5, L is a multiple of 4, the precision is exact and a
 * workgroup of each role fits one CU's LDS together (outer windows up to 15 x 15 at
 * L' = 4, 19 x 19 at L' = 2, 21 x 21 at L' = 5): the transform is bound by HBM bandwidth
 * and the detector by FP64 arithmetic and LDS, and a CU holds one workgroup of each, so
 * their times overlap instead of adding.  Otherwise the two run one after the other on the
 * stream.
 *   cube_next    : device, H*W*L float32 [y][x][band], or NULL (no transform: hsad_detect);
 *                  must not overlap the detector's outputs
 *   L, levels    : as hsad_dwt; their L' must equal Lp
 *   approx_next  : device, H*W*Lp float32 written; must not overlap any other argument
 *   x            : device, H*W*Lp float32, the cube to score, or NULL (transform only:
 *                  hsad_dwt; p, z_alpha, lrx, dwrx, stats, mask and ws are then ignored)
 *   p ... ws_bytes : as hsad_detect
 *   start, stop  : events taken when the launch that holds the transform starts and ends
 *                  (the shared launch, or the transform's own), or NULL; not recorded when
 *                  cube_next is NULL
 * Errors: as hsad_dwt and hsad_detect; HSAD_EINVAL if both cubes are NULL, if the two L'
 * differ, if approx_next overlaps another argument or if cube_next overlaps lrx, dwrx,
 * mask, stats or ws (nothing is enqueued then). */
int hsad_dwt_detect_fused(const float *cube_next, int64_t L, int levels, float *approx_next,
                          const float *x, int64_t H, int64_t W, int64_t Lp, const hsad_window_params *p,
                          double z_alpha, float *lrx, float *dwrx, double *stats, uint8_t *mask, void *ws,
                          size_t ws_bytes, hipStream_t stream, hipEvent_t start, hipEvent_t stop);

/* One step of a three-stage pipeline over a stream of cubes, for the L' <= 8 box path of the
 * detection step: the DWT of cube k + 1 (Sec. 3), LRX + DWRX of cube k (eqs. 1, 5) with its
 * per-tile (count, mean, M2) partials left in ws, and the eq. (12) threshold and mask of
 * cube k - 1 (Sec. 5.3.2) from the scores and partials the previous call left.  Over two
 * calls the outputs for one cube equal hsad_detect's bit for bit (the partials are merged in
 * hsad_detect's fixed order).  When L' <= 5, L is a multiple of 4 and the LDS of the
 * transform's and the detector's workgroups fits one CU together (as hsad_dwt_detect_fused),
 * and both cube_next and x are given, the three stages share one launch; otherwise they run
 * one after the other on the stream.  Any stage is skipped when its input is NULL.
 *   cube_next, L, levels, approx_next : as hsad_dwt_detect_fused; L' of (L, levels) = Lp
 *   x      : device, H*W*Lp float32, the reduced cube k, or NULL
 *   p      : window parameters; exact precision, L' <= 8 and windows the box path takes
 *   lrx, dwrx : device, H*W float32 written (dwrx may be NULL)
 *   ws     : device workspace of at least hsad_detect_workspace_bytes; receives cube k's
 *            partials
 *   prev_lrx  : device, H*W float32, cube k - 1's LRX map, or NULL
 *   prev_ws   : the workspace the call that scored cube k - 1 filled (same H, W, Lp and
 *               windows); also scratch for the merge when the image has more than 1024 tiles
 *   z_alpha, prev_stats, prev_mask : as hsad_detect's z_alpha, stats and mask (mask may be
 *               NULL), for cube k - 1
 *   start, stop : events taken when the launch that holds the transform starts and ends, or
 *               NULL; not recorded when cube_next is NULL
 * No two arguments that one stage writes may overlap any other argument.
 * Errors: HSAD_EINVAL (nothing to do, an overlap, a missing output, the two L' differ);
 * HSAD_EUNSUPPORTED when the detector is not on the exact box path; as hsad_dwt and
 * hsad_detect otherwise.  Nothing is enqueued on an error found on the host. */
int hsad_detect_stream_step(const float *cube_next, int64_t L, int levels, float *approx_next, const float *x,
                            int64_t H, int64_t W, int64_t Lp, const hsad_window_params *p, float *lrx, float *dwrx,
                            void *ws, size_t ws_bytes, const float *prev_lrx, void *prev_ws, double z_alpha,
                            double *prev_stats, uint8_t *prev_mask, hipStream_t stream, hipEvent_t start,
                            hipEvent_t stop);

/* Size of the static device array hsad_detect_noalloc takes its workspace from. */
#define HSAD_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): hsad_detect with the same arguments
 * and results, except that the workspace is a static device array of
 * HSAD_NOALLOC_SCRATCH_BYTES bytes instead of a caller buffer.  Each GPU the library runs
 * on holds its own copy of the array from the first load of the library until the process
 * ends; its address is looked up once per device on the first call there.  The call
 * allocates and frees nothing (no hipMalloc, hipFree or allocating library routine).
 * The array keeps what the last call left in it; nothing in it needs clearing.  All calls
 * on one GPU share the array, so calls that overlap on one GPU (from any stream or
 * thread) race and must be serialised by the caller.
 * Errors: as hsad_detect; HSAD_ENOMEM (with the sizes in the message) when the smallest
 * workspace hsad_detect accepts for these arguments exceeds HSAD_NOALLOC_SCRATCH_BYTES
 * (nothing is enqueued then). */
int hsad_detect_noalloc(const float *x, int64_t H, int64_t W, int64_t Lp, const hsad_window_params *p,
                        double z_alpha, float *lrx, float *dwrx, double *stats, uint8_t *mask,
                        hipStream_t stream);

/* DWEST, eqs. (2)-(4): C_diff = C_inner - C_annulus, m_diff = m_inner - m_annulus.
 * The eigenvalues of C_diff and the projections v_i^T m_diff come from an FP64
 * Householder tridiagonalisation followed by the implicit QL iteration, with every
 * transform also applied to m_diff (the eigenvectors are never formed); the eigenvalues
 * > 1e-12 * max|eigenvalue| are "positive".  A pixel whose QL iteration does not converge
 * within 64 sweeps per eigenvalue gets NaN scores and npos = -1.  With the workspace
 * hsad_workspace_bytes reports, the tridiagonal forms of up to 2^20 pixels are kept in it
 * (3 L' doubles each) so that one QL launch covers them all; a smaller workspace (down to
 * the 1 x 1 minimum) runs the same arithmetic chunk by chunk.
 * Outputs, each a device [y][x] array:
 *   scores         : ||V_P^T m_diff||_2 (invariant to eigenvector signs), float32
 *   scores_literal : sum_P |v_i^T m_diff| (eq. 4 with each v_i signed so that its
 *                    projection is >= 0), float32, may be NULL
 *   npos           : |P| per pixel, int32, may be NULL
 * Needs inner >= 1.  load_rel is ignored (DWEST does not invert a covariance).
 * Errors as hsad_lrx. */
int hsad_dwest(const float *x, int64_t H, int64_t W, int64_t Lp, const hsad_window_params *p,
               float *scores, float *scores_literal, int32_t *npos, void *ws,
               size_t ws_bytes, hipStream_t stream);

/* Device workspace of hsad_global_rx (bytes; 0 for npix < 1, L' < 1 or L' > 256). */
size_t hsad_global_rx_workspace_bytes(int64_t npix, int64_t Lp);

/* Global RX: eq. (1) of Sec. 2.1 with the background formed by all npix pixels of the
 * image (the detector the paper's local variants start from).
 *   mu = (1/N) sum_p x_p,  C = (1/N) sum_p (x_p - mu)(x_p - mu)^T  (two passes, exact centring),
 *   score_p = (x_p - mu)^T (C + lambda I)^-1 (x_p - mu),  lambda = load_rel tr(C)/L' (>= 1e-30).
 * FP64 sums (the Gram on FP64 matrix cores), an FP64 Cholesky of C + lambda I and its
 * inverse, then every score as the squared norm of L^-1 (x_p - mu), also on matrix cores.
 * All reductions run in a fixed order (deterministic).  If C + lambda I is not
 * numerically positive definite (or the cube holds a non-finite value) every score is +inf.
 *   x      : device, npix * L' float32, [p][k] (any image of npix pixels, e.g. H * W)
 *   scores : device, npix float32
 *   mean   : device, L' doubles written (mu), or NULL
 *   cov    : device, L' * L' doubles written (C before loading, row-major), or NULL
 *   ws     : device workspace of at least hsad_global_rx_workspace_bytes(npix, L')
 * Errors: HSAD_EINVAL (NULL x / scores, npix or L' < 1, load_rel < 0 or not finite),
 * HSAD_EUNSUPPORTED (L' > 256, npix > 2^31), HSAD_ENOMEM, HSAD_EHIP. */
int hsad_global_rx(const float *x, int64_t npix, int64_t Lp, double load_rel, float *scores,
                   double *mean, double *cov, void *ws, size_t ws_bytes, hipStream_t stream);

/* Device workspace for hsad_threshold (bytes; independent of the caller's stream). */
size_t hsad_threshold_workspace_bytes(int64_t n);

/* Adaptive cut-off of eq. (12), tau = mu_d + z_alpha * sigma_d (Sec. 5.3.2).  mu_d and
 * sigma_d are the mean and population standard deviation of the finite entries of the
 * anomaly map.  They come from two FP64 passes with a fixed reduction tree, so the
 * result is deterministic.
 *   scores : device, n float32
 *   stats  : device, 4 doubles written {count, mu_d, sigma_d, tau}
 *   mask   : device, n uint8 written (scores > tau), or NULL for stats only
 * Errors: HSAD_EINVAL (n < 1, NULL scores/stats, non-finite z_alpha), HSAD_ENOMEM, HSAD_EHIP. */
int hsad_threshold(const float *scores, int64_t n, double z_alpha, double *stats, uint8_t *mask,
                   void *ws, size_t ws_bytes, hipStream_t stream);

/* Device workspace for hsad_auc (bytes). */
size_t hsad_auc_workspace_bytes(int64_t n);

/* Exact pixel-level ROC AUC counts (Sec. 5.3.1): over all pairs (positive p, negative q)
 * of the truth mask, counts[0] = #{s_p > s_q}, counts[1] = #{s_p == s_q}, counts[2] =
 * number of positives, counts[3] = number of negatives (device, 4 uint64).  The area is
 * (counts[0] + counts[1]/2) / (counts[2] * counts[3]).  Scores must be finite (NaN compares
 * false).  Cost is n x positives comparisons.
 * Errors: HSAD_EINVAL, HSAD_ENOMEM, HSAD_EHIP. */
int hsad_auc(const float *scores, const uint8_t *truth, int64_t n, uint64_t *counts, void *ws,
             size_t ws_bytes, hipStream_t stream);


/* ---------------------------------------------------------------------------------------
 * Uneven batches of scenes (persistent work-queue kernels, graph-capturable runs)
 * -------------------------------------------------------------------------------------*/
typedef struct hsad_scene {
    const float *cube;  /* device, H*W*L float32 [y][x][band] */
    float *approx;      /* device, H*W*L' float32, written (reduced cube) */
    float *lrx;         /* device, H*W float32, written, or NULL */
    float *dwrx;        /* device, H*W float32, written, or NULL (needs params.inner >= 1) */
    int64_t H, W, L;    /* L <= 4096, H*W <= 2^30 */
    int32_t levels;     /* DWT depth (Sec. 3); the reduced length L' must be <= 128 */
    int32_t reserved;   /* must be 0 */
    hsad_window_params params; /* precision must be AUTO or FP64 */
} hsad_scene;

typedef struct hsad_batch_options {
    int32_t wgs_per_cu;   /* persistent workgroups per CU (1..16) */
    int32_t dwt_pixels;   /* pixels per DWT work item, 0 = as many as fit 48 KiB of LDS */
    int64_t chunk_bytes;  /* Gram/Cholesky scratch per chunk (>= 1 MiB) */
    int32_t reserved;     /* must be 0 */
    int32_t pad;
} hsad_batch_options;

typedef struct hsad_batch_plan hsad_batch_plan;   /* opaque, host memory */

/* Default options (what hsad_batch_plan_create uses when opt is NULL). */
void hsad_batch_default_options(hsad_batch_options *opt);

/* Host-only: validates every scene and builds the work lists.  The detectors are the same
 * as hsad_dwt + hsad_lrx_dwrx per scene (same definitions and tolerances): scenes with
 * L' <= 8 go through the box-sum bucket, the others through the matrix-core Gram and FP64
 * Cholesky.  The work is ordered by estimated cost (largest first) and cut into items.
 * Errors: HSAD_EINVAL (NULL, sizes, windows, options), HSAD_EUNSUPPORTED (L' > 128). */
int hsad_batch_plan_create(const hsad_scene *scenes, int n, const hsad_batch_options *opt,
                           hsad_batch_plan **plan);

/* Device workspace the plan needs (queue counters, tables, Gram scratch). */
size_t hsad_batch_workspace_bytes(const hsad_batch_plan *plan);

/* Copies the plan's tables into ws and synchronises `stream` (one time, not capturable). */
int hsad_batch_upload(hsad_batch_plan *plan, void *ws, size_t ws_bytes, hipStream_t stream);

/* Enqueues the whole batch on `stream`: a counter reset (fill kernel), one persistent DWT
 * kernel, one persistent kernel per box bucket, and per Gram chunk the persistent Gram
 * kernels and one persistent Cholesky kernel.  No allocation, copy, memset or host
 * synchronisation, so it may be captured into a HIP graph and replayed.  ws must be the
 * workspace passed to hsad_batch_upload; runs on one workspace must not overlap. */
int hsad_batch_run(const hsad_batch_plan *plan, void *ws, hipStream_t stream);

/* Frees the host plan. */
int hsad_batch_plan_destroy(hsad_batch_plan *plan);

/* Autotuner: times every candidate schedule on this batch with HIP events, one warm-up
 * and one timed run each, and stores the fastest in *best.  The candidates cover
 * persistent workgroups per CU {1,2,4}, DWT item size {max, 8} and Gram chunk bytes
 * {1 GiB, 4 GiB}; those whose workspace exceeds ws_bytes are skipped.  If cache_path
 * is not NULL, the result is cached there as JSON keyed by GPU architecture, the library
 * build (a hash of its sources) and the batch signature (shapes, levels, windows), and a
 * cached entry whose plan fits ws_bytes is returned without timing (*best_ms = -1); one
 * that does not fit is tuned again.  ws is overwritten.  Synchronises `stream`.
 * Errors: HSAD_EINVAL, HSAD_ENOMEM (no candidate fits), HSAD_EHIP. */
int hsad_batch_autotune(const hsad_scene *scenes, int n, void *ws, size_t ws_bytes,
                        hipStream_t stream, const char *cache_path, hsad_batch_options *best,
                        double *best_ms);

/* info[0..7] = {scenes, pixels, DWT items, box items, Gram items, Gram chunks,
 * box-bucket pixels, Gram-bucket pixels}; n >= 8. */
int hsad_batch_plan_info(const hsad_batch_plan *plan, int64_t *info, int n);

/* ---------------------------------------------------------------------------------------
 * Exact LRX/DWRX at a list of pixels
 * -------------------------------------------------------------------------------------*/
/* LRX (eq. 1) and DWRX (eq. 5) of the pixels idx[0..nidx) of the reduced cube x (same
 * definitions, windows and loading as hsad_lrx_dwrx), computed by the FP64 matrix-core
 * Gram and the FP64 Cholesky.  Only lrx[idx[j]] / dwrx[idx[j]] are written; the rest of
 * the maps is left as it was.  Duplicates are allowed.  ws needs at least (L'+2) L' doubles; larger
 * workspaces process more pixels per chunk (up to 192 MiB worth).  precision must be
 * AUTO or FP64.  The statistics come from the per-pixel matrix-core Gram (the full-map
 * calls may use sliding box sums instead; both are exact FP64 paths within the same
 * tolerance).  Entries of idx outside [0, H*W) are skipped.
 * Errors: HSAD_EINVAL, HSAD_ENOMEM, HSAD_EHIP. */
int hsad_lrx_dwrx_at(const float *x, int64_t H, int64_t W, int64_t Lp, const hsad_window_params *p,
                     const int32_t *idx, int64_t nidx, float *lrx, float *dwrx, void *ws, size_t ws_bytes,
                     hipStream_t stream);

/* ---------------------------------------------------------------------------------------
 * Learned surrogate of the LRX score
 *
 * Not part of the paper: a per-pixel MLP that predicts log1p(LRX) (eq. 1) from local
 * features, so that the exact detector only runs where the prediction is close to the
 * eq. (12) threshold, plus a seeded audit sample that measures the prediction error and
 * triggers an exact fallback.
 *   Features (D = 3 L'), for each band i of the reduced cube, over the annulus
 *   (outer minus inner window): z_i = (x_i - mu_i)/sqrt(v_i + 1e-12), log(v_i + 1e-12)
 *   and mu_i, where mu_i and v_i are the annulus mean and 1/n variance.
 *   Network: D inputs (normalised per column, zero padded to Dp = 32 ceil(D/32) <= 256)
 *   -> 128 ReLU -> 128 ReLU -> 1.  BF16 matrix-core products with FP32 accumulation.
 *   Parameters (FP32, nparams values): W1 [Dp][128], b1 [128], W2 [128][128], b2 [128],
 *   w3 [128], b3, 3 padding values.  h1 = relu(x W1 + b1), h2 = relu(h1 W2 + b2),
 *   y = h2 . w3 + b3.  The BF16 copy (nbf16 values) holds W1 transposed [128][Dp],
 *   W2 transposed [128][128] and W2 [128][128]; hsad_mlp_sync and every training step
 *   keep it equal to the rounded FP32 weights.
 * -------------------------------------------------------------------------------------*/
typedef struct hsad_mlp_model {
    const float *params;   /* device, nparams FP32 */
    const uint16_t *wbf;   /* device, nbf16 BF16 bit patterns */
    const float *norm;     /* device, 2 D floats: {shift, scale} per input column */
    int64_t Lp;            /* reduced band count the model was trained for */
    int32_t Dp;            /* padded input width */
    int32_t reserved;      /* must be 0 */
    double rmse_val;       /* validation RMSE of log1p(score) */
} hsad_mlp_model;

typedef struct hsad_surrogate_options {
    double z_alpha;         /* eq. (12) */
    double band_k;          /* band half-width = band_k * rmse_val around log1p(tau) */
    double audit_frac;      /* fraction of pixels audited (seeded, uniform), 0..1 */
    double fallback_factor; /* exact fallback when the audit RMSE > fallback_factor * rmse_val */
    uint64_t seed;          /* audit stream seed */
    double band_quantile;   /* 0, or widen the band to this quantile of the audited |error|, [0, 1) */
    double max_exact_frac;  /* exact fallback when more than this fraction would be recomputed, (0, 1] */
    int32_t exact_above;    /* 1: also recompute every pixel predicted above the band (the detections) */
    int32_t reserved;       /* must be 0 */
} hsad_surrogate_options;

typedef struct hsad_surrogate_report {
    int64_t pixels;      /* H * W */
    int64_t selected;    /* pixels scored exactly (H * W after a fallback) */
    int64_t band;        /* pixels inside the near-threshold band */
    int64_t audit;       /* audited pixels */
    double audit_rmse;   /* RMSE of the prediction on the audit, log1p space */
    double audit_max;    /* largest |error| on the audit, log1p space */
    double tau_pred;     /* eq. (12) threshold of the predicted map */
    double tau;          /* eq. (12) threshold of the final map */
    int32_t fallback;    /* 1 when the whole map was recomputed exactly */
    int32_t reserved;
    double band_width;   /* half-width of the recomputed band, log1p space */
    int64_t audit_flips; /* audited pixels whose predicted and exact scores lie on different
                            sides of the predicted map's eq. (12) threshold */
} hsad_surrogate_report;

/* Sizes for a reduced band count: D = 3 L', Dp, nparams (FP32) and nbf16 (BF16) counts.
 * Errors: HSAD_EINVAL (L' outside 1..85). */
int hsad_mlp_dims(int64_t Lp, int32_t *D, int32_t *Dp, int64_t *nparams, int64_t *nbf16);

/* Features of every pixel of the reduced cube x.  With norm == NULL, writes FP32 rows
 * feat [H*W][3 L'] (z, log-variance, mean blocks); otherwise writes the normalised BF16
 * rows packed [H*W][Dp], (f - norm[2k]) * norm[2k+1], zero padded.  Windows as for LRX.
 * Errors: HSAD_EINVAL, HSAD_EHIP. */
int hsad_surrogate_features(const float *x, int64_t H, int64_t W, int64_t Lp, const hsad_window_params *p,
                            const float *norm, int32_t Dp, float *feat, uint16_t *packed, hipStream_t stream);

/* Column normalisation of an n x D FP32 matrix: norm[2c] = mean, norm[2c+1] = 1 / population
 * standard deviation (1 for a constant column).  Errors: HSAD_EINVAL, HSAD_EHIP. */
int hsad_mlp_norm_stats(const float *feat, int64_t n, int32_t D, float *norm, hipStream_t stream);

/* BF16 rows [n][Dp] = (feat - norm[2k]) * norm[2k+1], zero padded.  Errors: HSAD_EINVAL, HSAD_EHIP. */
int hsad_mlp_pack(const float *feat, int64_t n, int32_t D, int32_t Dp, const float *norm, uint16_t *out,
                  hipStream_t stream);

/* Training targets tgt = log1p(scores); non-finite scores give NaN, which training skips. */
int hsad_surrogate_targets(const float *scores, int64_t n, float *tgt, hipStream_t stream);

/* Refreshes the BF16 copy wbf from the FP32 parameters. */
int hsad_mlp_sync(const float *params, int32_t Dp, uint16_t *wbf, hipStream_t stream);

/* Predictions yhat[r] (log1p space) for n packed BF16 rows X [n][Dp].
 * Errors: HSAD_EINVAL, HSAD_EHIP. */
int hsad_mlp_infer(const uint16_t *X, int64_t n, int32_t Dp, const float *params, const uint16_t *wbf,
                   float *yhat, hipStream_t stream);

/* Workspace of hsad_mlp_gradient / hsad_mlp_train_step: one FP32 gradient partial per
 * 64 rows of the batch. */
size_t hsad_mlp_train_workspace_bytes(int64_t batch, int32_t Dp);

/* Gradient of the mean squared error (1/batch) sum_j (y(X[rows[j]]) - tgt[rows[j]])^2
 * with respect to the parameters: grad[0..nparams) and grad[nparams] = the loss.
 * X holds nX packed rows [nX][Dp] and tgt nX targets; rows[0..batch) selects the batch.
 * Entries of rows outside [0, nX) and rows whose target is NaN contribute nothing (the
 * mean still divides by batch).  The
 * forward pass uses the BF16 weights and rounds h1, h2 and the back-propagated errors to
 * BF16; sums of partials run in a fixed order, so repeated calls agree bitwise.
 * Errors: HSAD_EINVAL, HSAD_ENOMEM, HSAD_EHIP. */
int hsad_mlp_gradient(const uint16_t *X, int64_t nX, const float *tgt, const int32_t *rows, int64_t batch,
                      int32_t Dp, const float *params, const uint16_t *wbf, float *grad, void *ws, size_t ws_bytes,
                      hipStream_t stream);

/* One Adam step (Kingma and Ba 2015: beta1 0.9, beta2 0.999, eps 1e-8, bias correction
 * with `step` >= 1) on the FP32 parameters from the gradient of hsad_mlp_gradient;
 * updates adam_m, adam_v (nparams FP32 each, zero before step 1) and the BF16 copy.
 * loss (device, 1 float, may be NULL) receives the batch loss before the update. */
int hsad_mlp_train_step(const uint16_t *X, int64_t nX, const float *tgt, const int32_t *rows, int64_t batch,
                        int32_t Dp, float *params, uint16_t *wbf, float *adam_m, float *adam_v, int64_t step,
                        float lr, float *loss, void *ws, size_t ws_bytes, hipStream_t stream);

/* Workspace of hsad_error_stats (bytes). */
size_t hsad_error_stats_workspace_bytes(int64_t n);

/* Error of predictions against references, e = yhat - r with r = log1p(ref) when
 * ref_is_score, else ref.  Over rows with (flags[i] & flag_mask) != 0 (all rows when flags
 * is NULL) and finite e: out (device, 3 doubles) = {count, RMSE, max |e|}.  Fixed-order
 * reduction.  Errors: HSAD_EINVAL, HSAD_ENOMEM, HSAD_EHIP. */
int hsad_error_stats(const float *yhat, const float *ref, int32_t ref_is_score, const uint8_t *flags,
                     int32_t flag_mask, int64_t n, double *out, void *ws, size_t ws_bytes, hipStream_t stream);

/* Workspace of hsad_surrogate_select (bytes). */
size_t hsad_surrogate_select_workspace_bytes(int64_t n);

/* Pixels sent to the exact detector.  flags[i] = 1 when |yhat[i] - log1p(stats[3])| <= band
 * (NaN predictions included), plus 2 when the upper 32 bits of SplitMix64 output i of the
 * stream seeded with `seed` (state seed + (i+1) 0x9E3779B97F4A7C15, then the standard
 * finaliser) are below audit_frac * 2^32.  The indices of the flagged pixels are written to
 * idx in ascending order; counts (device, 3 uint32) = {flagged, band, audit}.  stats is
 * the device output of hsad_threshold.  Three launches, no atomics (deterministic).
 * Errors: HSAD_EINVAL, HSAD_ENOMEM, HSAD_EHIP. */
int hsad_surrogate_select(const float *yhat, int64_t n, const double *stats, double band, uint64_t seed,
                          double audit_frac, uint8_t *flags, int32_t *idx, uint32_t *counts, void *ws,
                          size_t ws_bytes, hipStream_t stream);

/* Workspace of hsad_surrogate_run (bytes). */
size_t hsad_surrogate_workspace_bytes(int64_t H, int64_t W, int64_t Lp, int32_t Dp, const hsad_window_params *p);

/* Hybrid LRX map of the reduced cube x: features, predictions, eq. (12) on the predicted
 * scores expm1(yhat), selection (hsad_surrogate_select with band = band_k * rmse_val),
 * exact LRX at the selected pixels, audit statistics, and, when the audit RMSE exceeds
 * fallback_factor * rmse_val, exact LRX of the whole map.  With band_quantile > 0 the
 * audit's |error| histogram (bins of 1/256 in log1p space) sets a wider band when its
 * band_quantile quantile exceeds band_k * rmse_val; the pixels of that band are also
 * recomputed exactly, and when the band and the audit together exceed max_exact_frac of
 * the pixels the whole map is recomputed instead.  With exact_above the band extends upward
 * without limit, so every predicted detection carries its exact score.  Then eq. (12) and the mask (if mask !=
 * NULL) of the final map.  scores: device, H*W float32 (exact at the selected pixels,
 * expm1(prediction) elsewhere).  rep: host.  Synchronises `stream` up to five times.
 * Errors: HSAD_EINVAL (arguments, model/cube mismatch), HSAD_ENOMEM, HSAD_EHIP. */
int hsad_surrogate_run(const float *x, int64_t H, int64_t W, int64_t Lp, const hsad_window_params *p,
                       const hsad_mlp_model *model, const hsad_surrogate_options *opt, float *scores,
                       uint8_t *mask, hsad_surrogate_report *rep, void *ws, size_t ws_bytes, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* HSAD_H */
