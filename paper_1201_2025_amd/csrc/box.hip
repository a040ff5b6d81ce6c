// box.hip -- fused window statistics + loading + Cholesky + LRX/DWRX for short spectra
// (L' <= 8), the regime of the paper's DWT-reduced detectors (Sec. 4: four samples).
//
// Statistics (Sec. 2.1 local background; Sec. 2.2 inner/outer windows).  For pixel p the
// annulus A = outer window \ inner window, both clipped to the image.  Its mean and 1/n
// covariance come from box sums of the features
//     f_i = x_i - ref_i          (L' linear features)
//     q_ij = f_i f_j, i <= j     (L'(L'+1)/2 quadratic features)
//     b = [pixel has a non-finite component]
// where ref is one pixel of the tile.  Every feature is exact in FP64: the difference of
// two FP32 values and the product of two such differences both fit in 53 bits.  The sums
// are FP64, so C = Q/n - mu_f mu_f^T keeps about 12 significant digits even when |mu_f|^2
// is 1e4 times the smallest eigenvalue of C.  This data-dependent cancellation rules
// out FP32 sums here.
//
// Per 32 x 16 output tile (512 threads, one output pixel each; 16 x 16 when the wider
// tile's LDS does not fit, and in the batch engine):
//   1. stage the (32+2R) x (16+2R) halo tile of the reduced cube in LDS (coalesced).  Pixels
//      outside the image or with a non-finite component take the reference value, and
//      the second kind is flagged;
//   2. for each feature chunk and each window (inner, then outer): vertical box sums,
//      one job per (column, block of 4 output rows) with every feature of the chunk in
//      registers, over only the columns that window's horizontal sums read; then the
//      horizontal window sums in short sliding segments of 8 outputs per job (the first
//      sum of a segment taken directly, the next ones by adding the entering column and
//      subtracting the leaving one).  S = outer - inner gives the annulus sums directly;
//   3. mu, C, diagonal loading lambda = load_rel tr(C)/L' (floor 1e-30), Cholesky in
//      registers (FP64), z = L^-1 d and score = |z|^2 for d = x_p - mu (LRX, eq. 1)
//      and d = m_in - mu (DWRX, eq. 5).
//   A non-finite sample in the annulus makes the covariance non-finite, and the score
//   is +inf as in the definition.  A non-finite centre or inner-window value propagates
//   through d, from the raw values (a rare path that re-reads the inner window).
// HBM traffic is the reduced cube once (the halo re-reads hit L2) and the score maps.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include "internal.hpp"
#include "dev_box.hpp"
#include "dev_dwt.hpp"
#include "dev_thr.hpp"

namespace hsad {

template <int LP, int GCMAX, int TXW>
__global__ __launch_bounds__(TXW * TY) void box_lrx_dwrx_kernel(const float *__restrict__ x, int H,
                                                                int W, int R, int RI, int has_inner,
                                                                double load_rel,
                                                                float *__restrict__ lrx,
                                                                float *__restrict__ dwrx,
                                                                double *__restrict__ part)
{
    extern __shared__ double smem[];
    box_tile<LP, GCMAX, TXW>(x, H, W, R, RI, has_inner, load_rel, lrx, dwrx, blockIdx.y, blockIdx.x, smem,
                             part);
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

// LDS use of the default variant is at most that of the 15-feature chunk
bool box_supported(int64_t Lp, const Windows &w)
{
    return Lp >= 1 && Lp <= 8 && box_smem_lp(Lp, w.ro) <= kBoxMaxSmem;
}

static int g_box_gc = 0;   // 0: default feature chunk; 15 / 8 / 5 forced (tuning, tests)
static int g_box_tx = 0;   // 0: widest tile whose LDS fits; 16 forced (tuning, tests)

// default chunk width per L' (features per round of vertical and horizontal sums; the
// tile keeps L' + L'(L'+1)/2 + 1 features): the fastest of 5 / 8 / 15 for hsad_detect with
// 5 x 5 / 15 x 15 windows, at 512 x 512 and at 1024 x 1024 alike (32 x 16 tiles).  At
// 512 x 512, L' = 2: 18.0 vs 21.4 us (5); L' = 3: 24.1 vs 26.0 (8); L' = 4: 28.1 vs 30.4 (5);
// L' = 5: 40.2 vs 45.8 (15); L' = 6 / 7 / 8: 49.7 / 64.6 / 70.1 vs 59.7 / 73.4 / 94.0 (8)
static constexpr int kBoxBestGc[9] = {5, 5, 8, 5, 8, 5, 15, 15, 15};
static int box_gc(int Lp)
{
    return g_box_gc ? g_box_gc : kBoxBestGc[Lp >= 0 && Lp <= 8 ? Lp : 0];
}

template <int LP, int GCMAX> static int box_width(int R)
{
    // 32 x 16 tiles: 9-10 % faster than 16 x 16 at L' = 4 and 7 (512^2 and 1024^2, 15 x 15
    // outer windows), bit-identical sums
    return g_box_tx != 16 && box_smem<LP, GCMAX, 32>(R) <= kBoxMaxSmem ? 32 : 16;
}

template <int LP> static int box_width_lp(int R)
{
    const int gc = box_gc(LP);
    return gc == 8 ? box_width<LP, 8>(R) : gc == 15 ? box_width<LP, 15>(R) : box_width<LP, 5>(R);
}

template <int LP, int GCMAX, int TXW>
static int box_launch_tw(const float *x, int64_t H, int64_t W, const Windows &w, double load_rel,
                         float *lrx, float *dwrx, double *part, hipStream_t s)
{
    const size_t sh = box_smem<LP, GCMAX, TXW>(w.ro);
    if (int rc = allow_lds((const void *)box_lrx_dwrx_kernel<LP, GCMAX, TXW>, sh, "box_lrx_dwrx_kernel"))
        return rc;
    dim3 grid((unsigned)((W + TXW - 1) / TXW), (unsigned)((H + TY - 1) / TY)), block(TXW * TY);
    hipLaunchKernelGGL((box_lrx_dwrx_kernel<LP, GCMAX, TXW>), grid, block, sh, s, x, (int)H, (int)W, w.ro,
                       w.ri, w.inner > 0 ? 1 : 0, load_rel, lrx, dwrx, part);
    return check_launch("box_lrx_dwrx_kernel");
}

template <int LP, int GCMAX>
static int box_launch_gc(const float *x, int64_t H, int64_t W, const Windows &w, double load_rel,
                         float *lrx, float *dwrx, double *part, hipStream_t s)
{
    if (box_width<LP, GCMAX>(w.ro) == 32)
        return box_launch_tw<LP, GCMAX, 32>(x, H, W, w, load_rel, lrx, dwrx, part, s);
    return box_launch_tw<LP, GCMAX, 16>(x, H, W, w, load_rel, lrx, dwrx, part, s);
}

template <int LP>
static int box_launch(const float *x, int64_t H, int64_t W, const Windows &w, double load_rel,
                      float *lrx, float *dwrx, double *part, hipStream_t s)
{
    const int gc = box_gc(LP);
    switch (gc) {
    case 8: return box_launch_gc<LP, 8>(x, H, W, w, load_rel, lrx, dwrx, part, s);
    case 15: return box_launch_gc<LP, 15>(x, H, W, w, load_rel, lrx, dwrx, part, s);
    default: return box_launch_gc<LP, 5>(x, H, W, w, load_rel, lrx, dwrx, part, s);
    }
}

int wave_lrx_dwrx_launch(const float *x, int64_t H, int64_t W, int64_t Lp, const Windows &w,
                         double load_rel, float *lrx, float *dwrx, hipStream_t s);
bool wave_supported(int64_t Lp, const Windows &w);
int box_variant();

size_t box_tiles(int64_t H, int64_t W) { return (size_t)((H + TY - 1) / TY) * (size_t)((W + 15) / 16); }

size_t box_tiles_used(int64_t H, int64_t W, int64_t Lp, const Windows &w)
{
    int tw = 16;
    switch (Lp) {
    case 1: tw = box_width_lp<1>(w.ro); break;
    case 2: tw = box_width_lp<2>(w.ro); break;
    case 3: tw = box_width_lp<3>(w.ro); break;
    case 4: tw = box_width_lp<4>(w.ro); break;
    case 5: tw = box_width_lp<5>(w.ro); break;
    case 6: tw = box_width_lp<6>(w.ro); break;
    case 7: tw = box_width_lp<7>(w.ro); break;
    case 8: tw = box_width_lp<8>(w.ro); break;
    default: break;
    }
    return (size_t)((H + TY - 1) / TY) * (size_t)((W + tw - 1) / tw);
}

int box_lrx_dwrx_launch(const float *x, int64_t H, int64_t W, int64_t Lp, const Windows &w,
                        double load_rel, float *lrx, float *dwrx, hipStream_t s, double *part)
{
    if (H > (1 << 24) || W > (1 << 24)) return fail(HSAD_EUNSUPPORTED, "box path: image too large");
    const int v = box_variant();
    if (v == 2 && !part && wave_supported(Lp, w))
        return wave_lrx_dwrx_launch(x, H, W, Lp, w, load_rel, lrx, dwrx, s);
    switch (Lp) {
    case 1: return box_launch<1>(x, H, W, w, load_rel, lrx, dwrx, part, s);
    case 2: return box_launch<2>(x, H, W, w, load_rel, lrx, dwrx, part, s);
    case 3: return box_launch<3>(x, H, W, w, load_rel, lrx, dwrx, part, s);
    case 4: return box_launch<4>(x, H, W, w, load_rel, lrx, dwrx, part, s);
    case 5: return box_launch<5>(x, H, W, w, load_rel, lrx, dwrx, part, s);
    case 6: return box_launch<6>(x, H, W, w, load_rel, lrx, dwrx, part, s);
    case 7: return box_launch<7>(x, H, W, w, load_rel, lrx, dwrx, part, s);
    case 8: return box_launch<8>(x, H, W, w, load_rel, lrx, dwrx, part, s);
    default: return fail(HSAD_EUNSUPPORTED, "box path: L' > 8");
    }
}

// ------------------------------------------------------------------------------------
// One launch for the DWT of one cube and the detector on another, reduced cube (and the
// threshold of a third)
// ------------------------------------------------------------------------------------
// The LDS-staged DWT streams the cube from HBM and leaves the FP64 units mostly idle; the
// detector tile is bound by FP64 arithmetic, LDS traffic and barrier latency and leaves HBM
// idle.  Launched back to back their times add.  Here they are two roles of one grid of
// 512-thread workgroups (two per CU by LDS and registers): a DWT workgroup reduces 512
// pixels, a detector workgroup scores one 32 x 16 tile.  The roles alternate in runs of
// `run` workgroup ids, so that most CUs hold one workgroup of each and the detector's
// arithmetic runs under the DWT's HBM stream (at 512 x 512 x 224, J = 6, 5 / 15 windows:
// 52.6 us per launch with runs of 128 against 63 us for the two kernels back to back; runs
// of 8 to 512, two chunks of the cube in flight per DWT workgroup, and 256-thread
// workgroups with 16 x 16 tiles, three or four per CU, all measured slower).  Each role's
// arithmetic is that of its own kernel, so the results are bit-identical to the two
// launches.  Optionally a third role, placed after the other two, takes the eq. (12)
// threshold of an earlier map: each of its workgroups merges that map's tile partials in
// the threshold kernel's order (identical tau) and writes the mask of 2048 pixels, so a
// stream of cubes needs one launch per cube (53.5 us where the three kernels take 66 us).
constexpr int kFusedNT = 512;
static int g_fused_run = 128;   // role run length in workgroup ids (tuning, tests)

template <int LP, int VEC, int GCMAX>
__global__ __launch_bounds__(kFusedNT) __attribute__((amdgpu_waves_per_eu(4, 4))) void dwt_box_fused_kernel(
    const float *__restrict__ cube, int64_t npix, int L, const double *__restrict__ coef,
    float *__restrict__ approx, int nd, const float *__restrict__ x, int H, int W, int R, int RI,
    int has_inner, double load_rel, float *__restrict__ lrx, float *__restrict__ dwrx,
    double *__restrict__ part, int nb, int ntx, int run, FusedThr thr)
{
    extern __shared__ double smem[];
    const int b = blockIdx.x;
    if (b >= nd + nb) {
        // threshold role: eq. (12) of an earlier map from its tile partials, then the mask of
        // 2048 of its pixels
        constexpr int kPF = 4;
        const int idx = b - nd - nb, t = threadIdx.x;
        const int64_t i0 = (int64_t)idx * (kFusedNT * kPF) + t;
        float sv[kPF];
#pragma unroll
        for (int k = 0; k < kPF; ++k) {
            const int64_t i = i0 + k * kFusedNT;
            sv[k] = thr.s[i < npix ? i : npix - 1];
        }
        ThrParts pp;
        thr_load_parts(thr.part, thr.nblk, t, pp);
        const double tau = thr_merge_tau(pp, thr.nblk, thr.z, smem, smem + 3 * kThrMergeThreads,
                                         idx == 0 ? thr.stats : nullptr);
        if (thr.mask) {
#pragma unroll
            for (int k = 0; k < kPF; ++k) {
                const int64_t i = i0 + k * kFusedNT;
                if (i < npix) thr.mask[i] = ((double)sv[k] > tau) ? 1 : 0;
            }
        }
        return;
    }
    const int m = min(nd, nb) / run;   // full run pairs
    int role, idx;
    if (b < 2 * m * run) {
        role = (b / run) & 1;
        idx = (b / (2 * run)) * run + b % run;
    } else {
        const int r = b - 2 * m * run, dl = nd - m * run;
        role = r < dl ? 0 : 1;
        idx = m * run + (r < dl ? r : r - dl);
    }
    if (role == 0)
        dwt_equiv_lds_block<LP, VEC, true, kFusedNT>(cube, npix, L, coef, approx, reinterpret_cast<float *>(smem),
                                                     idx);
    else
        box_tile<LP, GCMAX, kFusedNT / TY, false>(x, H, W, R, RI, has_inner, load_rel, lrx, dwrx, idx / ntx, idx % ntx,
                                           smem, part, ntx);
}

template <int LP>
static int fused_launch(const float *cube, int64_t L, const double *coef, float *approx, const float *x,
                        int64_t H, int64_t W, const Windows &w, double load_rel, float *lrx, float *dwrx,
                        double *part, int64_t *nparts, const FusedThr *thr, hipStream_t s, hipEvent_t e0,
                        hipEvent_t e1)
{
    // the 32 x 16 detector tile with the default feature chunk: what hsad_detect runs
    constexpr int GC = kBoxBestGc[LP];
    constexpr int TXW = kFusedNT / TY;
    if (g_box_gc != 0 || g_box_tx == 16 || box_width<LP, GC>(w.ro) != TXW) return HSAD_EUNSUPPORTED;
    const size_t dwt_sh = (size_t)kFusedNT * kEqLd * sizeof(float);
    const size_t box_sh = box_smem<LP, GC, TXW>(w.ro);
    const size_t sh = box_sh > dwt_sh ? box_sh : dwt_sh;
    // two workgroups (one of each role) must fit a CU's 160 KiB of LDS
    if (2 * sh > 160 * 1024) return HSAD_EUNSUPPORTED;
    const int64_t npix = H * W;
    const int64_t nd = (npix + kFusedNT - 1) / kFusedNT;
    const int ntx = (int)((W + TXW - 1) / TXW);
    const int64_t nb = (int64_t)ntx * ((H + TY - 1) / TY);
    if (nd + nb > INT32_MAX) return HSAD_EUNSUPPORTED;
    // threshold role: one workgroup per 2048 pixels of the earlier map
    FusedThr tr{};
    int64_t nm = 0;
    if (thr) {
        if (thr->nblk < 1 || thr->nblk > kThrMergeThreads * kThrMergePer) return HSAD_EUNSUPPORTED;
        tr = *thr;
        nm = (npix + 4 * kFusedNT - 1) / (4 * kFusedNT);
    }
    if (nd + nb + nm > INT32_MAX) return HSAD_EUNSUPPORTED;
    const void *kern = (const void *)dwt_box_fused_kernel<LP, 4, GC>;
    if (int rc = allow_lds(kern, sh, "dwt_box_fused_kernel")) return rc;
    int Li = (int)L, ndi = (int)nd, Hi = (int)H, Wi = (int)W, R = w.ro, RI = w.ri, hi = w.inner > 0 ? 1 : 0;
    int nbi = (int)nb, ntxi = ntx, runi = g_fused_run;
    int64_t np = npix;
    void *args[] = {(void *)&cube, &np, &Li, (void *)&coef, (void *)&approx, &ndi, (void *)&x, &Hi, &Wi, &R, &RI,
                    &hi, &load_rel, (void *)&lrx, (void *)&dwrx, (void *)&part, &nbi, &ntxi, &runi, &tr};
    if (hipExtLaunchKernel(kern, dim3((unsigned)(nd + nb + nm)), dim3(kFusedNT), args, sh, s, e0, e1, 0) !=
        hipSuccess)
        return fail(HSAD_EHIP, "dwt_box_fused_kernel: launch failed");
    *nparts = nb;
    return check_launch("dwt_box_fused_kernel");
}

int dwt_box_fused_launch(const float *cube, int64_t L, int levels, float *approx, const float *x,
                         int64_t H, int64_t W, int64_t Lp, const Windows &w, double load_rel, float *lrx,
                         float *dwrx, double *part, int64_t *nparts, hipStream_t s, hipEvent_t e0, hipEvent_t e1,
                         const FusedThr *thr)
{
    // L' <= 5 and whole float4 band vectors: the forms where both roles fit 128 VGPRs (four
    // waves per SIMD, two workgroups per CU) without spilling
    if (Lp < 1 || Lp > 5 || L % 4 != 0 || g_fused_run < 1 || H > (1 << 24) || W > (1 << 24) ||
        L > INT32_MAX || !box_supported(Lp, w))
        return HSAD_EUNSUPPORTED;
    const double *coef = dwt_lds_coefs(L, levels, Lp, s);
    if (!coef) return HSAD_EUNSUPPORTED;
    switch (Lp) {
#define HSAD_FUSED_CASE(n) \
    case n: \
        return fused_launch<n>(cube, L, coef, approx, x, H, W, w, load_rel, lrx, dwrx, part, nparts, thr, s, e0, e1);
        HSAD_FUSED_CASE(1) HSAD_FUSED_CASE(2) HSAD_FUSED_CASE(3) HSAD_FUSED_CASE(4) HSAD_FUSED_CASE(5)
#undef HSAD_FUSED_CASE
    default: return HSAD_EUNSUPPORTED;
    }
}

}  // namespace hsad

extern "C" int hsad_internal_fused_run(int run)
{
    if (run < 1) return -1;
    hsad::g_fused_run = run;
    return 0;
}

extern "C" int hsad_internal_box_chunk(int gc)
{
    hsad::g_box_gc = gc;
    return 0;
}

extern "C" int hsad_internal_box_width(int tx)
{
    if (tx != 0 && tx != 16) return -1;
    hsad::g_box_tx = tx;
    return 0;
}

// =====================================================================================
// Wave-row variant: no LDS tile, no workgroup barriers.
//
// One wavefront owns `rpw` consecutive output rows and 64 - 2R consecutive output
// columns.  Lane l holds image column x0 - R + l.  It reads the 2R+1 pixels of its
// column window directly from global memory (one coalesced vector load per row; the
// reduced cube stays in L2), keeps the vertical box sums of every feature in registers
// and slides them down the rows.  The horizontal window sums come from cross-lane
// doubling: B1 = V, B2 = B1 + B1(l+1), B4, B8, ..., combined over the binary digits of the
// window width.  Output lane l then holds the sums of lanes l .. l+2R, which is the outer
// window of image column x0 + l.  Same features, exact FP64 sums and scoring as the tile
// kernel above.
// =====================================================================================
namespace hsad {
namespace {

// sum over lanes l .. l+w-1 of v (lanes past 63 contribute their own value, never read
// by an output lane because l + w - 1 <= 63 there)
__device__ __forceinline__ double lane_window_sum(double v, int w)
{
    double blk = v;      // block of 2^k lanes starting at l
    double acc = 0.0;
    int off = 0;
    for (int k = 0; (1 << k) <= w; ++k) {
        if (w & (1 << k)) {
            // take block of size 2^k starting at l + off
            acc += __shfl_down(blk, off, 64);
            off += 1 << k;
        }
        const int step = 1 << k;
        if ((2 << k) <= w) blk += __shfl_down(blk, step, 64);
    }
    return acc;
}

template <int LP>
__device__ __forceinline__ void load_pixel(const float *__restrict__ x, int H, int W, int gy,
                                           int gx, const double *ref, double *f, double &b)
{
    b = 0.0;
#pragma unroll
    for (int i = 0; i < LP; ++i) f[i] = 0.0;
    if (gy < 0 || gy >= H || gx < 0 || gx >= W) return;
    const float *src = x + ((size_t)gy * W + gx) * LP;
    float v[LP];
    if constexpr (LP % 4 == 0) {
#pragma unroll
        for (int k = 0; k < LP / 4; ++k) {
            const float4 q = reinterpret_cast<const float4 *>(src)[k];
            v[4 * k] = q.x;
            v[4 * k + 1] = q.y;
            v[4 * k + 2] = q.z;
            v[4 * k + 3] = q.w;
        }
    } else {
#pragma unroll
        for (int i = 0; i < LP; ++i) v[i] = src[i];
    }
    bool fin = true;
#pragma unroll
    for (int i = 0; i < LP; ++i) fin = fin && isfinite(v[i]);
    if (!fin) {
        b = 1.0;
        return;
    }
#pragma unroll
    for (int i = 0; i < LP; ++i) f[i] = (double)v[i] - ref[i];
}
}  // namespace

template <int LP, int RPW>
__global__ __launch_bounds__(256) void wave_lrx_dwrx_kernel(const float *__restrict__ x, int H,
                                                           int W, int R, int RI, int has_inner,
                                                           double load_rel, int ncb, int nrb,
                                                           float *__restrict__ lrx,
                                                           float *__restrict__ dwrx)
{
    using C = BoxCfg<LP, 64>;   // one chunk: every feature in registers
    const int lane = threadIdx.x & 63;
    const int wave = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (wave >= ncb * nrb) return;
    const int cb = wave % ncb, rbk = wave / ncb;
    const int OUTW = 64 - 2 * R;
    const int x0 = cb * OUTW, r0 = rbk * RPW;
    const int gx = x0 - R + lane;

    // wave-uniform reference pixel
    double ref[LP];
    {
        const int ry = min(r0, H - 1), rx = min(x0 + OUTW / 2, W - 1);
        const float *rp = x + ((size_t)ry * W + rx) * LP;
#pragma unroll
        for (int i = 0; i < LP; ++i) {
            const float v = rp[i];
            ref[i] = isfinite(v) ? (double)v : 0.0;
        }
    }

    double Vo[C::GT], Vi[C::GT];
#pragma unroll
    for (int g = 0; g < C::GT; ++g) {
        Vo[g] = 0.0;
        Vi[g] = 0.0;
    }
    for (int dy = -R; dy <= R; ++dy) {
        double f[LP], b;
        load_pixel<LP>(x, H, W, r0 + dy, gx, ref, f, b);
        const bool inn = has_inner && dy >= -RI && dy <= RI;
#pragma unroll
        for (int g = 0; g < C::GT; ++g) {
            const double v = feat<LP>(f, b, g);
            Vo[g] += v;
            if (inn) Vi[g] += v;
        }
    }

#pragma unroll
    for (int i = 0; i < RPW; ++i) {
        const int r = r0 + i;
        if (i > 0) {
            if (r >= H) break;
            double fa[LP], ba, fb[LP], bb;
            load_pixel<LP>(x, H, W, r + R, gx, ref, fa, ba);
            load_pixel<LP>(x, H, W, r - R - 1, gx, ref, fb, bb);
#pragma unroll
            for (int g = 0; g < C::GT; ++g) Vo[g] += feat<LP>(fa, ba, g) - feat<LP>(fb, bb, g);
            if (has_inner) {
                load_pixel<LP>(x, H, W, r + RI, gx, ref, fa, ba);
                load_pixel<LP>(x, H, W, r - RI - 1, gx, ref, fb, bb);
#pragma unroll
                for (int g = 0; g < C::GT; ++g) Vi[g] += feat<LP>(fa, ba, g) - feat<LP>(fb, bb, g);
            }
        }
        // horizontal sums: outer over lanes l..l+2R, inner over lanes l+R-RI..l+R+RI
        double S[C::GT];
        double sin_lin[LP];
        double in_bad = 0.0;
#pragma unroll
        for (int g = 0; g < C::GT; ++g) {
            double so = lane_window_sum(Vo[g], 2 * R + 1);
            if (has_inner) {
                const double si = __shfl_down(lane_window_sum(Vi[g], 2 * RI + 1), R - RI, 64);
                so -= si;
                if (g < LP) sin_lin[g] = si;
                if (g == C::G) in_bad = si;
            }
            S[g] = so;
        }
        if (!has_inner) {
#pragma unroll
            for (int k = 0; k < LP; ++k) sin_lin[k] = 0.0;
        }
        const int px = x0 + lane;
        if (lane >= OUTW || px >= W || r >= H) continue;

        const int n_o = clip_count(r, R, H) * clip_count(px, R, W);
        const int n_i = has_inner ? clip_count(r, RI, H) * clip_count(px, RI, W) : 0;
        const double inv_na = 1.0 / (double)(n_o - n_i);
        const bool ann_bad = S[C::G] > 0.5;
        double mu[LP];
#pragma unroll
        for (int k = 0; k < LP; ++k) mu[k] = S[k] * inv_na;
        double Lm[LP][LP];
        double tr = 0.0;
        {
            int g = LP;
#pragma unroll
            for (int a = 0; a < LP; ++a)
#pragma unroll
                for (int c = a; c < LP; ++c) {
                    const double cv = S[g++] * inv_na - mu[a] * mu[c];
                    Lm[c][a] = cv;
                    if (a == c) tr += cv;
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
            const double inv = rsqrt(d);
            Lm[j][j] = inv;
#pragma unroll
            for (int a = j + 1; a < LP; ++a) {
                double t = Lm[a][j];
#pragma unroll
                for (int k = 0; k < j; ++k) t -= Lm[a][k] * Lm[j][k];
                Lm[a][j] = t * inv;
            }
        }
        const size_t o = (size_t)r * W + px;
        if (lrx) {
            const float *pc = x + o * LP;
            double z[LP], s = 0.0;
#pragma unroll
            for (int a = 0; a < LP; ++a) {
                double t = ((double)pc[a] - ref[a]) - mu[a];
#pragma unroll
                for (int k = 0; k < a; ++k) t -= Lm[a][k] * z[k];
                z[a] = t * Lm[a][a];
                s += z[a] * z[a];
            }
            lrx[o] = (pd && !ann_bad) ? (float)s : INFINITY;
        }
        if (dwrx) {
            if (in_bad > 0.5) {
#pragma unroll
                for (int k = 0; k < LP; ++k) sin_lin[k] = 0.0;
                for (int dy = -RI; dy <= RI; ++dy)
                    for (int dx = -RI; dx <= RI; ++dx) {
                        const int yy = r + dy, xx = px + dx;
                        if (yy < 0 || yy >= H || xx < 0 || xx >= W) continue;
                        const float *raw = x + ((size_t)yy * W + xx) * LP;
#pragma unroll
                        for (int k = 0; k < LP; ++k) sin_lin[k] += (double)raw[k] - ref[k];
                    }
            }
            const double inv_ni = 1.0 / (double)n_i;
            double z[LP], s = 0.0;
#pragma unroll
            for (int a = 0; a < LP; ++a) {
                double t = sin_lin[a] * inv_ni - mu[a];
#pragma unroll
                for (int k = 0; k < a; ++k) t -= Lm[a][k] * z[k];
                z[a] = t * Lm[a][a];
                s += z[a] * z[a];
            }
            dwrx[o] = (pd && !ann_bad) ? (float)s : INFINITY;
        }
    }
}

static int g_box_variant = 0;   // 0 auto, 1 tile kernel, 2 wave-row kernel

static int g_wave_rpw = 2;

template <int LP, int RPW>
static int wave_launch_rpw(const float *x, int64_t H, int64_t W, const Windows &w, double load_rel,
                           float *lrx, float *dwrx, hipStream_t s)
{
    const int outw = 64 - 2 * w.ro;
    const int ncb = (int)((W + outw - 1) / outw);
    const int nrb = (int)((H + RPW - 1) / RPW);
    const int64_t waves = (int64_t)ncb * nrb;
    dim3 grid((unsigned)((waves + 3) / 4)), block(256);
    hipLaunchKernelGGL((wave_lrx_dwrx_kernel<LP, RPW>), grid, block, 0, s, x, (int)H, (int)W, w.ro,
                       w.ri, w.inner > 0 ? 1 : 0, load_rel, ncb, nrb, lrx, dwrx);
    return check_launch("wave_lrx_dwrx_kernel");
}

template <int LP>
static int wave_launch(const float *x, int64_t H, int64_t W, const Windows &w, double load_rel,
                       float *lrx, float *dwrx, hipStream_t s)
{
    switch (g_wave_rpw) {
    case 1: return wave_launch_rpw<LP, 1>(x, H, W, w, load_rel, lrx, dwrx, s);
    case 4: return wave_launch_rpw<LP, 4>(x, H, W, w, load_rel, lrx, dwrx, s);
    default: return wave_launch_rpw<LP, 2>(x, H, W, w, load_rel, lrx, dwrx, s);
    }
}

bool wave_supported(int64_t Lp, const Windows &w) { return Lp >= 1 && Lp <= 8 && 2 * w.ro <= 40; }

int box_variant() { return g_box_variant; }

int wave_lrx_dwrx_launch(const float *x, int64_t H, int64_t W, int64_t Lp, const Windows &w,
                         double load_rel, float *lrx, float *dwrx, hipStream_t s)
{
    switch (Lp) {
    case 1: return wave_launch<1>(x, H, W, w, load_rel, lrx, dwrx, s);
    case 2: return wave_launch<2>(x, H, W, w, load_rel, lrx, dwrx, s);
    case 3: return wave_launch<3>(x, H, W, w, load_rel, lrx, dwrx, s);
    case 4: return wave_launch<4>(x, H, W, w, load_rel, lrx, dwrx, s);
    case 5: return wave_launch<5>(x, H, W, w, load_rel, lrx, dwrx, s);
    case 6: return wave_launch<6>(x, H, W, w, load_rel, lrx, dwrx, s);
    case 7: return wave_launch<7>(x, H, W, w, load_rel, lrx, dwrx, s);
    case 8: return wave_launch<8>(x, H, W, w, load_rel, lrx, dwrx, s);
    default: return fail(HSAD_EUNSUPPORTED, "wave path: L' > 8");
    }
}

}  // namespace hsad

extern "C" int hsad_internal_box_variant(int variant, int rpw)
{
    hsad::g_box_variant = variant;
    if (rpw == 1 || rpw == 2 || rpw == 4) hsad::g_wave_rpw = rpw;
    return 0;
}
