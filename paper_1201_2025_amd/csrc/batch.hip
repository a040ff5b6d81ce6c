// batch.hip -- uneven batches of scenes (different H, W, L, DWT depth and windows) run by
// persistent work-queue kernels.
//
// A plan is built on the host once per batch.  It validates every scene, sorts the work
// by estimated cost, cuts it into work items and lays out one device workspace.  That
// workspace holds queue counters, the scene table, the item lists and the
// Gram-factorisation scratch.  hsad_batch_upload copies the tables once.
// hsad_batch_run only enqueues kernels:
//   1. a fill kernel zeroes the queue counters (no memset nodes, so the sequence is safe
//      to capture into a HIP graph and replay);
//   2. one persistent DWT kernel for every scene: items are (scene, run of pixels), and
//      the LDS cascade body handles each scene's own L and depth;
//   3. per L' <= 8 "box" bucket, one persistent kernel popping 16 x 16 output tiles of the
//      scenes in that bucket (the body is compiled per L');
//   4. for the remaining scenes (L' > 8) the pixels are cut into chunks that fit the
//      workspace.  Per chunk, one persistent Gram kernel per tile-count class (a wavefront
//      per pixel, four pixels per item) and then one persistent Cholesky kernel (one
//      pixel per item).
// Each persistent workgroup pops item indices from its queue counter with an atomic
// add, and exits when the index passes the item count, so every wave reaches the exit.
// Items are ordered largest first, so the tail of each queue is short.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "internal.hpp"
#include "dev_box.hpp"
#include "dev_chol.hpp"
#include "dev_dwt.hpp"
#include "dev_boxg.hpp"
#include "dev_gram.hpp"

namespace hsad {

struct SceneDev {
    const float *cube;
    float *approx;
    float *lrx;
    float *dwrx;
    int H, W, L, levels, Lp, R, RI, has_inner;
    double load_rel;
    int dwt_P;         // pixels per DWT item
    int bucket;        // 0: box (fused), 1: gram + Cholesky, 2: box statistics + Cholesky
    uint32_t outer_magic;
    int pad;
};

struct Item {          // generic item: scene + two integers + workspace offset (doubles)
    int scene;
    int a;             // DWT: first pixel / box, box statistics: tile row / gram: first pixel
    int b;             // DWT: pixel count / box, box statistics: tile col / gram: pixel count
    int raw;           // chol: 1 for a box-statistics record
    int64_t ws_off;    // gram / box statistics / chol: offset of the (first) record in the chunk ws
};

static constexpr int kCounters = 16384;           // queue counters (uint32)
static constexpr int kDwtLdsDoubles = 6144;       // 48 KiB of LDS for the DWT items
static constexpr int kGramMT[5] = {1, 3, 6, 10, 16};

}  // namespace hsad

// ----------------------------------------------------------------------------------------
// plan
// ----------------------------------------------------------------------------------------
struct hsad_batch_plan {
    std::vector<hsad_scene> scenes;
    std::vector<hsad::SceneDev> sdev;
    std::vector<hsad::Item> dwt_items;
    // box buckets: L' -> items
    std::vector<std::pair<int, std::vector<hsad::Item>>> box;
    std::vector<int> box_R;                      // max outer half-width per bucket
    // gram chunks
    struct GramLaunch {
        int mt;                                  // tiles per pass (template)
        int64_t first, count;                    // range in gram_items
        int lds_doubles_per_wave;
    };
    struct Chunk {
        std::vector<GramLaunch> grams;
        int64_t boxg_first, boxg_count;          // range in boxg_items
        size_t boxg_smem;                        // LDS of the largest box-statistics tile
        int64_t chol_first, chol_count;          // range in chol_items
        int max_Lp;
    };
    std::vector<hsad::Item> boxg_items;
    int boxg_resident_kb = 0;                    // resident-staging budget the LDS sizes assume
    std::vector<hsad::Item> gram_items;
    std::vector<hsad::Item> chol_items;
    std::vector<Chunk> chunks;
    int64_t chunk_doubles = 0;
    hsad_batch_options opt;
    // workspace layout (bytes)
    size_t off_scenes = 0, off_dwt = 0, off_box = 0, off_boxg = 0, off_gram = 0, off_chol = 0, off_chunk = 0;
    size_t total = 0;
    std::vector<size_t> box_off;                 // per bucket
    bool uploaded = false;
    void *ws = nullptr;
};

namespace hsad {

// ----------------------------------------------------------------------------------------
// persistent kernels
// ----------------------------------------------------------------------------------------
__device__ inline int pop_item(unsigned *ctr, int *slot)
{
    if (threadIdx.x == 0) *slot = (int)atomicAdd(ctr, 1u);
    __syncthreads();
    const int it = *slot;
    __syncthreads();
    return it;
}

__global__ void batch_reset_kernel(unsigned *ctr, int n)
{
    for (int i = threadIdx.x; i < n; i += blockDim.x) ctr[i] = 0u;
}

__global__ __launch_bounds__(256) void batch_dwt_kernel(const SceneDev *__restrict__ sc,
                                                        const Item *__restrict__ items, int n,
                                                        unsigned *ctr, Taps taps)
{
    __shared__ double lds[kDwtLdsDoubles];
    __shared__ int slot;
    for (;;) {
        const int it = pop_item(ctr, &slot);
        if (it >= n) break;
        const Item m = items[it];
        const SceneDev &s = sc[m.scene];
        dwt_cascade_tile(s.cube, m.a, m.b, s.L, s.levels, s.Lp, taps, s.approx, lds, s.dwt_P);
        __syncthreads();
    }
}

template <int LP>
__global__ __launch_bounds__(256) void batch_box_kernel(const SceneDev *__restrict__ sc,
                                                        const Item *__restrict__ items, int n,
                                                        unsigned *ctr)
{
    extern __shared__ double smem[];
    __shared__ int slot;
    for (;;) {
        const int it = pop_item(ctr, &slot);
        if (it >= n) break;
        const Item m = items[it];
        const SceneDev &s = sc[m.scene];
        constexpr int GC = (LP >= 5 && LP <= 7) ? 8 : 5;
        box_tile<LP, GC>(s.approx, s.H, s.W, s.R, s.RI, s.has_inner, s.load_rel, s.lrx, s.dwrx, m.a,
                         m.b, smem);
        __syncthreads();
    }
}

template <int MT>
__global__ __launch_bounds__(256) void batch_gram_kernel(const SceneDev *__restrict__ sc,
                                                         const Item *__restrict__ items, int n,
                                                         unsigned *ctr, double *chunk_ws,
                                                         int wave_doubles)
{
    extern __shared__ double lds[];
    __shared__ int slot;
    const int wv = threadIdx.x >> 6;
    for (;;) {
        const int it = pop_item(ctr, &slot);
        if (it >= n) break;
        const Item m = items[it];
        const SceneDev &s = sc[m.scene];
        if (wv < m.b) {
            GramArgs a;
            a.means_ready = 0;
            a.x = s.approx;
            a.H = s.H;
            a.W = s.W;
            a.Lp = s.Lp;
            a.R = s.R;
            a.RI = s.RI;
            a.has_inner = s.has_inner;
            a.mode = GRAM_LRX;
            a.pix0 = m.a;
            a.npix = m.b;
            a.ws = chunk_ws + m.ws_off;
            a.outer_magic = s.outer_magic;
            a.idx = nullptr;
            gram_pixel<0, MT>(a, wv, lds + (size_t)wv * wave_doubles);
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void batch_boxg_kernel(const SceneDev *__restrict__ sc,
                                                         const Item *__restrict__ items, int n,
                                                         unsigned *ctr, double *chunk_ws, int resident_kb)
{
    extern __shared__ unsigned char bgs[];
    __shared__ int slot;
    for (;;) {
        const int it = pop_item(ctr, &slot);
        if (it >= n) break;
        const Item m = items[it];
        const SceneDev &s = sc[m.scene];
        boxg_tile(s.approx, s.H, s.W, s.Lp, s.R, s.RI, s.has_inner, chunk_ws + m.ws_off, -1,
                  (int64_t)(s.Lp + 3) * s.Lp, m.a, m.b, bgs, resident_kb);
        __syncthreads();
    }
}

// one wavefront per pixel item (L' <= 64), four wavefronts per workgroup; each wavefront
// takes kCholGrab consecutive items per atomic
static constexpr unsigned kCholGrab = 8;

__global__ __launch_bounds__(256) void batch_chol_wave_kernel(const SceneDev *__restrict__ sc,
                                                              const Item *__restrict__ items, int n,
                                                              unsigned *ctr, double *chunk_ws, int lds_per_wave)
{
    extern __shared__ double cw[];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    double *A = cw + (size_t)wv * lds_per_wave;
    for (;;) {
        unsigned it0 = 0;
        if (lane == 0) it0 = atomicAdd(ctr, kCholGrab);
        it0 = __shfl(it0, 0, 64);
        if (it0 >= (unsigned)n) break;
        const unsigned it1 = it0 + kCholGrab < (unsigned)n ? it0 + kCholGrab : (unsigned)n;
        for (unsigned it = it0; it < it1; ++it) {
            const Item m = items[it];
            const SceneDev &s = sc[m.scene];
            const int64_t p = m.a;
            chol_wave_pixel(chunk_ws + m.ws_off, s.Lp, m.raw, s.load_rel, s.lrx ? s.lrx + p : nullptr,
                            s.dwrx ? s.dwrx + p : nullptr, A);
            wave_sync_lds();
        }
    }
}

// G lanes per pixel item (register-resident rows, L' + 2 <= G), 256 / G items per workgroup
template <int G>
__global__ __launch_bounds__(256) void batch_chol_group_kernel(const SceneDev *__restrict__ sc,
                                                               const Item *__restrict__ items, int n,
                                                               double *chunk_ws)
{
    int it = (int)((blockIdx.x * 256 + threadIdx.x) / G);
    // G = 64: one item per wavefront; saying so lets the item and its scene be read with
    // scalar loads and keeps L' (the loop bounds) uniform
    if constexpr (G == 64) it = __builtin_amdgcn_readfirstlane(it);
    const bool active = it < n;
    const Item m = items[active ? it : 0];
    const SceneDev &s = sc[m.scene];
    const int64_t p = m.a;
    __shared__ double colbuf[256];
    chol_group_pixel<G>(chunk_ws + m.ws_off, s.Lp, m.raw, s.load_rel, active, s.lrx ? s.lrx + p : nullptr,
                        s.dwrx ? s.dwrx + p : nullptr, colbuf + (threadIdx.x & ~(G - 1)));
}

__global__ __launch_bounds__(256) void batch_chol_kernel(const SceneDev *__restrict__ sc,
                                                         const Item *__restrict__ items, int n,
                                                         unsigned *ctr, double *chunk_ws)
{
    extern __shared__ double sm[];
    __shared__ int slot;
    for (;;) {
        const int it = pop_item(ctr, &slot);
        if (it >= n) break;
        const Item m = items[it];
        const SceneDev &s = sc[m.scene];
        const int64_t p = m.a;
        chol_pixel(chunk_ws + m.ws_off, s.Lp, s.load_rel, s.lrx ? s.lrx + p : nullptr,
                   s.dwrx ? s.dwrx + p : nullptr, sm, m.raw);
    }
}

// ----------------------------------------------------------------------------------------
// host side
// ----------------------------------------------------------------------------------------
static int num_cus()
{
    static int cus = 0;
    if (!cus) {
        int dev = 0;
        hipDeviceProp_t p;
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&p, dev) == hipSuccess)
            cus = p.multiProcessorCount;
        if (cus <= 0) cus = 256;
    }
    return cus;
}

static size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

static int gram_class(int Lp)
{
    const int T = (Lp + 15) / 16, nt = T * (T + 1) / 2;
    return nt <= 1 ? 0 : nt <= 3 ? 1 : nt <= 6 ? 2 : nt <= 10 ? 3 : 4;
}

}  // namespace hsad

using namespace hsad;

extern "C" {

void hsad_batch_default_options(hsad_batch_options *o)
{
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->wgs_per_cu = 2;
    o->dwt_pixels = 0;                       // 0: as many as fit 48 KiB of LDS (max 64)
    o->chunk_bytes = (int64_t)2 << 30;
}

int hsad_batch_plan_create(const hsad_scene *scenes, int n, const hsad_batch_options *opt,
                           hsad_batch_plan **out)
{
    clear_error();
    if (!scenes || n < 1 || !out) return fail(HSAD_EINVAL, "hsad_batch_plan_create: bad arguments");
    auto *P = new hsad_batch_plan();
    if (opt) P->opt = *opt; else hsad_batch_default_options(&P->opt);
    if (P->opt.wgs_per_cu < 1 || P->opt.wgs_per_cu > 16 || P->opt.chunk_bytes < (1 << 20) ||
        P->opt.dwt_pixels < 0 || P->opt.reserved != 0) {
        delete P;
        return fail(HSAD_EINVAL, "hsad_batch_plan_create: bad options");
    }
    P->scenes.assign(scenes, scenes + n);
    int max_lp = 0;
    for (int i = 0; i < n; ++i) {
        const hsad_scene &s = scenes[i];
        const std::string who = "hsad_batch_plan_create: scene " + std::to_string(i);
        if (!s.cube || !s.approx || (!s.lrx && !s.dwrx)) {
            delete P;
            return fail(HSAD_EINVAL, who + ": NULL pointer");
        }
        if (s.H < 1 || s.W < 1 || s.L < 1 || s.L > 4096 || s.H * s.W > (int64_t)1 << 30 ||
            s.levels < 0 || s.reserved != 0) {
            delete P;
            return fail(HSAD_EINVAL, who + ": bad size or levels");
        }
        int64_t Lp = s.L;
        for (int j = 0; j < s.levels; ++j) {
            if (Lp < 2) {
                delete P;
                return fail(HSAD_EINVAL, who + ": levels too deep");
            }
            Lp = (Lp + 1) / 2;
        }
        const hsad_window_params &p = s.params;
        if ((p.outer & 1) == 0 || p.outer < 1 || p.outer > HSAD_MAX_WINDOW || p.inner < 0 ||
            (p.inner && (p.inner & 1) == 0) || p.inner >= p.outer || !(p.load_rel >= 0.0) ||
            !std::isfinite(p.load_rel) || p.reserved != 0 ||
            (p.precision != HSAD_PREC_AUTO && p.precision != HSAD_PREC_FP64) ||
            (s.dwrx && p.inner < 1) || (p.inner > 0 && s.H <= p.inner && s.W <= p.inner)) {
            delete P;
            return fail(HSAD_EINVAL, who + ": bad window parameters (batches run the exact FP64 path)");
        }
        if (Lp > 128) {
            delete P;
            return fail(HSAD_EUNSUPPORTED, who + ": L' above 128 in a batch");
        }
        SceneDev d;
        std::memset(&d, 0, sizeof(d));
        d.cube = s.cube;
        d.approx = s.approx;
        d.lrx = s.lrx;
        d.dwrx = s.dwrx;
        d.H = (int)s.H;
        d.W = (int)s.W;
        d.L = (int)s.L;
        d.levels = s.levels;
        d.Lp = (int)Lp;
        d.R = p.outer / 2;
        d.RI = p.inner / 2;
        d.has_inner = p.inner > 0;
        d.load_rel = p.load_rel;
        const int64_t per = dwt_cascade_lds_doubles(s.L, 1);
        int64_t dp = kDwtLdsDoubles / per;
        if (dp > 64) dp = 64;
        if (P->opt.dwt_pixels > 0 && P->opt.dwt_pixels < dp) dp = P->opt.dwt_pixels;
        if (dp < 1) {
            delete P;
            return fail(HSAD_EUNSUPPORTED, who + ": L too large for the batch DWT");
        }
        d.dwt_P = (int)dp;
        Windows w{p.inner, p.outer, p.inner / 2, p.outer / 2};
        d.bucket = box_supported(Lp, w) ? 0 : boxg_supported(Lp, w) ? 2 : 1;
        d.outer_magic = (uint32_t)((((uint64_t)1 << 32) + p.outer - 1) / p.outer);
        P->sdev.push_back(d);
        if (Lp > max_lp) max_lp = (int)Lp;
    }
    // scene order by decreasing cost (largest first keeps the queues' tails short)
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    auto cost = [&](int i) {
        const SceneDev &d = P->sdev[i];
        const double np = (double)d.H * d.W;
        const double win = (2.0 * d.R + 1) * (2.0 * d.R + 1);
        const double stats = d.bucket == 1 ? win * d.Lp * d.Lp / 16.0
                             : d.bucket == 2 ? 40.0 * d.Lp * (d.Lp + 1) / 2.0 + d.Lp * d.Lp * d.Lp / 6.0
                                             : 0.0;
        return np * (d.L + stats);
    };
    std::sort(order.begin(), order.end(), [&](int a, int b) { return cost(a) > cost(b); });
    for (int i : order) {
        const SceneDev &d = P->sdev[i];
        const int64_t np = (int64_t)d.H * d.W;
        for (int64_t p0 = 0; p0 < np; p0 += d.dwt_P)
            P->dwt_items.push_back(Item{i, (int)p0, (int)std::min<int64_t>(d.dwt_P, np - p0), 0, 0});
    }
    // box buckets
    for (int lp = 1; lp <= 8; ++lp) {
        std::vector<Item> items;
        int maxR = 0;
        for (int i : order) {
            const SceneDev &d = P->sdev[i];
            if (d.bucket != 0 || d.Lp != lp) continue;
            maxR = std::max(maxR, d.R);
            for (int by = 0; by < (d.H + 15) / 16; ++by)
                for (int bx = 0; bx < (d.W + 15) / 16; ++bx) items.push_back(Item{i, by, bx, 0, 0});
        }
        if (!items.empty()) {
            P->box.emplace_back(lp, std::move(items));
            P->box_R.push_back(maxR);
        }
    }
    // gram chunks
    P->boxg_resident_kb = boxg_resident_kb();
    const int64_t budget = P->opt.chunk_bytes / (int64_t)sizeof(double);
    hsad_batch_plan::Chunk cur;
    cur.boxg_first = 0;
    cur.boxg_count = 0;
    cur.boxg_smem = 0;
    cur.chol_first = 0;
    cur.chol_count = 0;
    cur.max_Lp = 0;
    int64_t used = 0;
    std::vector<std::vector<Item>> cls(5);
    auto flush = [&]() {
        if (cur.chol_count == 0) return;
        for (int c = 0; c < 5; ++c) {
            if (cls[c].empty()) continue;
            hsad_batch_plan::GramLaunch g;
            g.mt = kGramMT[c];
            g.first = (int64_t)P->gram_items.size();
            g.count = (int64_t)cls[c].size();
            int maxlp = 0;
            for (const Item &m : cls[c]) maxlp = std::max(maxlp, P->sdev[m.scene].Lp);
            g.lds_doubles_per_wave = (int)gram_wave_doubles(maxlp, 0);
            P->gram_items.insert(P->gram_items.end(), cls[c].begin(), cls[c].end());
            cur.grams.push_back(g);
            cls[c].clear();
        }
        P->chunks.push_back(cur);
        P->chunk_doubles = std::max<int64_t>(P->chunk_doubles, used);
        cur = hsad_batch_plan::Chunk();
        cur.boxg_first = (int64_t)P->boxg_items.size();
        cur.boxg_count = 0;
        cur.boxg_smem = 0;
        cur.chol_first = (int64_t)P->chol_items.size();
        cur.chol_count = 0;
        cur.max_Lp = 0;
        used = 0;
    };
    for (int i : order) {
        const SceneDev &d = P->sdev[i];
        if (d.bucket != 2) continue;
        const int64_t per = (int64_t)(d.Lp + 3) * d.Lp, tile = per * 256;
        const int nby = (d.H + 15) / 16, nbx = (d.W + 15) / 16;
        for (int by = 0; by < nby; ++by)
            for (int bx = 0; bx < nbx; ++bx) {
                if (used + tile > budget) flush();
                P->boxg_items.push_back(Item{i, by, bx, 0, used});
                ++cur.boxg_count;
                cur.boxg_smem = std::max(cur.boxg_smem, bg_smem_bytes(d.Lp, d.R, boxg_resident_kb()));
                for (int ty = 0; ty < 16; ++ty)
                    for (int tx = 0; tx < 16; ++tx) {
                        const int py = by * 16 + ty, px = bx * 16 + tx;
                        if (py >= d.H || px >= d.W) continue;
                        P->chol_items.push_back(Item{i, py * d.W + px, 1, 1, used + per * (ty * 16 + tx)});
                        ++cur.chol_count;
                    }
                cur.max_Lp = std::max(cur.max_Lp, d.Lp);
                used += tile;
            }
    }
    for (int i : order) {
        const SceneDev &d = P->sdev[i];
        if (d.bucket != 1) continue;
        const int64_t per = (int64_t)(d.Lp + 2) * d.Lp;
        const int64_t np = (int64_t)d.H * d.W;
        for (int64_t p0 = 0; p0 < np; p0 += 4) {
            const int cnt = (int)std::min<int64_t>(4, np - p0);
            if (used + per * cnt > budget) flush();
            cls[gram_class(d.Lp)].push_back(Item{i, (int)p0, cnt, 0, used});
            for (int k = 0; k < cnt; ++k) {
                P->chol_items.push_back(Item{i, (int)(p0 + k), 1, 0, used + per * k});
                ++cur.chol_count;
            }
            cur.max_Lp = std::max(cur.max_Lp, d.Lp);
            used += per * cnt;
        }
    }
    flush();
    if ((int)P->chunks.size() * 7 + (int)P->box.size() + 1 > kCounters) {
        delete P;
        return fail(HSAD_EUNSUPPORTED, "hsad_batch_plan_create: too many chunks; raise chunk_bytes");
    }
    // workspace layout
    size_t off = align_up(kCounters * sizeof(unsigned), 256);
    P->off_scenes = off;
    off = align_up(off + P->sdev.size() * sizeof(SceneDev), 256);
    P->off_dwt = off;
    off = align_up(off + P->dwt_items.size() * sizeof(Item), 256);
    for (auto &b : P->box) {
        P->box_off.push_back(off);
        off = align_up(off + b.second.size() * sizeof(Item), 256);
    }
    P->off_boxg = off;
    off = align_up(off + P->boxg_items.size() * sizeof(Item), 256);
    P->off_gram = off;
    off = align_up(off + P->gram_items.size() * sizeof(Item), 256);
    P->off_chol = off;
    off = align_up(off + P->chol_items.size() * sizeof(Item), 256);
    P->off_chunk = off;
    off = align_up(off + (size_t)P->chunk_doubles * sizeof(double), 256);
    P->total = off;
    *out = P;
    return HSAD_OK;
}

size_t hsad_batch_workspace_bytes(const hsad_batch_plan *plan) { return plan ? plan->total : 0; }

int hsad_batch_upload(hsad_batch_plan *P, void *ws, size_t ws_bytes, hipStream_t s)
{
    clear_error();
    if (!P || !ws) return fail(HSAD_EINVAL, "hsad_batch_upload: NULL argument");
    if (ws_bytes < P->total) return fail(HSAD_ENOMEM, "hsad_batch_upload: workspace too small");
    std::vector<char> host(P->off_chunk, 0);
    std::memcpy(host.data() + P->off_scenes, P->sdev.data(), P->sdev.size() * sizeof(SceneDev));
    std::memcpy(host.data() + P->off_dwt, P->dwt_items.data(), P->dwt_items.size() * sizeof(Item));
    for (size_t b = 0; b < P->box.size(); ++b)
        std::memcpy(host.data() + P->box_off[b], P->box[b].second.data(),
                    P->box[b].second.size() * sizeof(Item));
    if (!P->boxg_items.empty())
        std::memcpy(host.data() + P->off_boxg, P->boxg_items.data(), P->boxg_items.size() * sizeof(Item));
    if (!P->gram_items.empty())
        std::memcpy(host.data() + P->off_gram, P->gram_items.data(), P->gram_items.size() * sizeof(Item));
    if (!P->chol_items.empty())
        std::memcpy(host.data() + P->off_chol, P->chol_items.data(), P->chol_items.size() * sizeof(Item));
    if (hipMemcpyAsync(ws, host.data(), host.size(), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return fail(HSAD_EHIP, "hsad_batch_upload: copy failed");
    P->uploaded = true;
    P->ws = ws;
    return HSAD_OK;
}

int hsad_batch_run(const hsad_batch_plan *P, void *ws, hipStream_t s)
{
    clear_error();
    if (!P || !ws) return fail(HSAD_EINVAL, "hsad_batch_run: NULL argument");
    if (!P->uploaded || P->ws != ws)
        return fail(HSAD_EINVAL, "hsad_batch_run: workspace not uploaded with hsad_batch_upload");
    char *base = (char *)ws;
    unsigned *ctr = (unsigned *)base;
    const SceneDev *sc = (const SceneDev *)(base + P->off_scenes);
    const int grid = num_cus() * P->opt.wgs_per_cu;
    int c = 0;
    hipLaunchKernelGGL(batch_reset_kernel, dim3(1), dim3(256), 0, s, ctr, kCounters);
    Taps taps;
    for (int t = 0; t < 8; ++t) taps.h[t] = db4_filter()[t];
    hipLaunchKernelGGL(batch_dwt_kernel, dim3(grid), dim3(256), 0, s, sc,
                       (const Item *)(base + P->off_dwt), (int)P->dwt_items.size(), ctr + c++, taps);
    if (int rc = check_launch("batch_dwt_kernel")) return rc;
    for (size_t b = 0; b < P->box.size(); ++b) {
        const int lp = P->box[b].first, R = P->box_R[b];
        const Item *it = (const Item *)(base + P->box_off[b]);
        const int n = (int)P->box[b].second.size();
        size_t sh = 0;
        const void *fn = nullptr;
        switch (lp) {
#define HSAD_BB(L_)                                                                            \
    case L_:                                                                                   \
        sh = box_smem<L_, ((L_) >= 5 && (L_) <= 7) ? 8 : 5>(R);                                 \
        fn = (const void *)batch_box_kernel<L_>;                                               \
        break;
            HSAD_BB(1) HSAD_BB(2) HSAD_BB(3) HSAD_BB(4) HSAD_BB(5) HSAD_BB(6) HSAD_BB(7) HSAD_BB(8)
#undef HSAD_BB
        default: return fail(HSAD_EUNSUPPORTED, "hsad_batch_run: box bucket");
        }
        if (int rc = allow_lds(fn, sh, "batch_box_kernel")) return rc;
        switch (lp) {
#define HSAD_BL(L_)                                                                            \
    case L_:                                                                                   \
        hipLaunchKernelGGL(batch_box_kernel<L_>, dim3(grid), dim3(256), sh, s, sc, it, n, ctr + c); \
        break;
            HSAD_BL(1) HSAD_BL(2) HSAD_BL(3) HSAD_BL(4) HSAD_BL(5) HSAD_BL(6) HSAD_BL(7) HSAD_BL(8)
#undef HSAD_BL
        }
        ++c;
        if (int rc = check_launch("batch_box_kernel")) return rc;
    }
    double *chunk_ws = (double *)(base + P->off_chunk);
    const Item *bgi = (const Item *)(base + P->off_boxg);
    const Item *gi = (const Item *)(base + P->off_gram);
    const Item *ci = (const Item *)(base + P->off_chol);
    for (const auto &ch : P->chunks) {
        if (ch.boxg_count > 0) {
            if (int rc = allow_lds((const void *)batch_boxg_kernel, ch.boxg_smem, "batch_boxg_kernel")) return rc;
            int g2 = (int)std::min<int64_t>(grid, ch.boxg_count);
            hipLaunchKernelGGL(batch_boxg_kernel, dim3(g2), dim3(256), ch.boxg_smem, s, sc, bgi + ch.boxg_first,
                               (int)ch.boxg_count, ctr + c, chunk_ws, P->boxg_resident_kb);
            ++c;
            if (int rc = check_launch("batch_boxg_kernel")) return rc;
        }
        for (const auto &g : ch.grams) {
            const size_t sh = (size_t)g.lds_doubles_per_wave * 4 * sizeof(double);
            const int n = (int)g.count;
            const Item *it = gi + g.first;
#define HSAD_GL(M_)                                                                              \
    do {                                                                                         \
        if (int rc = allow_lds((const void *)batch_gram_kernel<M_>, sh, "batch_gram_kernel")) return rc; \
        hipLaunchKernelGGL(batch_gram_kernel<M_>, dim3(grid), dim3(256), sh, s, sc, it, n, ctr + c, \
                           chunk_ws, g.lds_doubles_per_wave);                                    \
    } while (0)
            switch (g.mt) {
            case 1: HSAD_GL(1); break;
            case 3: HSAD_GL(3); break;
            case 6: HSAD_GL(6); break;
            case 10: HSAD_GL(10); break;
            default: HSAD_GL(16); break;
            }
#undef HSAD_GL
            ++c;
            if (int rc = check_launch("batch_gram_kernel")) return rc;
        }
        if (ch.max_Lp + 2 <= 64) {
            const int G = ch.max_Lp + 2 <= 16 ? 16 : ch.max_Lp + 2 <= 32 ? 32 : 64;
            const int n = (int)ch.chol_count;
            dim3 g2((unsigned)(((int64_t)n * G + 255) / 256));
            if (G == 16)
                hipLaunchKernelGGL(batch_chol_group_kernel<16>, g2, dim3(256), 0, s, sc, ci + ch.chol_first, n, chunk_ws);
            else if (G == 32)
                hipLaunchKernelGGL(batch_chol_group_kernel<32>, g2, dim3(256), 0, s, sc, ci + ch.chol_first, n, chunk_ws);
            else
                hipLaunchKernelGGL(batch_chol_group_kernel<64>, g2, dim3(256), 0, s, sc, ci + ch.chol_first, n, chunk_ws);
            if (int rc = check_launch("batch_chol_group_kernel")) return rc;
        } else if (ch.max_Lp <= 64) {
            const int per_wave = (int)chol_wave_lds_doubles(ch.max_Lp);
            const size_t sh = (size_t)4 * per_wave * sizeof(double);
            if (int rc = allow_lds((const void *)batch_chol_wave_kernel, sh, "batch_chol_wave_kernel")) return rc;
            hipLaunchKernelGGL(batch_chol_wave_kernel, dim3(grid * 2), dim3(256), sh, s, sc, ci + ch.chol_first,
                               (int)ch.chol_count, ctr + c, chunk_ws, per_wave);
            ++c;
            if (int rc = check_launch("batch_chol_wave_kernel")) return rc;
        } else {
            const size_t sh = chol_smem_doubles(ch.max_Lp) * sizeof(double);
            const int nt = ch.max_Lp <= 32 ? 64 : 256;
            if (int rc = allow_lds((const void *)batch_chol_kernel, sh, "batch_chol_kernel")) return rc;
            hipLaunchKernelGGL(batch_chol_kernel, dim3(grid * (nt == 64 ? 4 : 1)), dim3(nt), sh, s, sc,
                               ci + ch.chol_first, (int)ch.chol_count, ctr + c, chunk_ws);
            ++c;
            if (int rc = check_launch("batch_chol_kernel")) return rc;
        }
    }
    return HSAD_OK;
}

int hsad_batch_plan_destroy(hsad_batch_plan *plan)
{
    delete plan;
    return HSAD_OK;
}

int hsad_batch_plan_info(const hsad_batch_plan *P, int64_t *info, int n)
{
    if (!P || !info || n < 8) return fail(HSAD_EINVAL, "hsad_batch_plan_info: bad arguments");
    int64_t npix = 0, box_px = 0, gram_px = 0;
    for (const auto &d : P->sdev) {
        const int64_t np = (int64_t)d.H * d.W;
        npix += np;
        (d.bucket != 0 ? gram_px : box_px) += np;
    }
    int64_t box_items = 0;
    for (const auto &b : P->box) box_items += (int64_t)b.second.size();
    info[0] = (int64_t)P->sdev.size();
    info[1] = npix;
    info[2] = (int64_t)P->dwt_items.size();
    info[3] = box_items;
    info[4] = (int64_t)P->gram_items.size();
    info[5] = (int64_t)P->chunks.size();
    info[6] = box_px;
    info[7] = gram_px;
    return HSAD_OK;
}

}  // extern "C"

// ----------------------------------------------------------------------------------------
// autotuner: times candidate schedules with HIP events and caches the winner in a JSON
// file keyed by device and batch signature
// ----------------------------------------------------------------------------------------
#include <cstdio>
#include <fstream>
#include <mutex>
#include <sstream>

namespace hsad {

static std::mutex g_tune_mu;

static std::string batch_signature(const hsad_scene *sc, int n)
{
    uint64_t h = 1469598103934665603ull;   // FNV-1a over the shape and window parameters
    auto mix = [&](int64_t v) {
        for (int b = 0; b < 8; ++b) {
            h ^= (uint64_t)((v >> (8 * b)) & 0xff);
            h *= 1099511628211ull;
        }
    };
    for (int i = 0; i < n; ++i) {
        mix(sc[i].H);
        mix(sc[i].W);
        mix(sc[i].L);
        mix(sc[i].levels);
        mix(sc[i].params.inner);
        mix(sc[i].params.outer);
    }
    int dev = 0;
    hipDeviceProp_t p;
    std::string arch = "unknown";
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&p, dev) == hipSuccess)
        arch = p.gcnArchName;
    char buf[64];
    std::snprintf(buf, sizeof buf, "%016llx", (unsigned long long)h);
    // the library build (a hash of its sources): schedules tuned for other kernels are not reused
#ifndef HSAD_BUILD_ID
#define HSAD_BUILD_ID "unknown"
#endif
    return arch.substr(0, arch.find(':')) + "/" + HSAD_BUILD_ID + "/" + std::to_string(n) + "/" + buf;
}

static bool cache_lookup(const char *path, const std::string &key, hsad_batch_options *o)
{
    if (!path) return false;
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        // one entry per line: "key": [wgs_per_cu, dwt_pixels, chunk_bytes, ms],
        const auto q = line.find('"' + key + '"');
        if (q == std::string::npos) continue;
        long long a, b, c;
        double ms;
        const auto br = line.find('[', q);
        if (br == std::string::npos) continue;
        if (std::sscanf(line.c_str() + br, "[%lld, %lld, %lld, %lf]", &a, &b, &c, &ms) == 4) {
            hsad_batch_default_options(o);
            o->wgs_per_cu = (int)a;
            o->dwt_pixels = (int)b;
            o->chunk_bytes = c;
            return true;
        }
    }
    return false;
}

static void cache_store(const char *path, const std::string &key, const hsad_batch_options &o, double ms)
{
    if (!path) return;
    std::vector<std::string> lines;
    {
        std::ifstream f(path);
        std::string line;
        while (std::getline(f, line))
            if (line.find("\": [") != std::string::npos && line.find('"' + key + '"') == std::string::npos)
                lines.push_back(line);
    }
    char buf[256];
    std::snprintf(buf, sizeof buf, "  \"%s\": [%d, %d, %lld, %.4f]", key.c_str(), o.wgs_per_cu,
                  o.dwt_pixels, (long long)o.chunk_bytes, ms);
    lines.push_back(buf);
    std::ofstream f(path, std::ios::trunc);
    f << "{\n";
    for (size_t i = 0; i < lines.size(); ++i) {
        std::string l = lines[i];
        while (!l.empty() && (l.back() == ',' || l.back() == ' ')) l.pop_back();
        f << l << (i + 1 < lines.size() ? ",\n" : "\n");
    }
    f << "}\n";
}

}  // namespace hsad

extern "C" int hsad_batch_autotune(const hsad_scene *scenes, int n, void *ws, size_t ws_bytes,
                                   hipStream_t s, const char *cache_path, hsad_batch_options *best,
                                   double *best_ms)
{
    using namespace hsad;
    clear_error();
    if (!scenes || n < 1 || !ws || !best) return fail(HSAD_EINVAL, "hsad_batch_autotune: bad arguments");
    std::lock_guard<std::mutex> lk(g_tune_mu);
    const std::string key = batch_signature(scenes, n);
    hsad_batch_options cached;
    if (cache_lookup(cache_path, key, &cached)) {
        // a cached schedule is used only if its plan fits the caller's workspace
        hsad_batch_plan *P = nullptr;
        const bool fits = hsad_batch_plan_create(scenes, n, &cached, &P) == HSAD_OK && P->total <= ws_bytes;
        if (P) hsad_batch_plan_destroy(P);
        clear_error();
        if (fits) {
            *best = cached;
            if (best_ms) *best_ms = -1.0;
            return HSAD_OK;
        }
    }
    const int wgs[] = {1, 2, 4};
    const int dps[] = {0, 8};
    const int64_t chunks[] = {(int64_t)1 << 30, (int64_t)4 << 30};
    double bms = 1e300;
    bool any = false;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(HSAD_EHIP, "hsad_batch_autotune: event creation failed");
    for (int w : wgs)
        for (int dp : dps)
            for (int64_t cb : chunks) {
                hsad_batch_options o;
                hsad_batch_default_options(&o);
                o.wgs_per_cu = w;
                o.dwt_pixels = dp;
                o.chunk_bytes = cb;
                hsad_batch_plan *P = nullptr;
                if (hsad_batch_plan_create(scenes, n, &o, &P) != HSAD_OK) continue;
                if (P->total > ws_bytes || hsad_batch_upload(P, ws, ws_bytes, s) != HSAD_OK) {
                    hsad_batch_plan_destroy(P);
                    continue;
                }
                float ms = 0.f;
                bool ok = hsad_batch_run(P, ws, s) == HSAD_OK;        // warm-up
                ok = ok && hipEventRecord(e0, s) == hipSuccess;
                ok = ok && hsad_batch_run(P, ws, s) == HSAD_OK;
                ok = ok && hipEventRecord(e1, s) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
                     hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
                hsad_batch_plan_destroy(P);
                if (!ok) {
                    (void)hipEventDestroy(e0);
                    (void)hipEventDestroy(e1);
                    return fail(HSAD_EHIP, "hsad_batch_autotune: candidate run failed");
                }
                if (ms < bms) {
                    bms = ms;
                    *best = o;
                    any = true;
                }
            }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (!any) return fail(HSAD_ENOMEM, "hsad_batch_autotune: no candidate fits the workspace");
    cache_store(cache_path, key, *best, bms);
    if (best_ms) *best_ms = bms;
    return HSAD_OK;
}
