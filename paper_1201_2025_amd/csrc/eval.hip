// eval.hip -- post-processing of an anomaly map: the adaptive threshold of eq. (12) with
// its mask (Sec. 5.3.2), and the exact ROC AUC counts (Sec. 5.3.1).
//
// Threshold: tau = mu_d + Z sigma_d over the finite scores, with the population standard
// deviation.  Each block takes two passes over its chunk (mean, then centred squares).
// The block results are combined with Chan's pairwise update of (count, mean, M2) in a
// fixed tree.  Everything is FP64 and deterministic.  Two launches: block statistics,
// then merge + mask (s > tau).
// AUC: the Mann-Whitney counts over pixel pairs (positive p, negative q):
// greater = #{s_p > s_q}, equal = #{s_p == s_q}.  Positive scores are compacted into the
// workspace, then each negative pixel is compared with all of them through LDS tiles.
// The counts are exact 64-bit integers; AUC = (greater + equal/2) / (npos * nneg).
#include <hip/hip_runtime.h>

#include <cmath>

#include "internal.hpp"
#include "dev_thr.hpp"

namespace hsad {

static constexpr int kRedBlocks = 1024;
static constexpr int kRedThreads = 256;

__device__ __forceinline__ double block_reduce_sum(double v, double *red)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) red[wv] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += red[i];
    __syncthreads();
    return s;   // valid in thread 0
}

// Per-block statistics of the finite scores: count, mean (two passes over the block's
// chunk, so the centred sum of squares M2 is exact up to rounding) -> part[3*b .. 3*b+2].
__global__ __launch_bounds__(kRedThreads) void thr_block_kernel(const float *__restrict__ s,
                                                                int64_t n, int64_t chunk,
                                                                double *__restrict__ part)
{
    __shared__ double red[8];
    __shared__ double bmean;
    const int64_t b0 = (int64_t)blockIdx.x * chunk;
    const int64_t b1 = b0 + chunk < n ? b0 + chunk : n;
    double c = 0.0, sum = 0.0;
    for (int64_t i = b0 + threadIdx.x; i < b1; i += blockDim.x) {
        const float v = s[i];
        if (isfinite(v)) {
            c += 1.0;
            sum += (double)v;
        }
    }
    c = block_reduce_sum(c, red);
    sum = block_reduce_sum(sum, red);
    if (threadIdx.x == 0) bmean = c > 0 ? sum / c : 0.0;
    __syncthreads();
    const double m = bmean;
    double m2 = 0.0;
    for (int64_t i = b0 + threadIdx.x; i < b1; i += blockDim.x) {
        const float v = s[i];
        if (isfinite(v)) {
            const double d = (double)v - m;
            m2 += d * d;
        }
    }
    m2 = block_reduce_sum(m2, red);
    if (threadIdx.x == 0) {
        part[3 * blockIdx.x] = c;
        part[3 * blockIdx.x + 1] = m;
        part[3 * blockIdx.x + 2] = m2;
    }
}

// Every block merges the per-block statistics with the same fixed tree (so they agree
// bit for bit), block 0 stores stats = {count, mu, sigma, tau}, and all blocks write
// the mask (s > tau) for their part of the map.
__global__ __launch_bounds__(kRedThreads) void thr_merge_mask_kernel(const float *__restrict__ s,
                                                                     int64_t n, int nblk,
                                                                     const double *__restrict__ part,
                                                                     double z,
                                                                     double *__restrict__ stats,
                                                                     uint8_t *__restrict__ mask)
{
    __shared__ double sh[3 * kRedThreads];
    __shared__ double tau_s;
    static_assert(kRedThreads == kThrMergeThreads, "one merge tree");
    // The thread's first kPF scores and its (at most four) partials are loaded up front,
    // from clamped indices, so all these round trips overlap each other and the merge.
    constexpr int kPF = 4;
    const int t = threadIdx.x;
    const int64_t i0 = (int64_t)blockIdx.x * kRedThreads + t, st = (int64_t)gridDim.x * kRedThreads;
    float sv[kPF];
#pragma unroll
    for (int k = 0; k < kPF; ++k) {
        const int64_t i = i0 + k * st;
        sv[k] = s[i < n ? i : n - 1];
    }
    ThrParts pp;
    thr_load_parts(part, nblk, t, pp);
    // block 0 stores stats = {count, mu, sigma, tau}
    const double tau = thr_merge_tau(pp, nblk, z, sh, &tau_s, blockIdx.x == 0 ? stats : nullptr);
    if (!mask) return;
#pragma unroll
    for (int k = 0; k < kPF; ++k) {
        const int64_t i = i0 + k * st;
        if (i < n) mask[i] = ((double)sv[k] > tau) ? 1 : 0;
    }
    for (int64_t i = i0 + kPF * st; i < n; i += st) mask[i] = ((double)s[i] > tau) ? 1 : 0;
}

// ---- AUC ----
__global__ void auc_clear_kernel(unsigned long long *counts, unsigned long long *npos_ctr)
{
    if (threadIdx.x < 4) counts[threadIdx.x] = 0ull;
    if (threadIdx.x == 0) *npos_ctr = 0ull;
}

__global__ __launch_bounds__(256) void auc_compact_kernel(const float *__restrict__ s,
                                                          const uint8_t *__restrict__ truth,
                                                          int64_t n,
                                                          unsigned long long *__restrict__ npos_ctr,
                                                          float *__restrict__ pos)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        if (truth[i]) {
            const unsigned long long k = atomicAdd(npos_ctr, 1ull);
            pos[k] = s[i];
        }
    }
}

static constexpr int kAucTile = 4096;

__global__ __launch_bounds__(256) void auc_count_kernel(const float *__restrict__ s,
                                                        const uint8_t *__restrict__ truth,
                                                        int64_t n,
                                                        const unsigned long long *__restrict__ npos_ctr,
                                                        const float *__restrict__ pos,
                                                        unsigned long long *__restrict__ counts)
{
    __shared__ float tile[kAucTile];
    __shared__ unsigned long long red[8];
    const int64_t npos = (int64_t)*npos_ctr;
    unsigned long long gt = 0, eq = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t first = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    // every thread of the block walks the same tiles; pixels are grid-strided
    const int64_t nloops = (n + stride - 1) / stride;
    for (int64_t t0 = 0; t0 < npos; t0 += kAucTile) {
        const int nt = (int)((npos - t0) < kAucTile ? (npos - t0) : kAucTile);
        __syncthreads();
        for (int k = threadIdx.x; k < nt; k += blockDim.x) tile[k] = pos[t0 + k];
        __syncthreads();
        for (int64_t it = 0; it < nloops; ++it) {
            const int64_t i = first + it * stride;
            if (i >= n || truth[i]) continue;
            const float v = s[i];
            unsigned int g = 0, e = 0;
            for (int k = 0; k < nt; ++k) {
                const float p = tile[k];
                g += (p > v) ? 1u : 0u;
                e += (p == v) ? 1u : 0u;
            }
            gt += g;
            eq += e;
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        gt += __shfl_xor(gt, o);
        eq += __shfl_xor(eq, o);
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) {
        red[wv] = gt;
        red[4 + wv] = eq;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long a = 0, b = 0;
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) {
            a += red[i];
            b += red[4 + i];
        }
        atomicAdd(&counts[0], a);
        atomicAdd(&counts[1], b);
    }
}

__global__ void auc_finish_kernel(int64_t n, const unsigned long long *npos_ctr,
                                  unsigned long long *counts)
{
    if (threadIdx.x == 0) {
        counts[2] = *npos_ctr;
        counts[3] = (unsigned long long)n - *npos_ctr;
    }
}

// Merges consecutive runs of partials, in order, down to at most kRedBlocks partials (one
// thread per output partial).
__global__ __launch_bounds__(256) void thr_fold_kernel(const double *__restrict__ part, int64_t nblk,
                                                       int64_t run, int nout, double *__restrict__ out)
{
    const int o = blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= nout) return;
    double na = 0.0, ma = 0.0, Ma = 0.0;
    const int64_t b0 = (int64_t)o * run, b1 = b0 + run < nblk ? b0 + run : nblk;
    for (int64_t b = b0; b < b1; ++b) chan_merge(na, ma, Ma, part[3 * b], part[3 * b + 1], part[3 * b + 2]);
    out[3 * o] = na;
    out[3 * o + 1] = ma;
    out[3 * o + 2] = Ma;
}

size_t threshold_fold_doubles() { return (size_t)kRedBlocks * 3; }

int threshold_from_partials(const float *scores, int64_t n, const double *part, int64_t nblk, double z,
                            double *stats, uint8_t *mask, double *fold, hipStream_t s)
{
    if (nblk > kRedBlocks) {
        const int64_t run = (nblk + kRedBlocks - 1) / kRedBlocks;
        const int nout = (int)((nblk + run - 1) / run);
        hipLaunchKernelGGL(thr_fold_kernel, dim3((unsigned)((nout + 255) / 256)), dim3(256), 0, s, part, nblk,
                           run, nout, fold);
        part = fold;
        nblk = nout;
    }
    int64_t mblk = (n + kRedThreads * 4 - 1) / (kRedThreads * 4);
    if (mblk > kRedBlocks) mblk = kRedBlocks;
    hipLaunchKernelGGL(thr_merge_mask_kernel, dim3((unsigned)mblk), dim3(kRedThreads), 0, s, scores, n,
                       (int)nblk, part, z, stats, mask);
    return check_launch("thr_merge_mask_kernel");
}

}  // namespace hsad

using namespace hsad;

extern "C" {

size_t hsad_threshold_workspace_bytes(int64_t n)
{
    (void)n;
    return (size_t)kRedBlocks * 3 * sizeof(double);
}

int hsad_threshold(const float *scores, int64_t n, double z_alpha, double *stats, uint8_t *mask,
                   void *ws, size_t ws_bytes, hipStream_t stream)
{
    clear_error();
    if (!scores || !stats || n < 1) return fail(HSAD_EINVAL, "hsad_threshold: bad arguments");
    if (!std::isfinite(z_alpha)) return fail(HSAD_EINVAL, "hsad_threshold: z_alpha not finite");
    if (!ws || ws_bytes < hsad_threshold_workspace_bytes(n))
        return fail(HSAD_ENOMEM, "hsad_threshold: workspace too small");
    double *part = (double *)ws;
    // ~1024 scores per block, at most kRedBlocks blocks
    int64_t nblk = (n + 1023) / 1024;
    if (nblk > kRedBlocks) nblk = kRedBlocks;
    const int64_t chunk = (n + nblk - 1) / nblk;
    hipLaunchKernelGGL(thr_block_kernel, dim3((unsigned)nblk), dim3(kRedThreads), 0, stream, scores, n,
                       chunk, part);
    int64_t mblk = (n + kRedThreads * 4 - 1) / (kRedThreads * 4);
    if (mblk > kRedBlocks) mblk = kRedBlocks;
    hipLaunchKernelGGL(thr_merge_mask_kernel, dim3((unsigned)mblk), dim3(kRedThreads), 0, stream, scores,
                       n, (int)nblk, part, z_alpha, stats, mask);
    return check_launch("hsad_threshold");
}

size_t hsad_auc_workspace_bytes(int64_t n)
{
    return 256 + (size_t)(n > 0 ? n : 0) * sizeof(float);
}

int hsad_auc(const float *scores, const uint8_t *truth, int64_t n, uint64_t *counts, void *ws,
             size_t ws_bytes, hipStream_t stream)
{
    clear_error();
    if (!scores || !truth || !counts || n < 1) return fail(HSAD_EINVAL, "hsad_auc: bad arguments");
    if (!ws || ws_bytes < hsad_auc_workspace_bytes(n))
        return fail(HSAD_ENOMEM, "hsad_auc: workspace too small");
    unsigned long long *ctr = (unsigned long long *)ws;
    float *pos = (float *)((char *)ws + 256);
    unsigned long long *cnt = (unsigned long long *)counts;
    int nblk = (int)((n + 255) / 256);
    if (nblk > 2048) nblk = 2048;
    hipLaunchKernelGGL(auc_clear_kernel, dim3(1), dim3(64), 0, stream, cnt, ctr);
    hipLaunchKernelGGL(auc_compact_kernel, dim3(nblk), dim3(256), 0, stream, scores, truth, n, ctr, pos);
    hipLaunchKernelGGL(auc_count_kernel, dim3(nblk), dim3(256), 0, stream, scores, truth, n, ctr, pos, cnt);
    hipLaunchKernelGGL(auc_finish_kernel, dim3(1), dim3(64), 0, stream, n, ctr, cnt);
    return check_launch("hsad_auc");
}

}  // extern "C"
