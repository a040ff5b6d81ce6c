// eval.hip -- post-processing of an anomaly map: the adaptive threshold of eq. (12) with
// its mask (Sec. 5.3.2), and the exact ROC AUC counts (Sec. 5.3.1).
//
// Threshold: tau = mu_d + Z sigma_d over the finite scores, with the population standard
// deviation from two passes (mean, then centred squares).  The reductions are FP64 with
// a fixed block count, so results are deterministic.  mask = (s > tau).
// AUC: the Mann-Whitney counts over pixel pairs (positive p, negative q):
// greater = #{s_p > s_q}, equal = #{s_p == s_q}.  Positive scores are compacted into the
// workspace, then each negative pixel is compared with all of them through LDS tiles.
// The counts are exact 64-bit integers; AUC = (greater + equal/2) / (npos * nneg).
#include <hip/hip_runtime.h>

#include <cmath>

#include "internal.hpp"

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

// mode 0: (count, sum) of finite scores; mode 1: sum of (s - mu)^2 with mu = stats[1]
__global__ __launch_bounds__(kRedThreads) void thr_partial_kernel(const float *__restrict__ s,
                                                                  int64_t n, int mode,
                                                                  const double *__restrict__ stats,
                                                                  double *__restrict__ part)
{
    __shared__ double red[8];
    const double mu = mode ? stats[1] : 0.0;
    double a = 0.0, b = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const float v = s[i];
        if (isfinite(v)) {
            if (mode == 0) {
                a += 1.0;
                b += (double)v;
            } else {
                const double d = (double)v - mu;
                b += d * d;
            }
        }
    }
    a = block_reduce_sum(a, red);
    b = block_reduce_sum(b, red);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = a;
        part[2 * blockIdx.x + 1] = b;
    }
}

// stats = {count, mu, sigma, tau}
__global__ __launch_bounds__(kRedThreads) void thr_final_kernel(const double *__restrict__ part,
                                                                int nblk, int mode, double z,
                                                                double *__restrict__ stats)
{
    __shared__ double red[8];
    double a = 0.0, b = 0.0;
    for (int i = threadIdx.x; i < nblk; i += blockDim.x) {
        a += part[2 * i];
        b += part[2 * i + 1];
    }
    a = block_reduce_sum(a, red);
    b = block_reduce_sum(b, red);
    if (threadIdx.x == 0) {
        if (mode == 0) {
            stats[0] = a;
            stats[1] = a > 0 ? b / a : NAN;
        } else {
            const double sig = stats[0] > 0 ? sqrt(b / stats[0]) : NAN;
            stats[2] = sig;
            stats[3] = stats[1] + z * sig;
        }
    }
}

__global__ __launch_bounds__(kRedThreads) void thr_mask_kernel(const float *__restrict__ s,
                                                               int64_t n,
                                                               const double *__restrict__ stats,
                                                               uint8_t *__restrict__ mask)
{
    const double tau = stats[3];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        mask[i] = ((double)s[i] > tau) ? 1 : 0;
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

}  // namespace hsad

using namespace hsad;

extern "C" {

size_t hsad_threshold_workspace_bytes(int64_t n)
{
    (void)n;
    return (size_t)kRedBlocks * 2 * sizeof(double);
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
    int nblk = (int)((n + kRedThreads - 1) / kRedThreads);
    if (nblk > kRedBlocks) nblk = kRedBlocks;
    hipLaunchKernelGGL(thr_partial_kernel, dim3(nblk), dim3(kRedThreads), 0, stream, scores, n, 0,
                       stats, part);
    hipLaunchKernelGGL(thr_final_kernel, dim3(1), dim3(kRedThreads), 0, stream, part, nblk, 0,
                       z_alpha, stats);
    hipLaunchKernelGGL(thr_partial_kernel, dim3(nblk), dim3(kRedThreads), 0, stream, scores, n, 1,
                       stats, part);
    hipLaunchKernelGGL(thr_final_kernel, dim3(1), dim3(kRedThreads), 0, stream, part, nblk, 1,
                       z_alpha, stats);
    if (mask)
        hipLaunchKernelGGL(thr_mask_kernel, dim3(nblk), dim3(kRedThreads), 0, stream, scores, n,
                           stats, mask);
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
