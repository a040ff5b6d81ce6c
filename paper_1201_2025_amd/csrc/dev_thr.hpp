// dev_thr.hpp -- device body of the eq. (12) merge (Sec. 5.3.2): the threshold statistics of
// a score map from per-block (count, mean, M2) partials, shared by the merge-and-mask kernel
// and the threshold role of the pipelined detection launch.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>

namespace hsad {

// threads that take part in the merge tree, and partials per thread
constexpr int kThrMergeThreads = 256, kThrMergePer = 4;

// Chan et al.'s pairwise update of (count, mean, M2).
__device__ __forceinline__ void chan_merge(double &na, double &ma, double &Ma, double nb, double mb,
                                           double Mb)
{
    const double nn = na + nb;
    if (nb == 0.0) return;
    if (na == 0.0) {
        na = nb;
        ma = mb;
        Ma = Mb;
        return;
    }
    const double d = mb - ma;
    ma += d * (nb / nn);
    Ma += Mb + d * d * (na * nb / nn);
    na = nn;
}

// The partials thread t merges first: t, t + 256, t + 512, t + 768 (clamped loads; only
// those below nblk are merged).  Threads t >= 256 load nothing.
struct ThrParts {
    double n[kThrMergePer], m[kThrMergePer], M[kThrMergePer];
};

__device__ __forceinline__ void thr_load_parts(const double *__restrict__ part, int nblk, int t, ThrParts &p)
{
#pragma unroll
    for (int k = 0; k < kThrMergePer; ++k) {
        const int i = t + k * kThrMergeThreads, ic = i < nblk ? i : nblk - 1;
        p.n[k] = t < kThrMergeThreads ? part[3 * ic] : 0.0;
        p.m[k] = t < kThrMergeThreads ? part[3 * ic + 1] : 0.0;
        p.M[k] = t < kThrMergeThreads ? part[3 * ic + 2] : 0.0;
    }
}

// Merges nblk <= 1024 partials in a fixed order (thread t merges its four, then a pairwise
// tree, t with t + w for w = 128 ... 1, the last six levels inside wavefront 0), so every
// workgroup that runs it gets the same bits.  Every thread of the workgroup must call it
// (barriers); threads 0..255 take part.  sh: 3 * 256 doubles of LDS, tau_s: one double of
// LDS.  Writes stats = {count, mu, sigma, tau} when stats is not null; returns tau.
__device__ inline double thr_merge_tau(const ThrParts &p, int nblk, double z, double *sh, double *tau_s,
                                       double *__restrict__ stats)
{
    const int t = threadIdx.x;
    double na = 0.0, ma = 0.0, Ma = 0.0;
    if (t < kThrMergeThreads) {
#pragma unroll
        for (int k = 0; k < kThrMergePer; ++k)
            if (t + k * kThrMergeThreads < nblk) chan_merge(na, ma, Ma, p.n[k], p.m[k], p.M[k]);
        sh[3 * t] = na;
        sh[3 * t + 1] = ma;
        sh[3 * t + 2] = Ma;
    }
    __syncthreads();
    for (int w = kThrMergeThreads / 2; w >= 64; w >>= 1) {
        if (t < w) {
            chan_merge(na, ma, Ma, sh[3 * (t + w)], sh[3 * (t + w) + 1], sh[3 * (t + w) + 2]);
            sh[3 * t] = na;
            sh[3 * t + 1] = ma;
            sh[3 * t + 2] = Ma;
        }
        __syncthreads();
    }
    if (t < 64) {
        for (int w = 32; w > 0; w >>= 1) {
            const double nb = __shfl_down(na, w, 64), mb = __shfl_down(ma, w, 64), Mb = __shfl_down(Ma, w, 64);
            if (t < w) chan_merge(na, ma, Ma, nb, mb, Mb);
        }
        if (t == 0) {
            const double cnt = na, mu = cnt > 0 ? ma : NAN;
            const double sig = cnt > 0 ? sqrt(Ma / cnt) : NAN;
            *tau_s = mu + z * sig;
            if (stats) {
                stats[0] = cnt;
                stats[1] = mu;
                stats[2] = sig;
                stats[3] = *tau_s;
            }
        }
    }
    __syncthreads();
    return *tau_s;
}

}  // namespace hsad
