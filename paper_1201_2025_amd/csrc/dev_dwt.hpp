// dev_dwt.hpp -- device body of the LDS cascade DWT (Sec. 3 eqs. 8-9, Fig. 1), shared by the
// per-cube kernel and the persistent batch kernel.
#pragma once
#include <hip/hip_runtime.h>

namespace hsad {

struct Taps {
    double h[8];
};

// LDS doubles needed for a tile of P spectra of length L.
__host__ __device__ inline int64_t dwt_cascade_lds_doubles(int64_t L, int64_t P)
{
    return P * ((L + 1) + ((L + 1) / 2 + 1));
}

// J levels of the periodised low-pass on np (<= P) contiguous spectra starting at pixel p0;
// a workgroup of 256 threads; lds holds dwt_cascade_lds_doubles(L, P) doubles.  The
// levels run in FP64 with ping-pong buffers and one barrier per level.
__device__ inline void dwt_cascade_tile(const float *__restrict__ cube, int64_t p0, int np, int L,
                                        int levels, int Lp, const Taps &taps,
                                        float *__restrict__ out, double *lds, int P)
{
    const int S0 = L + 1;                 // odd stride of the level-0 buffer
    const int S1 = (L + 1) / 2 + 1;       // stride of the level-1 buffer
    double *buf0 = lds;                   // P * S0
    double *buf1 = lds + (size_t)P * S0;  // P * S1
    const int tid = threadIdx.x;

    // coalesced load of np contiguous spectra
    const float *src = cube + p0 * (int64_t)L;
    const int total = np * L;
    for (int t = tid; t < total; t += 256) {
        const int p = t / L, i = t - p * L;
        buf0[p * S0 + i] = (double)src[t];
    }
    __syncthreads();

    double *cur = buf0, *nxt = buf1;
    int scur = S0, snxt = S1;
    int n = L;
    for (int j = 0; j < levels; ++j) {
        const int ne = n + (n & 1), m = ne / 2;
        // lanes over k (64 per pixel row), 4 pixel rows per pass of 256 threads
        for (int p = tid >> 6; p < np; p += 4) {
            const double *x = cur + p * scur;
            for (int k = tid & 63; k < m; k += 64) {
                double s = 0.0;
#pragma unroll
                for (int t = 0; t < 8; ++t) {
                    int i = 2 * k - t;       // >= -7; short levels (ne < 8) wrap twice
                    while (i < 0) i += ne;
                    s = fma(taps.h[t], x[i < n ? i : n - 1], s);
                }
                nxt[p * snxt + k] = s;
            }
        }
        __syncthreads();
        double *tp = cur; cur = nxt; nxt = tp;
        int ts = scur; scur = snxt; snxt = ts;
        n = m;
    }
    // coalesced store of np * Lp outputs
    float *dst = out + p0 * (int64_t)Lp;
    for (int t = tid; t < np * Lp; t += 256) {
        const int p = t / Lp, k = t - p * Lp;
        dst[t] = (float)cur[p * scur + k];
    }
}

}  // namespace hsad
