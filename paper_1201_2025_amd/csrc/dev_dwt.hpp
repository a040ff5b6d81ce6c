// dev_dwt.hpp -- device bodies of the DWT (Sec. 3 eqs. 8-9, Fig. 1): the LDS cascade (per-cube
// and persistent batch kernels), the banded and the LDS-staged equivalent filters (the
// per-cube kernels and the fused DWT + detector launch).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

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

    // coalesced load of np contiguous spectra, four unconditional loads per thread in
    // flight (index clamped), then the stores
    const float *src = cube + p0 * (int64_t)L;
    const int total = np * L;
    for (int t0 = 0; t0 < total; t0 += 4 * 256) {
        float v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int t = t0 + 256 * u + tid;
            v[u] = src[t < total ? t : total - 1];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int t = t0 + 256 * u + tid;
            if (t < total) {
                const int p = t / L, i = t - p * L;
                buf0[p * S0 + i] = (double)v[u];
            }
        }
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


// ------------------------------------------------------------------------------------
// Banded equivalent filter.  After J levels, output k depends only on a circular window of
// the input: at most 7 (2^J - 1) + 1 samples, because each level reads 8 taps at stride 2
// (the odd-length extension only repeats a neighbouring sample).  coef holds, for every
// output k, W coefficients of that window ([L'][W], FP64, zero past the row's own width),
// and start[k] its first input index.  The cascade's composite map is the same linear map,
// so this gives the cascade's result with W FMAs per output instead of 8 per level, in one
// pass over the input.
// ------------------------------------------------------------------------------------
// LDS floats of a tile of P spectra: input rows of L + W - 1 samples (the first W - 1 samples
// repeated after the last, so that a window never wraps), odd stride; output rows of stride L'|1.
__host__ __device__ inline int64_t dwt_banded_lds_floats(int64_t L, int64_t Lp, int64_t W, int64_t P)
{
    return P * ((L + W - 1) | 1) + P * (Lp | 1);
}

// np (<= P <= 64) contiguous spectra starting at pixel p0; a workgroup of NT threads.
// Stage: the np*L contiguous input floats are copied into padded LDS rows (float4 loads
// when L % 4 == 0), with the circular extension.  Compute: lane = pixel, wavefront w takes
// outputs k = w, w + NT/64, ..., so k (and every coefficient address) is uniform across the
// wavefront, and a lane reads W consecutive samples of its own row (odd stride: no bank
// conflicts; constant offsets).  FP64 accumulation.  Write-out: the np*L' outputs leave
// through padded LDS rows as one contiguous store.
// magic_L = ceil(2^32 / L), magic_Lp = ceil(2^32 / L'): exact quotients for t < 64 L.
template <int VEC, int NT = 256>
__device__ inline void dwt_banded_tile(const float *__restrict__ cube, int64_t p0, int np, int L, int Lp,
                                       int W, const double *__restrict__ coef,
                                       const int32_t *__restrict__ start, uint32_t magic_L,
                                       uint32_t magic_Lp, float *__restrict__ out, float *lds, int P)
{
    const int LDP = (L + W - 1) | 1, LDO = Lp | 1;
    const uint32_t ext = (uint32_t)(W - 1);
    float *xs = lds;                          // P * LDP
    float *os = lds + (size_t)P * LDP;        // P * LDO
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;

    const float *src = cube + p0 * (int64_t)L;
    const int total = np * L;
    if constexpr (VEC == 4) {
        const int nv = total >> 2;
        const float4 *s4 = reinterpret_cast<const float4 *>(src);
        // four loads per thread in flight: unconditional (index clamped), then the stores
        for (int v0 = 0; v0 < nv; v0 += 4 * NT) {
            float4 qs[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int v = v0 + NT * u + tid;
                qs[u] = s4[v < nv ? v : nv - 1];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int v = v0 + NT * u + tid;
                if (v >= nv) continue;
                const float4 q = qs[u];
                const uint32_t e = 4u * (uint32_t)v;
                const uint32_t r = __umulhi(e, magic_L);
                const uint32_t col = e - r * (uint32_t)L;
                float *d = xs + r * LDP + col;
                d[0] = q.x;
                d[1] = q.y;
                d[2] = q.z;
                d[3] = q.w;
                if (col < ext) {
                    float *dd = d + L;
                    const float qq[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        if (col + j < ext) dd[j] = qq[j];
                }
            }
        }
    } else {
        // L not a multiple of 4: the tile's np*L floats are still contiguous and start on a
        // 16-byte boundary (P is a multiple of 4), so they load as float4 and each element
        // finds its own row; the last total % 4 floats load one by one
        const int nv = total >> 2;
        const float4 *s4 = reinterpret_cast<const float4 *>(src);
        for (int v0 = 0; v0 < nv; v0 += 4 * NT) {
            float4 qs[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int v = v0 + NT * u + tid;
                qs[u] = s4[v < nv ? v : (nv > 0 ? nv - 1 : 0)];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int v = v0 + NT * u + tid;
                if (v >= nv) continue;
                const float qq[4] = {qs[u].x, qs[u].y, qs[u].z, qs[u].w};
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const uint32_t e = 4u * (uint32_t)v + (uint32_t)j;
                    const uint32_t r = __umulhi(e, magic_L);
                    const uint32_t col = e - r * (uint32_t)L;
                    xs[r * LDP + col] = qq[j];
                    if (col < ext) xs[r * LDP + col + L] = qq[j];
                }
            }
        }
        for (int t = 4 * nv + tid; t < total; t += NT) {
            const uint32_t r = __umulhi((uint32_t)t, magic_L);
            const uint32_t col = (uint32_t)t - r * (uint32_t)L;
            const float v = src[t];
            xs[r * LDP + col] = v;
            if (col < ext) xs[r * LDP + col + L] = v;
        }
    }
    __syncthreads();

    if (lane < np) {
        const float *xp = xs + lane * LDP;
        for (int k = wave; k < Lp; k += NT / 64) {
            const double *c = coef + (size_t)k * W;
            const float *xk = xp + start[k];
            double a0 = 0.0, a1 = 0.0;
            int t = 0;
            for (; t + 8 <= W; t += 8) {
#pragma unroll
                for (int u = 0; u < 8; u += 2) {
                    a0 = fma(c[t + u], (double)xk[t + u], a0);
                    a1 = fma(c[t + u + 1], (double)xk[t + u + 1], a1);
                }
            }
            for (; t < W; ++t) a0 = fma(c[t], (double)xk[t], a0);
            os[lane * LDO + k] = (float)(a0 + a1);
        }
    }
    __syncthreads();

    float *dst = out + p0 * (int64_t)Lp;
    const int ototal = np * Lp;
#pragma unroll 4
    for (int t = tid; t < ototal; t += NT) {
        const uint32_t r = __umulhi((uint32_t)t, magic_Lp);
        dst[t] = os[r * LDO + ((uint32_t)t - r * (uint32_t)Lp)];
    }
}

// ------------------------------------------------------------------------------------
// equivalent filter with coalesced, LDS-staged band chunks (Sec. 3: the J-level
// approximation as one L' x L matrix applied to each spectrum)
// ------------------------------------------------------------------------------------
typedef float fv2 __attribute__((ext_vector_type(2)));
typedef float fv4 __attribute__((ext_vector_type(4)));
template <int VEC> struct VecT;
template <> struct VecT<1> { using T = float; };
template <> struct VecT<2> { using T = fv2; };
template <> struct VecT<4> { using T = fv4; };

template <int VEC>
__device__ __forceinline__ float lane_elem(const typename VecT<VEC>::T &v, int e)
{
    if constexpr (VEC == 1) {
        return v;
    } else {
        return v[e];
    }
}

// A workgroup of NT threads owns NT consecutive pixels (one per thread) and walks the
// spectrum in chunks of 32 bands.  Each chunk is loaded with whole 128-byte lines per pixel
// (8 lanes x 16 bytes, or 32 lanes x 4 bytes when L is not a multiple of 4) into LDS.
// There it is transposed to one row per pixel (stride 33 floats, conflict-free).  The
// next chunk's loads are issued into registers before the current chunk is computed, so
// HBM streaming overlaps the FP64 FMAs.  Load addresses are clamped into the tile (last
// pixel, last vector of the chunk) so every lane loads unconditionally: loads under a
// lane-dependent condition cost about 15 % of the bandwidth here.  The clamped duplicates
// land in LDS cells that are never read.
//   coef : [L][L'] doubles (band-major composite matrix)
//   tile : NT * kEqLd floats of LDS
//   blk  : index of the block of NT pixels
constexpr int kEqCB = 32, kEqTP = 256, kEqLd = kEqCB + 1;

template <int LP, int VEC, bool NTL, int NT>
__device__ inline void dwt_equiv_lds_block(const float *__restrict__ cube, int64_t npix, int L,
                                           const double *__restrict__ coef, float *__restrict__ out,
                                           float *tile, int64_t blk)
{
    constexpr int PER = kEqCB / VEC;              // vectors per thread per chunk
    static_assert(kEqCB % VEC == 0, "chunk of whole vectors");
    using V = typename VecT<VEC>::T;
    const int t = threadIdx.x;
    const int64_t p0 = blk * NT;
    const int np = (int)((npix - p0) < NT ? (npix - p0) : NT);
    const int nchunk = (L + kEqCB - 1) / kEqCB;
    constexpr int SEG = kEqCB / VEC;              // vectors per pixel segment (= PER: NT pixels, NT threads)

    auto load_chunk = [&](V (&buf)[PER], int c0) {
        const int cb = (L - c0) < kEqCB ? (L - c0) : kEqCB;
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int q = t + NT * i;
            const int p = min(q / SEG, np - 1), j = min((q % SEG) * VEC, cb - VEC);
            // the cube is read exactly once: non-temporal loads keep it from displacing
            // cached data
            const V *a = reinterpret_cast<const V *>(cube + (p0 + p) * (int64_t)L + c0 + j);
            buf[i] = NTL ? __builtin_nontemporal_load(a) : *a;
        }
    };
    auto store_chunk = [&](const V (&buf)[PER]) {
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int q = t + NT * i;
            const int p = q / SEG, j = q % SEG;
#pragma unroll
            for (int e = 0; e < VEC; ++e) tile[p * kEqLd + j * VEC + e] = lane_elem<VEC>(buf[i], e);
        }
    };

    double acc[LP];
#pragma unroll
    for (int k = 0; k < LP; ++k) acc[k] = 0.0;
    auto compute = [&](int c0) {
        const int cb = (L - c0) < kEqCB ? (L - c0) : kEqCB;
        const float *row = tile + t * kEqLd;
        const double *cf = coef + (size_t)c0 * LP;
        if (cb == kEqCB) {
#pragma unroll 8
            for (int b = 0; b < kEqCB; ++b) {
                const double xv = (double)row[b];
#pragma unroll
                for (int k = 0; k < LP; ++k) acc[k] = fma(cf[b * LP + k], xv, acc[k]);
            }
        } else {
            for (int b = 0; b < cb; ++b) {
                const double xv = (double)row[b];
#pragma unroll
                for (int k = 0; k < LP; ++k) acc[k] = fma(cf[b * LP + k], xv, acc[k]);
            }
        }
    };

    V buf[PER];
    load_chunk(buf, 0);
    for (int ch = 0; ch < nchunk; ++ch) {
        const int c0 = ch * kEqCB;
        store_chunk(buf);
        __syncthreads();
        if (ch + 1 < nchunk) load_chunk(buf, c0 + kEqCB);
        compute(c0);
        __syncthreads();
    }
    if (t >= np) return;
    float *dst = out + (p0 + t) * LP;
    if constexpr (LP % 4 == 0) {
#pragma unroll
        for (int k = 0; k < LP; k += 4)
            *reinterpret_cast<float4 *>(dst + k) =
                make_float4((float)acc[k], (float)acc[k + 1], (float)acc[k + 2], (float)acc[k + 3]);
    } else if constexpr (LP % 2 == 0) {
#pragma unroll
        for (int k = 0; k < LP; k += 2)
            *reinterpret_cast<float2 *>(dst + k) = make_float2((float)acc[k], (float)acc[k + 1]);
    } else {
#pragma unroll
        for (int k = 0; k < LP; ++k) dst[k] = (float)acc[k];
    }
}

}  // namespace hsad
