// dev_gram.hpp -- device body of the per-pixel window statistics on matrix cores (one
// wavefront per pixel), shared by the per-cube kernel and the persistent batch kernel.
// See gram.hip for the method notes.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

#include "internal.hpp"

namespace hsad {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

struct GramArgs {
    const float *x;
    int H, W, Lp;
    int R, RI, has_inner;
    int mode;            // GramMode
    int64_t pix0;        // first pixel of the chunk
    int npix;            // pixels in the chunk
    double *ws;          // chunk workspace, (Lp+2)*Lp doubles per pixel
    uint32_t outer_magic;  // ceil(2^32 / outer) for k / outer
    const int32_t *idx;  // optional pixel list: pixel = idx[pix0 + local] (NULL: pix0 + local)
    int means_ready;     // workgroup kernel: the means are already in rows L', L'+1 of each record
};


__device__ __forceinline__ bool sample_pos(const GramArgs &a, int py, int px, int k, int &sy,
                                           int &sx, bool &in_inner)
{
    const int outer = 2 * a.R + 1;
    const int q = (int)__umulhi((uint32_t)k, a.outer_magic);
    const int dy = q - a.R, dx = k - q * outer - a.R;
    sy = py + dy;
    sx = px + dx;
    in_inner = a.has_inner && dy >= -a.RI && dy <= a.RI && dx >= -a.RI && dx <= a.RI;
    return sy >= 0 && sy < a.H && sx >= 0 && sx < a.W;
}

__device__ __forceinline__ int clipn(int c, int r, int n)
{
    const int lo = c - r < 0 ? 0 : c - r, hi = c + r > n - 1 ? n - 1 : c + r;
    return hi - lo + 1;
}

// Layout of one wave's LDS region (doubles): stage[T][64] then mu[Lpad], mi[Lpad].
template <int PREC, int kMaxTilesPerPass>
__device__ inline void gram_pixel(const GramArgs &a, int local, double *stage)
{
    const int lane = threadIdx.x & 63;
    const int T = (a.Lp + 15) >> 4;
    const int Lpad = T * 16;
    double *mu = stage + (size_t)T * 64 * (PREC == 2 || PREC == 3 ? 2 : 1);
    double *mi = mu + Lpad;
    const int64_t pix = a.idx ? (int64_t)a.idx[a.pix0 + local] : a.pix0 + local;
    if (pix < 0 || pix >= (int64_t)a.H * a.W) return;   // listed index outside the image: skipped
    const int py = (int)(pix / a.W), px = (int)(pix - (int64_t)py * a.W);
    const int c16 = lane & 15, g4 = lane >> 4;
    const int K = (2 * a.R + 1) * (2 * a.R + 1);
    const int n_o = clipn(py, a.R, a.H) * clipn(px, a.R, a.W);
    const int n_i = a.has_inner ? clipn(py, a.RI, a.H) * clipn(px, a.RI, a.W) : 0;
    const int n_a = n_o - n_i;
    if constexpr (PREC != 0) {
        // a clipped annulus (image borders) with fewer than 2 L' samples gives a nearly
        // singular covariance, which the reduced precisions would not resolve: FP64 there
        if (a.mode == GRAM_LRX && n_a < 2 * a.Lp) {
            gram_pixel<0, kMaxTilesPerPass>(a, local, stage);
            return;
        }
    }

    // ---- pass 1: FP64 sums over the annulus and the inner window ----
    // Loads are unconditional (clamped coordinates and component) with a wave-uniform
    // trip count; samples outside the window or the image are dropped by selects.  A load
    // under a lane-dependent branch whose value is used inside it would wait for its round
    // trip before the next one is issued.
    for (int b = 0; b < T; ++b) {
        const int comp = 16 * b + c16;
        const int cc = comp < a.Lp ? comp : a.Lp - 1;
        double sa = 0.0, si = 0.0;
#pragma unroll 4
        for (int k0 = 0; k0 < K; k0 += 4) {
            const int k = k0 + g4;
            int sy, sx;
            bool inn;
            const bool ok = sample_pos(a, py, px, k < K ? k : K - 1, sy, sx, inn) && k < K && comp < a.Lp;
            const int cy = sy < 0 ? 0 : sy >= a.H ? a.H - 1 : sy, cx = sx < 0 ? 0 : sx >= a.W ? a.W - 1 : sx;
            const double v = (double)a.x[((size_t)cy * a.W + cx) * a.Lp + cc];
            si += ok && inn ? v : 0.0;
            sa += ok && !inn ? v : 0.0;
        }
        // reduce over the four sample groups (lanes c16, c16+16, c16+32, c16+48)
        sa += __shfl_xor(sa, 16);
        sa += __shfl_xor(sa, 32);
        si += __shfl_xor(si, 16);
        si += __shfl_xor(si, 32);
        if (g4 == 0) {
            mu[comp] = comp < a.Lp ? sa / (double)n_a : 0.0;
            mi[comp] = (comp < a.Lp && n_i > 0) ? si / (double)n_i : 0.0;
        }
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");

    double *out = a.ws + (size_t)local * (a.Lp + 2) * a.Lp;
    // vectors: LRX mode rows Lp (x_p - mu) and Lp+1 (m_in - mu); DWEST row Lp (m_in - mu)
    for (int comp = lane; comp < a.Lp; comp += 64) {
        const double m = mu[comp];
        if (a.mode == GRAM_LRX) {
            out[(size_t)a.Lp * a.Lp + comp] = (double)a.x[(size_t)pix * a.Lp + comp] - m;
            out[(size_t)(a.Lp + 1) * a.Lp + comp] = mi[comp] - m;
        } else {
            out[(size_t)a.Lp * a.Lp + comp] = mi[comp] - m;
        }
    }

    // ---- pass 2: MFMA Gram over tiles (bi <= bj), up to 16 tiles per pass ----
    const int ntiles = T * (T + 1) / 2;
    const double wa = a.mode == GRAM_DWEST ? -1.0 / (double)n_a : 1.0;
    const double wi = a.mode == GRAM_DWEST ? 1.0 / (double)(n_i > 0 ? n_i : 1) : 0.0;
    const double scale_out = a.mode == GRAM_DWEST ? 1.0 : 1.0 / (double)n_a;
    constexpr int KG = (PREC == 2 || PREC == 3) ? 32 : 4;   // samples per MFMA
    constexpr int SPL = KG / 4;                              // samples per lane
    // inner samples only feed DWEST; annulus samples feed both modes
    const int nsets = a.mode == GRAM_DWEST ? 2 : 1;

    using Acc = typename std::conditional<PREC == 0, f64x4, f32x4>::type;
    for (int t0 = 0; t0 < ntiles; t0 += kMaxTilesPerPass) {
        const int nt = ntiles - t0 < kMaxTilesPerPass ? ntiles - t0 : kMaxTilesPerPass;
        // tile t of this pass -> (bi, bj), row-major over the upper triangle
        int tbi[kMaxTilesPerPass], tbj[kMaxTilesPerPass];
        {
            int rem = t0, bi = 0;
            while (bi < T && rem >= T - bi) {
                rem -= T - bi;
                ++bi;
            }
            int bj = bi + rem;
#pragma unroll
            for (int t = 0; t < kMaxTilesPerPass; ++t) {
                tbi[t] = bi;
                tbj[t] = bj;
                if (++bj >= T) {
                    ++bi;
                    bj = bi;
                }
            }
        }
        Acc acc[kMaxTilesPerPass];
#pragma unroll
        for (int t = 0; t < kMaxTilesPerPass; ++t)
            for (int e = 0; e < 4; ++e) acc[t][e] = 0;
        for (int set = 0; set < nsets; ++set) {
            // set 0: annulus (weight wa), set 1: inner window (weight wi)
            const double w = set == 0 ? wa : wi;
            for (int k0 = 0; k0 < K; k0 += KG) {
                // stage this lane's centred values for every block
                for (int b = 0; b < T; ++b) {
                    const int comp = 16 * b + c16;
                    double vals[SPL];
#pragma unroll
                    for (int s = 0; s < SPL; ++s) {
                        const int k = k0 + g4 * SPL + s;
                        int sy, sx;
                        bool inn;
                        const bool ok = sample_pos(a, py, px, k < K ? k : K - 1, sy, sx, inn) && k < K &&
                                        comp < a.Lp && (set == 0 ? !inn : inn);
                        const int cc = comp < a.Lp ? comp : a.Lp - 1;
                        const int cy = sy < 0 ? 0 : sy >= a.H ? a.H - 1 : sy;
                        const int cx = sx < 0 ? 0 : sx >= a.W ? a.W - 1 : sx;
                        const double xv = (double)a.x[((size_t)cy * a.W + cx) * a.Lp + cc];
                        vals[s] = ok ? xv - (set == 0 ? mu[cc] : mi[cc]) : 0.0;
                    }
                    if constexpr (PREC == 0) {
                        stage[b * 64 + lane] = vals[0];
                    } else if constexpr (PREC == 1) {
                        reinterpret_cast<float *>(stage)[b * 64 + lane] = (float)vals[0];
                    } else {
                        // 8 x 16-bit values per lane per block (16 bytes)
                        uint16_t *st16 = reinterpret_cast<uint16_t *>(stage) + (size_t)(b * 64 + lane) * 8;
#pragma unroll
                        for (int s = 0; s < 8; ++s) {
                            if constexpr (PREC == 2) {
                                __bf16 hv = (__bf16)(float)vals[s];
                                st16[s] = __builtin_bit_cast(uint16_t, hv);
                            } else {
                                _Float16 hv = (_Float16)(float)vals[s];
                                st16[s] = __builtin_bit_cast(uint16_t, hv);
                            }
                        }
                    }
                }
#pragma unroll
                for (int t = 0; t < kMaxTilesPerPass; ++t) {
                    if (t < nt) {
                        const int bi = tbi[t], bj = tbj[t];
                        if constexpr (PREC == 0) {
                            const double av = stage[bi * 64 + lane] * w, bv = stage[bj * 64 + lane];
                            acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[t], 0, 0, 0);
                        } else if constexpr (PREC == 1) {
                            const float *sf = reinterpret_cast<const float *>(stage);
                            acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(sf[bi * 64 + lane], sf[bj * 64 + lane],
                                                                          acc[t], 0, 0, 0);
                        } else if constexpr (PREC == 2) {
                            const bf16x8 *s8 = reinterpret_cast<const bf16x8 *>(stage);
                            acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(s8[bi * 64 + lane], s8[bj * 64 + lane],
                                                                             acc[t], 0, 0, 0);
                        } else {
                            const f16x8 *s8 = reinterpret_cast<const f16x8 *>(stage);
                            acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_f16(s8[bi * 64 + lane], s8[bj * 64 + lane],
                                                                            acc[t], 0, 0, 0);
                        }
                    }
                }
            }
        }
        // write the tiles (and their mirror images) scaled to covariances
#pragma unroll
        for (int t = 0; t < kMaxTilesPerPass; ++t) {
            if (t < nt) {
                const int bi = tbi[t], bj = tbj[t];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    // output element e of lane l: FP64 16x16x4 puts it at row 4e + (l>>4),
                    // the FP32/BF16/FP16 16x16 variants at row 4(l>>4) + e; column l&15
                    const int r = 16 * bi + (PREC == 0 ? 4 * e + g4 : 4 * g4 + e), c = 16 * bj + c16;
                    const double v = (double)acc[t][e] * scale_out;
                    // one writer per symmetric pair keeps the result deterministic
                    if (r < a.Lp && c < a.Lp && (bi < bj || r <= c)) {
                        out[(size_t)r * a.Lp + c] = v;
                        out[(size_t)c * a.Lp + r] = v;
                    }
                }
            }
        }
    }
}


// LDS doubles of one wavefront's region.
__host__ __device__ inline size_t gram_wave_doubles(int Lp, int prec)
{
    const int T = (Lp + 15) / 16;
    return (size_t)T * 64 * ((prec == 2 || prec == 3) ? 2 : 1) + 2 * (size_t)T * 16;
}

}  // namespace hsad
