// The per-tile body of the fused absorb -> solve -> emit kernel, shared by
// the single-grid fused launch and the batched persistent launch.
#pragma once

#include "device_common.h"

namespace dust {

constexpr int FUSED_TC = 16;  // default cells per tile (one MFMA M-block)

// Phase 1: heating of a 16-cell block into sH[16][Sp] (rows of the tile's
// LDS array) in the plan's scaled units H' = H 2^es.  Wave w computes grain
// tiles w, w+4, ... (NTW of them).
template <int MODE, int NTW>
__device__ __forceinline__ void fused_absorb(const PlanView& v, int64_t c0, int64_t C,
                                             const float* __restrict__ J, int64_t ldj,
                                             float* sH) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int row = lane & 15, kq = lane >> 4;
    const int64_t c = c0 + row;
    const bool cv = c < C;
    const float* jr = J + (cv ? c : 0) * ldj;
    const int tiles = v.Sp / 16;
    f32x4 acc[NTW];
#pragma unroll
    for (int t = 0; t < NTW; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};

    if constexpr (MODE == DUST_MIXED) {
        for (int k0 = 0; k0 < v.NL; k0 += 32) {
            const int kb = k0 + kq * 8;
            float x[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) x[i] = (cv && kb + i < v.NL) ? jr[kb + i] : 0.0f;
            bf16x8 ahi, alo;
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                ahi[i] = (__bf16)x[i];
                alo[i] = (__bf16)(x[i] - (float)ahi[i]);
            }
#pragma unroll
            for (int t = 0; t < NTW; ++t) {
                const int tile = wave + 4 * t;
                if (tile < tiles) {
                    const int s = tile * 16 + row;
                    const bf16x8 bhi = *reinterpret_cast<const bf16x8*>(v.khi + (int64_t)s * v.NLp + kb);
                    const bf16x8 blo = *reinterpret_cast<const bf16x8*>(v.klo + (int64_t)s * v.NLp + kb);
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi, bhi, acc[t], 0, 0, 0);
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi, blo, acc[t], 0, 0, 0);
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo, bhi, acc[t], 0, 0, 0);
                }
            }
        }
    } else {
        for (int k0 = 0; k0 < v.NL; k0 += 32) {
            float a[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int k = k0 + 4 * i + kq;
                a[i] = (cv && k < v.NL) ? jr[k] : 0.0f;
            }
#pragma unroll
            for (int t = 0; t < NTW; ++t) {
                const int tile = wave + 4 * t;
                if (tile < tiles) {
                    const float* kr = v.kf + (int64_t)(tile * 16 + row) * v.NLp + k0 + kq;
#pragma unroll
                    for (int i = 0; i < 8; ++i)
                        acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], kr[4 * i], acc[t], 0, 0, 0);
                }
            }
        }
    }
#pragma unroll
    for (int t = 0; t < NTW; ++t) {
        const int tile = wave + 4 * t;
        if (tile < tiles) {
            const int s = tile * 16 + row;
#pragma unroll
            for (int r = 0; r < 4; ++r) sH[(kq * 4 + r) * v.Sp + s] = acc[t][r];
        }
    }
}

// Phases 2 and 3 on a tile whose scaled heating sits in sH: solve every pair
// (T to device memory, 1/T back into sH), then emit the tile's SEDs.  The
// group minima of 1/T follow sH in LDS (see emit_accumulate).
template <int MODE, int TC>
__device__ __forceinline__ void fused_solve_emit(const PlanView& v, int64_t c0, int64_t C,
                                                 const float* __restrict__ m,
                                                 float* __restrict__ T, int64_t ldt,
                                                 float* __restrict__ L, int64_t ldl,
                                                 dust_counters* cnt, float* sH) {
    const int n = TC * v.Sp;
    // Same trip count for every lane: the mixed solve works wave-wide.
    for (int base = 0; base < n; base += blockDim.x) {
        const int i = base + threadIdx.x;
        const int cc = i / v.Sp, s = i - cc * v.Sp;
        const int64_t c = c0 + cc;
        const bool pair = i < n && s < v.S && c < C;
        float t = 0.0f;
        if constexpr (MODE == DUST_MIXED) {
            t = wave_solve_mixed(v, pair, pair ? s : 0, pair ? (double)sH[i] : 0.0, cnt);
        } else {
            if (pair)
                t = solve_newton_f32(v.kb + (int64_t)s * v.NLp, v.nu, v.NL, sH[i], v.gs[s],
                                     v.tol, v.maxit, cnt);
        }
        if (pair) T[c * ldt + s] = t;
        if (i < n) sH[i] = pair ? inv_temperature(t) : __builtin_inff();
    }
    __syncthreads();
    uint32_t* sChunk = reinterpret_cast<uint32_t*>(sH + n);
    fill_chunk_min<TC>(sH, sChunk, v.Sp);
    __syncthreads();
    float mc[TC];
#pragma unroll
    for (int cc = 0; cc < TC; ++cc) {
        const int64_t c = c0 + cc;
        mc[cc] = (c < C) ? ((m ? m[c] : 1.0f) * v.escale) : 0.0f;
    }
    for (int l0 = 0; l0 < v.NL; l0 += blockDim.x) {
        const int l = l0 + threadIdx.x;
        const bool lv = l < v.NL;
        const float nu = v.nu[lv ? l : 0];
        const float uw = wave_u_min(v.nu, l0 + (threadIdx.x & ~63), v.NL);
        float acc[TC];
        emit_accumulate<TC>(v.em + (lv ? l : 0), v.NLp, nu, uw, sH, sChunk, v.Sp, v.S, acc);
        if (lv) {
#pragma unroll
            for (int cc = 0; cc < TC; ++cc)
                if (c0 + cc < C) L[(c0 + cc) * ldl + l] = acc[cc] * mc[cc];
        }
    }
}

// One tile of TC cells (TC a multiple of 16) starting at cell c0; sH holds
// fused_lds_bytes(TC, Sp) bytes of LDS.  Ends with every thread past its last
// read of the tile's LDS.
template <int MODE, int TC, int NTW>
__device__ __forceinline__ void fused_tile(const PlanView& v, int64_t c0, int64_t C,
                                           const float* __restrict__ J, int64_t ldj,
                                           const float* __restrict__ m, float* __restrict__ T,
                                           int64_t ldt, float* __restrict__ L, int64_t ldl,
                                           dust_counters* cnt, float* sH) {
#pragma unroll
    for (int mb = 0; mb < TC / 16; ++mb)
        fused_absorb<MODE, NTW>(v, c0 + 16 * mb, C, J, ldj, sH + 16 * mb * v.Sp);
    __syncthreads();
    fused_solve_emit<MODE, TC>(v, c0, C, m, T, ldt, L, ldl, cnt, sH);
    __syncthreads();
}

}  // namespace dust
