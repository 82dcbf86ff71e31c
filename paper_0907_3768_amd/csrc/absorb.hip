// Heating, Eq. 6 (Section 4.2): H[c,s] = sum_l J[c,l] K[s,l], a dense
// contraction over wavelength on the MFMA units.
//
// One wave computes a 16-cell x (16 NT)-grain block; a workgroup of four
// waves covers 64 cells.  The grid's y dimension walks groups of 16 NT grains.
//   DUST_PLAIN_FP32: v_mfma_f32_16x16x4_f32 (exact FP32 products).
//   DUST_MIXED:      v_mfma_f32_16x16x32_bf16 on hi+lo splits,
//                    J_hi K_hi + J_hi K_lo + J_lo K_hi, FP32 accumulation.
// Operand layouts (CDNA3/4 MFMA): for 16x16xK, lane i feeds row (i mod 16)
// of A and column (i mod 16) of B, with K-elements [kq*K/4, (kq+1)*K/4) where
// kq = i / 16; the 4 accumulator values of lane i are rows 4 kq + r, column
// (i mod 16) of the 16x16 result.
#include "internal.h"

namespace dust {
namespace {

template <int NT>
__global__ __launch_bounds__(256) void absorb_bf16x3_kernel(PlanView v, int64_t C,
                                                            const float* __restrict__ J,
                                                            int64_t ldj, float* __restrict__ H,
                                                            int64_t ldh) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int row = lane & 15, kq = lane >> 4;
    const int64_t c0 = (int64_t)blockIdx.x * 64 + wave * 16;
    const int sg0 = blockIdx.y * NT * 16;
    const int64_t c = c0 + row;
    const bool cv = c < C;
    const float* jr = J + (cv ? c : 0) * ldj;
    f32x4 acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};

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
        for (int t = 0; t < NT; ++t) {
            const int s = sg0 + t * 16 + row;
            if (sg0 + t * 16 < v.Sp) {
                const bf16x8 bhi = *reinterpret_cast<const bf16x8*>(v.khi + (int64_t)s * v.NLp + kb);
                const bf16x8 blo = *reinterpret_cast<const bf16x8*>(v.klo + (int64_t)s * v.NLp + kb);
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi, bhi, acc[t], 0, 0, 0);
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi, blo, acc[t], 0, 0, 0);
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo, bhi, acc[t], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int s = sg0 + t * 16 + row;
        if (s < v.S) {
            const float inv = v.hinv[s];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t cc = c0 + kq * 4 + r;
                if (cc < C) H[cc * ldh + s] = acc[t][r] * inv;
            }
        }
    }
}

template <int NT>
__global__ __launch_bounds__(256) void absorb_f32_kernel(PlanView v, int64_t C,
                                                         const float* __restrict__ J,
                                                         int64_t ldj, float* __restrict__ H,
                                                         int64_t ldh) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int row = lane & 15, kq = lane >> 4;
    const int64_t c0 = (int64_t)blockIdx.x * 64 + wave * 16;
    const int sg0 = blockIdx.y * NT * 16;
    const int64_t c = c0 + row;
    const bool cv = c < C;
    const float* jr = J + (cv ? c : 0) * ldj;
    f32x4 acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};

    for (int k0 = 0; k0 < v.NL; k0 += 32) {
        float a[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int k = k0 + 4 * i + kq;
            a[i] = (cv && k < v.NL) ? jr[k] : 0.0f;
        }
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            if (sg0 + t * 16 < v.Sp) {
                const float* kr = v.kf + (int64_t)(sg0 + t * 16 + row) * v.NLp + k0 + kq;
#pragma unroll
                for (int i = 0; i < 8; ++i)
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], kr[4 * i], acc[t], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int s = sg0 + t * 16 + row;
        if (s < v.S) {
            const float inv = v.hinv[s];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t cc = c0 + kq * 4 + r;
                if (cc < C) H[cc * ldh + s] = acc[t][r] * inv;
            }
        }
    }
}

template <int NT>
hipError_t launch_nt(const PlanView& v, int64_t C, const float* J, int64_t ldj, float* H,
                     int64_t ldh, hipStream_t st) {
    const int tiles = v.Sp / 16;
    dim3 grid((unsigned)((C + 63) / 64), (unsigned)((tiles + NT - 1) / NT));
    if (v.mode == DUST_MIXED)
        hipLaunchKernelGGL(absorb_bf16x3_kernel<NT>, grid, dim3(256), 0, st, v, C, J, ldj, H, ldh);
    else
        hipLaunchKernelGGL(absorb_f32_kernel<NT>, grid, dim3(256), 0, st, v, C, J, ldj, H, ldh);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_absorb(const PlanView& v, int64_t C, const float* J, int64_t ldj, float* H,
                         int64_t ldh, hipStream_t st) {
    if (C == 0) return hipSuccess;
    const int tiles = v.Sp / 16;
    // As many grain tiles per wave as fit in 16 (64 accumulator registers).
    if (tiles <= 1) return launch_nt<1>(v, C, J, ldj, H, ldh, st);
    if (tiles <= 2) return launch_nt<2>(v, C, J, ldj, H, ldh, st);
    if (tiles <= 3) return launch_nt<3>(v, C, J, ldj, H, ldh, st);
    if (tiles <= 4) return launch_nt<4>(v, C, J, ldj, H, ldh, st);
    if (tiles <= 5) return launch_nt<5>(v, C, J, ldj, H, ldh, st);
    if (tiles <= 6) return launch_nt<6>(v, C, J, ldj, H, ldh, st);
    if (tiles <= 8) return launch_nt<8>(v, C, J, ldj, H, ldh, st);
    if (tiles <= 10) return launch_nt<10>(v, C, J, ldj, H, ldh, st);
    if (tiles <= 12) return launch_nt<12>(v, C, J, ldj, H, ldh, st);
    if (tiles <= 14) return launch_nt<14>(v, C, J, ldj, H, ldh, st);
    return launch_nt<16>(v, C, J, ldj, H, ldh, st);
}

}  // namespace dust
