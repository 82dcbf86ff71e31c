// Heating, Eq. 6 (Section 4.2): H[c,s] = sum_l J[c,l] K[s,l], a dense
// contraction over wavelength on the MFMA units.
//
// A workgroup computes the heating of 16 cells for every grain with the
// LDS-staged MFMA routine of the fused kernel (fused_absorb), then writes
// the 16 x S block of H with coalesced stores, undoing the per-grain power
// of two.
//   DUST_PLAIN_FP32: v_mfma_f32_16x16x4_f32 (exact FP32 products).
//   DUST_MIXED, DUST_TABLE_LINEAR:
//                    v_mfma_f32_16x16x32_bf16 on hi+lo splits,
//                    J_hi K_hi + J_hi K_lo + J_lo K_hi, FP32 accumulation.
#include "fused_body.h"

namespace dust {
namespace {

template <int MODE, int NTW>
__global__ __launch_bounds__(256) void absorb_kernel(PlanView v, int64_t C,
                                                     const float* __restrict__ J, int64_t ldj,
                                                     float* __restrict__ H, int64_t ldh) {
    extern __shared__ float lds[];  // sH [16][Sp], then the J staging buffers
    float* sH = lds;
    char* sStage = reinterpret_cast<char*>(lds + 16 * v.Sp);
    const int64_t c0 = (int64_t)blockIdx.x * 16;
    fused_absorb<MODE, NTW>(v, c0, C, J, ldj, sH, sStage);
    __syncthreads();
    for (int i = threadIdx.x; i < 16 * v.Sp; i += 256) {
        const int cc = i / v.Sp, s = i - cc * v.Sp;
        if (s < v.S && c0 + cc < C) H[(c0 + cc) * ldh + s] = sH[i] * v.hinv[s];
    }
}

template <int NTW>
hipError_t launch_ntw(const PlanView& v, int64_t C, const float* J, int64_t ldj, float* H,
                      int64_t ldh, hipStream_t st) {
    const dim3 grid((unsigned)((C + 15) / 16));
    const size_t lds = sizeof(float) * 16 * v.Sp + STAGE_BYTES;
    if (table_mode(v.mode))  // bf16 hi+lo heating
        hipLaunchKernelGGL((absorb_kernel<DUST_MIXED, NTW>), grid, dim3(256), lds, st, v, C, J,
                           ldj, H, ldh);
    else
        hipLaunchKernelGGL((absorb_kernel<DUST_PLAIN_FP32, NTW>), grid, dim3(256), lds, st, v, C,
                           J, ldj, H, ldh);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_absorb(const PlanView& v, int64_t C, const float* J, int64_t ldj, float* H,
                         int64_t ldh, hipStream_t st) {
    if (C == 0) return hipSuccess;
    const int ntw = (v.Sp / 16 + 3) / 4;  // grain tiles per wave in one pass
    if (ntw <= 1) return launch_ntw<1>(v, C, J, ldj, H, ldh, st);
    if (ntw <= 2) return launch_ntw<2>(v, C, J, ldj, H, ldh, st);
    if (ntw <= 3) return launch_ntw<3>(v, C, J, ldj, H, ldh, st);
    if (ntw <= 4) return launch_ntw<4>(v, C, J, ldj, H, ldh, st);
    return launch_ntw<4>(v, C, J, ldj, H, ldh, st);  // several passes
}

}  // namespace dust
