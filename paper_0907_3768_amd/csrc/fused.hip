// Fused absorb -> solve -> emit (Eqs. 6, 7, 9-10) for a tile of 16 cells per
// workgroup.  The heating tile goes from the MFMA accumulators to LDS, is
// solved in place (LDS then holds 1/T), and feeds the emission loop: H never
// reaches device memory and T is written once.
#include "fused_body.h"

namespace dust {
namespace {

// Resident waves per SIMD: six (80 VGPRs) -- more tiles in flight keep the
// phases of different tiles overlapping.  Up to 128 grains the compiler
// spills only inside the exact fallback for out-of-table pairs, which tiles
// without such pairs branch over; measured 4 % faster than five, seven
// slower.  Above 128 grains (three or four grain tiles per wave, J in
// 64-wavelength chunks) a few heating values spill too, and six waves still
// measured 0.4-2.6 % faster than five.
// TAIL: the emission's odd last grain group is its own step (grids whose
// grain count leaves an odd number of 8-grain groups).
template <int MODE, int NTW, bool TAIL>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6, 8))) void fused_kernel(
    PlanView v, int64_t C,
                                                   const float* __restrict__ J, int64_t ldj,
                                                   const float* __restrict__ m,
                                                   float* __restrict__ T, int64_t ldt,
                                                   float* __restrict__ L, int64_t ldl,
                                                   dust_counters* cnt) {
    extern __shared__ float sTile[];
    fused_tile<MODE, FUSED_TC, NTW, TAIL, fused_kc(NTW)>(v, (int64_t)blockIdx.x * FUSED_TC, C, J, ldj, m, T, ldt, L,
                                          ldl, cnt, sTile);
}

// Absorb + solve only (the first of the two-kernel form): T is written once
// and the emission kernel follows.
template <int MODE, int NTW>
__global__ __launch_bounds__(256) void absorb_solve_kernel(PlanView v, int64_t C,
                                                          const float* __restrict__ J,
                                                          int64_t ldj, float* __restrict__ T,
                                                          int64_t ldt, dust_counters* cnt) {
    extern __shared__ float lds[];  // sH [16][Sp], J staging, pending list
    char* sStage = reinterpret_cast<char*>(lds + FUSED_TC * v.Sp);
    const int64_t c0 = (int64_t)blockIdx.x * FUSED_TC;
    fused_absorb<MODE, NTW>(v, c0, C, J, ldj, lds, sStage);
    __syncthreads();
    fused_solve<MODE, FUSED_TC>(v, c0, C, T, ldt, cnt, lds,
                                reinterpret_cast<int*>(sStage + STAGE_BYTES));
}

template <int NTW>
hipError_t launch_as_ntw(const PlanView& v, int64_t C, const float* J, int64_t ldj, float* T,
                         int64_t ldt, dust_counters* cnt, hipStream_t st) {
    const size_t lds = sizeof(float) * FUSED_TC * v.Sp + STAGE_BYTES + SOLVE_LDS_BYTES;
    const dim3 grid((unsigned)((C + FUSED_TC - 1) / FUSED_TC));
    const int km = kernel_mode(v);
    if (km == DUST_MIXED)
        hipLaunchKernelGGL((absorb_solve_kernel<DUST_MIXED, NTW>), grid, dim3(256), lds, st, v,
                           C, J, ldj, T, ldt, cnt);
    else if (km == MODE_MIXED_F32)
        hipLaunchKernelGGL((absorb_solve_kernel<MODE_MIXED_F32, NTW>), grid, dim3(256), lds,
                           st, v, C, J, ldj, T, ldt, cnt);
    else if (km == MODE_MIXED_POLISH)
        hipLaunchKernelGGL((absorb_solve_kernel<MODE_MIXED_POLISH, NTW>), grid, dim3(256), lds,
                           st, v, C, J, ldj, T, ldt, cnt);
    else if (v.mode == DUST_TABLE_LINEAR)
        hipLaunchKernelGGL((absorb_solve_kernel<DUST_TABLE_LINEAR, NTW>), grid, dim3(256), lds,
                           st, v, C, J, ldj, T, ldt, cnt);
    else
        hipLaunchKernelGGL((absorb_solve_kernel<DUST_PLAIN_FP32, NTW>), grid, dim3(256), lds, st,
                           v, C, J, ldj, T, ldt, cnt);
    return hipGetLastError();
}

template <int NTW, bool TAIL>
hipError_t launch_ntw(const PlanView& v, int64_t C, const float* J, int64_t ldj, const float* m,
                      float* T, int64_t ldt, float* L, int64_t ldl, dust_counters* cnt,
                      hipStream_t st) {
    const size_t lds = fused_lds_bytes(FUSED_TC, v.Sp, Stage<fused_kc(NTW)>::BYTES);
    const dim3 grid((unsigned)((C + FUSED_TC - 1) / FUSED_TC));
    const int km = kernel_mode(v);
    if (km == DUST_MIXED)
        hipLaunchKernelGGL((fused_kernel<DUST_MIXED, NTW, TAIL>), grid, dim3(256), lds, st, v, C,
                           J, ldj, m, T, ldt, L, ldl, cnt);
    else if (km == MODE_MIXED_F32)
        hipLaunchKernelGGL((fused_kernel<MODE_MIXED_F32, NTW, TAIL>), grid, dim3(256), lds, st,
                           v, C, J, ldj, m, T, ldt, L, ldl, cnt);
    else if (km == MODE_MIXED_POLISH)
        hipLaunchKernelGGL((fused_kernel<MODE_MIXED_POLISH, NTW, TAIL>), grid, dim3(256), lds,
                           st, v, C, J, ldj, m, T, ldt, L, ldl, cnt);
    else if (v.mode == DUST_TABLE_LINEAR)
        hipLaunchKernelGGL((fused_kernel<DUST_TABLE_LINEAR, NTW, TAIL>), grid, dim3(256), lds,
                           st, v, C, J, ldj, m, T, ldt, L, ldl, cnt);
    else
        hipLaunchKernelGGL((fused_kernel<DUST_PLAIN_FP32, NTW, TAIL>), grid, dim3(256), lds, st,
                           v, C, J, ldj, m, T, ldt, L, ldl, cnt);
    return hipGetLastError();
}

template <bool TAIL>
hipError_t launch_fused_as(const PlanView& v, int64_t C, const float* J, int64_t ldj,
                           const float* m, float* T, int64_t ldt, float* L, int64_t ldl,
                           dust_counters* cnt, hipStream_t st) {
    const int ntw = (v.Sp / 16 + 3) / 4;  // grain tiles per wave in one pass
    if (ntw <= 1) return launch_ntw<1, TAIL>(v, C, J, ldj, m, T, ldt, L, ldl, cnt, st);
    if (ntw <= 2) return launch_ntw<2, TAIL>(v, C, J, ldj, m, T, ldt, L, ldl, cnt, st);
    if (ntw <= 3) return launch_ntw<3, TAIL>(v, C, J, ldj, m, T, ldt, L, ldl, cnt, st);
    return launch_ntw<4, TAIL>(v, C, J, ldj, m, T, ldt, L, ldl, cnt, st);  // 4: several passes above
}

}  // namespace

hipError_t launch_fused(const PlanView& v, int64_t C, const float* J, int64_t ldj, const float* m,
                        float* T, int64_t ldt, float* L, int64_t ldl, dust_counters* cnt,
                        hipStream_t st) {
    if (C == 0) return hipSuccess;
    if (((v.S + EMIT_GROUP - 1) / EMIT_GROUP) & 1)
        return launch_fused_as<true>(v, C, J, ldj, m, T, ldt, L, ldl, cnt, st);
    return launch_fused_as<false>(v, C, J, ldj, m, T, ldt, L, ldl, cnt, st);
}

hipError_t launch_absorb_solve(const PlanView& v, int64_t C, const float* J, int64_t ldj,
                               float* T, int64_t ldt, dust_counters* cnt, hipStream_t st) {
    if (C == 0) return hipSuccess;
    const int ntw = (v.Sp / 16 + 3) / 4;
    if (ntw <= 1) return launch_as_ntw<1>(v, C, J, ldj, T, ldt, cnt, st);
    if (ntw <= 2) return launch_as_ntw<2>(v, C, J, ldj, T, ldt, cnt, st);
    if (ntw <= 3) return launch_as_ntw<3>(v, C, J, ldj, T, ldt, cnt, st);
    if (ntw <= 4) return launch_as_ntw<4>(v, C, J, ldj, T, ldt, cnt, st);
    return launch_as_ntw<4>(v, C, J, ldj, T, ldt, cnt, st);  // several passes
}

}  // namespace dust
