// Cell SED, Eqs. 9-10 (Section 4.4):
//   L[c,l] = m[c] sum_s w_s C[s,l] B(lam_l, T[c,s]).
// A workgroup owns TC cells and 256 consecutive wavelengths; each lane owns
// one wavelength (coalesced L stores) and TC accumulators.  The tile's 1/T
// sits in LDS and is read with wave-uniform addresses (broadcast); the
// emission weights em[s,l] are read once per grain and reused for TC cells.
// Per term: one multiply, v_exp_f32, one subtract, v_rcp_f32, one multiply,
// one FMA.
#include "device_common.h"

namespace dust {
namespace {

constexpr int EMIT_TC = 16;

template <int TC>
__global__ __launch_bounds__(256) void emit_kernel(PlanView v, int64_t C,
                                                   const float* __restrict__ T, int64_t ldt,
                                                   const float* __restrict__ m,
                                                   float* __restrict__ L, int64_t ldl) {
    extern __shared__ float smem[];  // sInvT [TC][Sp], then sChunk [Sp/4][TC]
    float* sInvT = smem;
    uint32_t* sChunk = reinterpret_cast<uint32_t*>(smem + TC * v.Sp);
    const int64_t c0 = (int64_t)blockIdx.x * TC;
    for (int i = threadIdx.x; i < TC * v.Sp; i += 256) {
        const int cc = i / v.Sp, s = i - cc * v.Sp;
        sInvT[i] = (c0 + cc < C && s < v.S) ? inv_temperature(T[(c0 + cc) * ldt + s])
                                             : __builtin_inff();
    }
    __syncthreads();
    fill_chunk_min<TC>(sInvT, sChunk, v.Sp);
    __syncthreads();
    // Grids of at most two 64-wavelength chunks (one column of blocks): the
    // four waves split the tile's cells as well.
    const int nch = (v.NL + 63) >> 6;
    if (nch <= 2) {
        if (nch == 2)
            emit_cell_part<TC / 2, TC>(v, c0, C, m, L, ldl, sInvT, sChunk, 2);
        else
            emit_cell_part<TC / 4, TC>(v, c0, C, m, L, ldl, sInvT, sChunk, 1);
        return;
    }
    const int lw0 = blockIdx.y * 256 + (threadIdx.x & ~63);
    const int l = blockIdx.y * 256 + threadIdx.x;
    const bool lv = l < v.NL;
    const float nu = v.nu[lv ? l : 0];
    float acc[TC];
    emit_accumulate<TC>(v.em + (lv ? l : 0), v.NLp, nu, wave_u_min(v.nu, lw0, v.NL), sInvT,
                        sChunk, v.Sp, v.S, acc);
    if (!lv) return;
#pragma unroll
    for (int cc = 0; cc < TC; ++cc) {
        const int64_t c = c0 + cc;
        if (c < C) L[c * ldl + l] = acc[cc] * ((m ? m[c] : 1.0f) * v.escale);
    }
}

}  // namespace

hipError_t launch_emit(const PlanView& v, int64_t C, const float* T, int64_t ldt,
                       const float* m, float* L, int64_t ldl, hipStream_t st) {
    if (C == 0) return hipSuccess;
    dim3 grid((unsigned)((C + EMIT_TC - 1) / EMIT_TC), (unsigned)((v.NL + 255) / 256));
    const size_t lds = emit_lds_bytes(EMIT_TC, v.Sp);
    hipLaunchKernelGGL(emit_kernel<EMIT_TC>, grid, dim3(256), lds, st, v, C, T, ldt, m, L, ldl);
    return hipGetLastError();
}

}  // namespace dust
