// Cell SED, Eqs. 9-10 (Section 4.4):
//   L[c,l] = m[c] sum_s w_s C[s,l] B(lam_l, T[c,s]).
// A workgroup owns TC cells and 256 consecutive wavelengths, in blocks of
// 32; a wave takes one block at a time, its lanes 32 wavelengths x 2 rows of
// grain groups, each lane 16 partial sums (emit_block), and the rows' sums
// are added across lanes before the store.  The tile's 1/T sits in LDS; the
// emission weights em[s,l] are read once per grain and reused for the
// tile's cells.  An exact term is one multiply, v_exp_f32, one subtract,
// v_rcp_f32 and one FMA.
#include "device_common.h"

namespace dust {
namespace {

constexpr int EMIT_TC = 16;

template <int TC, bool TAIL>
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
    // Workgroup column y owns the 256 wavelengths from 256y, in blocks of
    // LW; wave w takes the column's blocks w, w + 4, ....  Grids with fewer
    // than four blocks (one column) split the tile's cells over the waves.
    constexpr int LW = 64 / EMIT_ROWS, BPC = 256 / LW;
    const int NB = (v.NL + LW - 1) / LW;
    if (NB >= 4) {
        const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
        const int end = (int)blockIdx.y * BPC + BPC < NB ? (int)blockIdx.y * BPC + BPC : NB;
        emit_tile<EMIT_ROWS, TC, TAIL>(v, c0, C, m, L, ldl, sInvT, sChunk, (int)blockIdx.y * BPC + w,
                                 4, end);
    } else if (v.NL > 64) {
        emit_cell_part<TC / 2, TC>(v, c0, C, m, L, ldl, sInvT, sChunk, 2);
    } else {
        emit_cell_part<TC / 4, TC>(v, c0, C, m, L, ldl, sInvT, sChunk, 1);
    }
}

}  // namespace

hipError_t launch_emit(const PlanView& v, int64_t C, const float* T, int64_t ldt,
                       const float* m, float* L, int64_t ldl, hipStream_t st) {
    if (C == 0) return hipSuccess;
    dim3 grid((unsigned)((C + EMIT_TC - 1) / EMIT_TC), (unsigned)((v.NL + 255) / 256));
    const size_t lds = emit_lds_bytes(EMIT_TC, v.Sp);
    if (((v.S + EMIT_GROUP - 1) / EMIT_GROUP) & 1)
        hipLaunchKernelGGL((emit_kernel<EMIT_TC, true>), grid, dim3(256), lds, st, v, C, T, ldt, m,
                           L, ldl);
    else
        hipLaunchKernelGGL((emit_kernel<EMIT_TC, false>), grid, dim3(256), lds, st, v, C, T, ldt,
                           m, L, ldl);
    return hipGetLastError();
}

}  // namespace dust
