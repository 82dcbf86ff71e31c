// Throughput probes of the vector ALU forms the emission and the solve are
// built from, so that the ALU peak the benchmark divides by can be checked
// on the device: each thread runs `iters` iterations of 8 independent chains
// and writes one float (its chains' sum) to out[thread].
#include "internal.h"

namespace dust {
namespace {

constexpr int PROBE_CHAINS = 8;

template <int KIND>
__global__ __launch_bounds__(256) void probe_kernel(float* __restrict__ out, int iters) {
    const int gid = blockIdx.x * 256 + threadIdx.x;
    float x[PROBE_CHAINS], y[PROBE_CHAINS];
#pragma unroll
    for (int i = 0; i < PROBE_CHAINS; ++i) {
        x[i] = 0.3f + 0.01f * i + 1e-7f * (float)(gid & 1023);
        y[i] = 0.5f - 0.01f * i;
    }
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int i = 0; i < PROBE_CHAINS; ++i) {
            if constexpr (KIND == DUST_PROBE_EXP2) {
                x[i] = __builtin_amdgcn_exp2f(-x[i]);
            } else if constexpr (KIND == DUST_PROBE_RCP) {
                x[i] = __builtin_amdgcn_rcpf(x[i] + 1.0f);
            } else if constexpr (KIND == DUST_PROBE_FMA) {
                x[i] = fmaf(x[i], 0.5f, 0.25f);
            } else if constexpr (KIND == DUST_PROBE_EXP2_FMA) {
                // an exponential and an independent FMA per chain step
                x[i] = __builtin_amdgcn_exp2f(-x[i]);
                y[i] = fmaf(y[i], 0.5f, 0.25f);
            } else {
                // the emission's exact term: mul, exp, sub, rcp, fma
                const float r = __builtin_amdgcn_rcpf(__builtin_amdgcn_exp2f(-(y[i] * x[i])) - 1.0f);
                x[i] = fmaf(0.5f, r, x[i]) * 0.5f;
            }
        }
    }
    float s = 0.0f;
#pragma unroll
    for (int i = 0; i < PROBE_CHAINS; ++i) s += x[i] + y[i];
    out[gid] = s;
}

}  // namespace
}  // namespace dust

extern "C" dust_status dust_probe_alu(int32_t kind, int32_t blocks, int32_t iters, float* out,
                                      void* stream) {
    using namespace dust;
    clear_error();
    if (blocks < 1 || blocks > (1 << 20)) return set_error(DUST_EINVAL, "blocks must be in [1, 2^20]");
    if (iters < 1 || iters > (1 << 20)) return set_error(DUST_EINVAL, "iters must be in [1, 2^20]");
    if (!out) return set_error(DUST_EINVAL, "out is NULL");
    const hipStream_t st = (hipStream_t)stream;
    switch (kind) {
        case DUST_PROBE_EXP2:
            hipLaunchKernelGGL(probe_kernel<DUST_PROBE_EXP2>, dim3(blocks), dim3(256), 0, st, out, iters);
            break;
        case DUST_PROBE_RCP:
            hipLaunchKernelGGL(probe_kernel<DUST_PROBE_RCP>, dim3(blocks), dim3(256), 0, st, out, iters);
            break;
        case DUST_PROBE_FMA:
            hipLaunchKernelGGL(probe_kernel<DUST_PROBE_FMA>, dim3(blocks), dim3(256), 0, st, out, iters);
            break;
        case DUST_PROBE_EXP2_FMA:
            hipLaunchKernelGGL(probe_kernel<DUST_PROBE_EXP2_FMA>, dim3(blocks), dim3(256), 0, st, out,
                               iters);
            break;
        case DUST_PROBE_TERM:
            hipLaunchKernelGGL(probe_kernel<DUST_PROBE_TERM>, dim3(blocks), dim3(256), 0, st, out, iters);
            break;
        default:
            return set_error(DUST_EINVAL, "unknown probe kind");
    }
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? DUST_OK : hip_error(e, "probe kernel");
}
