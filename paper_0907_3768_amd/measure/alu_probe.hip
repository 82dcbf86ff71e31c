// Throughput probes of the vector ALU forms (see alu_probe.h): each thread
// runs `iters` iterations of 8 independent chains and writes one float (its
// chains' sum) to out[thread].
#include <hip/hip_runtime.h>

#include "alu_probe.h"

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
            if constexpr (KIND == ALU_PROBE_EXP2) {
                x[i] = __builtin_amdgcn_exp2f(-x[i]);
            } else if constexpr (KIND == ALU_PROBE_RCP) {
                x[i] = __builtin_amdgcn_rcpf(x[i] + 1.0f);
            } else if constexpr (KIND == ALU_PROBE_FMA) {
                x[i] = fmaf(x[i], 0.5f, 0.25f);
            } else if constexpr (KIND == ALU_PROBE_EXP2_FMA) {
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

// FP64 FMA chains (same shape as the FP32 ones)
__global__ __launch_bounds__(256) void probe_fma64_kernel(float* __restrict__ out, int iters) {
    const int gid = blockIdx.x * 256 + threadIdx.x;
    double x[PROBE_CHAINS];
#pragma unroll
    for (int i = 0; i < PROBE_CHAINS; ++i) x[i] = 0.3 + 0.01 * i + 1e-7 * (double)(gid & 1023);
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int i = 0; i < PROBE_CHAINS; ++i) x[i] = fma(x[i], 0.5, 0.25);
    }
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < PROBE_CHAINS; ++i) s += x[i];
    out[gid] = (float)s;
}

template <int KIND>
void launch(int blocks, int iters, float* out, hipStream_t st) {
    if constexpr (KIND == ALU_PROBE_FMA64)
        hipLaunchKernelGGL(probe_fma64_kernel, dim3(blocks), dim3(256), 0, st, out, iters);
    else
        hipLaunchKernelGGL(probe_kernel<KIND>, dim3(blocks), dim3(256), 0, st, out, iters);
}

}  // namespace

extern "C" int alu_probe_run(int32_t kind, int32_t blocks, int32_t iters, float* out,
                             void* stream) {
    if (blocks < 1 || blocks > (1 << 20) || iters < 1 || iters > (1 << 20) || !out) return -1;
    const hipStream_t st = (hipStream_t)stream;
    switch (kind) {
        case ALU_PROBE_EXP2: launch<ALU_PROBE_EXP2>(blocks, iters, out, st); break;
        case ALU_PROBE_RCP: launch<ALU_PROBE_RCP>(blocks, iters, out, st); break;
        case ALU_PROBE_FMA: launch<ALU_PROBE_FMA>(blocks, iters, out, st); break;
        case ALU_PROBE_EXP2_FMA: launch<ALU_PROBE_EXP2_FMA>(blocks, iters, out, st); break;
        case ALU_PROBE_TERM: launch<ALU_PROBE_TERM>(blocks, iters, out, st); break;
        case ALU_PROBE_FMA64: launch<ALU_PROBE_FMA64>(blocks, iters, out, st); break;
        default: return -1;
    }
    return hipGetLastError() == hipSuccess ? 0 : -4;
}
