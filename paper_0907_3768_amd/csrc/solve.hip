// Temperature solve, Eq. 7 (Section 4.3).
//
// Plain FP32: one thread per (cell, grain); a workgroup serves one grain
// over 256 cells, as in the paper, so the grain's Planck weights and the
// wavelength table are wave-uniform and come through the scalar cache.
// Mixed: one thread per (cell, grain) in row-major order (coalesced H and T),
// an O(1) lookup in the grain's FP64 table and an FP64 Newton polish.
// Table-linear: the same layout, a bracketed search in the grain's table of
// powers at evenly spaced T and linear interpolation (Sections 2 and 5).
// Every form adds the optional extra heating Q to H first.
#include "device_common.h"

namespace dust {
namespace {

__global__ __launch_bounds__(256) void solve_plain_kernel(PlanView v, int64_t C,
                                                          const float* __restrict__ H,
                                                          int64_t ldh, float* __restrict__ T,
                                                          int64_t ldt, dust_counters* cnt) {
    const int s = blockIdx.y;
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    int evals = 0;
    if (c < C) {
        float h = H[c * ldh + s];
        if (v.q) h += v.q[c * v.ldq + s];
        const float t0 = v.warm ? T[c * ldt + s] : 0.0f;
        T[c * ldt + s] = solve_newton_f32(v.kb + (int64_t)s * v.NLp, v.nu, v.NL,
                                          h * v.hscale[s], v.gs[s], v.tol, v.maxit, t0, &evals,
                                          cnt);
    }
    if (cnt) wave_count_add(&cnt->n_newton_evals, evals);
}

// Table-linear: one thread per (cell, grain) in row-major order.
__global__ __launch_bounds__(256) void solve_table_kernel(PlanView v, int64_t C,
                                                          const float* __restrict__ H,
                                                          int64_t ldh, float* __restrict__ T,
                                                          int64_t ldt, dust_counters* cnt) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= C * v.S) return;
    const int64_t c = i / v.S;
    const int s = (int)(i - c * v.S);
    float h = H[c * ldh + s];
    if (v.q) h += v.q[c * v.ldq + s];
    T[c * ldt + s] = table_linear_T(v, s, h * v.hscale[s], cnt);
}

// One thread per (cell, grain) in row-major order: coalesced H and T.  Pairs
// outside the table go to an LDS list and are then solved exactly by the
// block's waves in turn (one pair per wave at a time, lanes over wavelength).
__global__ __launch_bounds__(256) void solve_mixed_kernel(PlanView v, int64_t C,
                                                          const float* __restrict__ H,
                                                          int64_t ldh, float* __restrict__ T,
                                                          int64_t ldt, dust_counters* cnt) {
    __shared__ int sCount;
    __shared__ int sList[256];
    if (threadIdx.x == 0) sCount = 0;
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const bool active = i < C * v.S;
    const int64_t c = active ? i / v.S : 0;
    const int s = active ? (int)(i - c * v.S) : 0;
    float h = active ? H[c * ldh + s] : 0.0f;
    if (active && v.q) h += v.q[c * v.ldq + s];
    const double hs = (double)(h * v.hscale[s]);
    float t = 0.0f;
    double lnT0;
    if (active) {
        if (table_lookup_f64(v, s, hs, &t, &lnT0, cnt) != 0)
            sList[atomicAdd(&sCount, 1)] = threadIdx.x;
        else
            T[c * ldt + s] = t;
    }
    __syncthreads();
    const int n = sCount;
    for (int e = threadIdx.x >> 6; e < n; e += blockDim.x >> 6) {
        const int64_t ip = (int64_t)blockIdx.x * 256 + sList[e];
        const int64_t cp = ip / v.S;
        const int sp = (int)(ip - cp * v.S);
        float hf = H[cp * ldh + sp];
        if (v.q) hf += v.q[cp * v.ldq + sp];
        const double hp = (double)(hf * v.hscale[sp]);
        const float tp = wave_solve_pending(v, sp, hp, cnt);
        if ((threadIdx.x & 63) == 0) T[cp * ldt + sp] = tp;
    }
}

}  // namespace

hipError_t launch_solve(const PlanView& v, int64_t C, const float* H, int64_t ldh, float* T,
                        int64_t ldt, dust_counters* cnt, hipStream_t st) {
    if (C == 0) return hipSuccess;
    if (v.mode == DUST_MIXED) {
        const int64_t n = C * v.S;
        hipLaunchKernelGGL(solve_mixed_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                           st, v, C, H, ldh, T, ldt, cnt);
    } else if (v.mode == DUST_TABLE_LINEAR) {
        const int64_t n = C * v.S;
        hipLaunchKernelGGL(solve_table_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                           st, v, C, H, ldh, T, ldt, cnt);
    } else {
        hipLaunchKernelGGL(solve_plain_kernel, dim3((unsigned)((C + 255) / 256), v.S), dim3(256),
                           0, st, v, C, H, ldh, T, ldt, cnt);
    }
    return hipGetLastError();
}

}  // namespace dust
