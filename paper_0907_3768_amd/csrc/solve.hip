// Temperature solve, Eq. 7 (Section 4.3).
//
// Plain FP32: a workgroup takes a tile of 64 cells x up to 16 grains.  The
// tile's heating (plus the extra term) is staged in LDS with coalesced
// loads; each wave then solves one grain at a time for the 64 cells (one
// cell per lane), as the paper's third kernel gives a block one species, so
// the grain's Planck weights and the wavelength table are wave-uniform and
// come through the scalar cache.  T goes back through the same LDS slots and
// leaves with coalesced stores; the Newton evaluations of the block are
// counted with one atomic.
// Mixed: four (cell, grain) pairs per thread, 256 apart in row-major order
// (coalesced H and T), each an O(1) lookup in the grain's inverse table
// ln T(ln H) (a cubic Hermite in FP64 between FP64 nodes, or in FP32 with the
// FP32 lookup), all four in flight together.
// Table-linear: the same layout, a bracketed search in the grain's table of
// powers at evenly spaced T and linear interpolation (Sections 2 and 5).
// Every form adds the optional extra heating Q to H first.
#include "device_common.h"

namespace dust {
namespace {

constexpr int PLAIN_CELLS = 64;    // cells per tile: one per lane
constexpr int PLAIN_GRAINS = 16;   // grains per tile at most

// LDS row stride of a tile of g grains: odd, so the 64 lanes reading one
// grain column hit distinct banks.
__host__ __device__ constexpr int plain_stride(int g) { return g | 1; }

__global__ __launch_bounds__(256) void solve_plain_kernel(PlanView v, int64_t C,
                                                          const float* __restrict__ H,
                                                          int64_t ldh, float* __restrict__ T,
                                                          int64_t ldt, dust_counters* cnt) {
    extern __shared__ float sX[];  // [64][ST]: heating in, T out
    __shared__ int sEvals[4];
    const int64_t c0 = (int64_t)blockIdx.x * PLAIN_CELLS;
    const int g0 = blockIdx.y * PLAIN_GRAINS;
    const int G = (v.S - g0 < PLAIN_GRAINS) ? v.S - g0 : PLAIN_GRAINS;
    const int ST = plain_stride(G);
    const int rows = (C - c0 < PLAIN_CELLS) ? (int)(C - c0) : PLAIN_CELLS;
    for (int i = threadIdx.x; i < rows * G; i += blockDim.x) {
        const int cc = i / G, sl = i - cc * G;
        const int64_t c = c0 + cc;
        float h = H[c * ldh + g0 + sl];
        if (v.q) h += v.q[c * v.ldq + g0 + sl];
        sX[cc * ST + sl] = h * v.hscale[g0 + sl];
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const bool live = lane < rows;
    int evals = 0;
    for (int sl = wave; sl < G; sl += 4) {
        const int s = g0 + sl;  // wave-uniform: the grain's weights come as scalars
        const float t0 = (live && v.warm) ? T[(c0 + lane) * ldt + s] : 0.0f;
        int ev;
        const float t = solve_newton_wave(v.kb + (int64_t)s * v.NLp, v.ku + (int64_t)s * v.NLp,
                                          v.nu, v.NL, live, live ? sX[lane * ST + sl] : 0.0f,
                                          v.gs[s], v.tol, v.maxit, t0, &ev, cnt);
        if (live) sX[lane * ST + sl] = t;
        evals += ev;
    }
    if (cnt) {
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) evals += __shfl_xor(evals, off, 64);
        if (lane == 0) sEvals[wave] = evals;
    }
    __syncthreads();
    if (cnt && threadIdx.x == 0) {
        const int n = sEvals[0] + sEvals[1] + sEvals[2] + sEvals[3];
        if (n) atomicAdd(reinterpret_cast<unsigned long long*>(&cnt->n_newton_evals),
                         (unsigned long long)n);
    }
    for (int i = threadIdx.x; i < rows * G; i += blockDim.x) {
        const int cc = i / G, sl = i - cc * G;
        T[(c0 + cc) * ldt + g0 + sl] = sX[cc * ST + sl];
    }
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

// Mixed: each thread takes MIXED_PER pairs 256 apart in row-major order
// (coalesced H and T) and looks all of them up before it stores any, so that
// their dependent loads (H, then the grain's inverse-table nodes) overlap: a
// single lookup per thread leaves the kernel waiting on memory latency.  Pairs
// outside the table go to an LDS list and are then solved exactly by the
// block's waves in turn (one pair per wave at a time, lanes over wavelength).
constexpr int MIXED_PER = 4;
constexpr int MIXED_BLOCK = 256 * MIXED_PER;  // pairs per workgroup

template <int MODE>
__device__ __forceinline__ int lookup_status(const PlanView& v, int s, float hs, float* T,
                                             bool active, dust_counters* cnt) {
    if constexpr (MODE == MODE_MIXED_POLISH) {
        if (!active) return LOOKUP_OK;
        return table_lookup_polish(v, s, hs, T, cnt) != 0 ? LOOKUP_PENDING : LOOKUP_OK;
    } else if constexpr (MODE == MODE_MIXED_F32) {
        return table_lookup_f32_nb(v, s, hs, T);
    } else {
        return table_lookup_f64_nb(v, s, hs, T);
    }
}

template <int MODE>
__global__ __launch_bounds__(256) void solve_mixed_kernel(PlanView v, int64_t C,
                                                          const float* __restrict__ H,
                                                          int64_t ldh, float* __restrict__ T,
                                                          int64_t ldt, dust_counters* cnt) {
    __shared__ int sCount;
    __shared__ int sList[MIXED_BLOCK];
    if (threadIdx.x == 0) sCount = 0;
    __syncthreads();
    const int64_t n = C * v.S;
    const int64_t base = (int64_t)blockIdx.x * MIXED_BLOCK + threadIdx.x;
    int64_t c[MIXED_PER];
    int s[MIXED_PER];
    float hs[MIXED_PER];
#pragma unroll
    for (int k = 0; k < MIXED_PER; ++k) {
        // past the end, read the last pair again (nothing is stored for it)
        const int64_t i = (base + k * 256 < n) ? base + k * 256 : n - 1;
        c[k] = i / v.S;
        s[k] = (int)(i - c[k] * v.S);
        float h = H[c[k] * ldh + s[k]];
        if (v.q) h += v.q[c[k] * v.ldq + s[k]];
        hs[k] = h * v.hscale[s[k]];
    }
    float t[MIXED_PER];
    int st[MIXED_PER];
#pragma unroll
    for (int k = 0; k < MIXED_PER; ++k)
        st[k] = lookup_status<MODE>(v, s[k], hs[k], &t[k], base + k * 256 < n, cnt);
    int nonfinite = 0;
#pragma unroll
    for (int k = 0; k < MIXED_PER; ++k) {
        if (base + k * 256 >= n) continue;
        if (st[k] == LOOKUP_PENDING) {
            sList[atomicAdd(&sCount, 1)] = threadIdx.x + k * 256;
        } else {
            nonfinite += st[k] == LOOKUP_NONFINITE;
            T[c[k] * ldt + s[k]] = t[k];
        }
    }
    if (cnt) wave_count_add(&cnt->n_nonfinite, nonfinite);
    __syncthreads();
    const int np = sCount;
    for (int e = threadIdx.x >> 6; e < np; e += blockDim.x >> 6) {
        const int64_t ip = (int64_t)blockIdx.x * MIXED_BLOCK + sList[e];
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
        const unsigned blocks = (unsigned)((n + MIXED_BLOCK - 1) / MIXED_BLOCK);
        if (v.f32_lookup)
            hipLaunchKernelGGL(solve_mixed_kernel<MODE_MIXED_F32>,
                               dim3(blocks), dim3(256), 0, st, v, C, H, ldh, T, ldt, cnt);
        else if (v.polish)
            hipLaunchKernelGGL(solve_mixed_kernel<MODE_MIXED_POLISH>, dim3(blocks), dim3(256), 0,
                               st, v, C, H, ldh, T, ldt, cnt);
        else
            hipLaunchKernelGGL(solve_mixed_kernel<DUST_MIXED>, dim3(blocks), dim3(256), 0, st, v,
                               C, H, ldh, T, ldt, cnt);
    } else if (v.mode == DUST_TABLE_LINEAR) {
        const int64_t n = C * v.S;
        hipLaunchKernelGGL(solve_table_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                           st, v, C, H, ldh, T, ldt, cnt);
    } else {
        const int gt = (v.S + PLAIN_GRAINS - 1) / PLAIN_GRAINS;
        const int G = v.S < PLAIN_GRAINS ? v.S : PLAIN_GRAINS;
        const size_t lds = sizeof(float) * PLAIN_CELLS * plain_stride(G);
        hipLaunchKernelGGL(solve_plain_kernel,
                           dim3((unsigned)((C + PLAIN_CELLS - 1) / PLAIN_CELLS), gt), dim3(256),
                           lds, st, v, C, H, ldh, T, ldt, cnt);
    }
    return hipGetLastError();
}

}  // namespace dust
