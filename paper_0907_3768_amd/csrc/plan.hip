// Plan-time kernels: the derived tables of a grid.
//
//  prep  (the paper's first kernel, Section 4.1): K = C dlam per grain and
//        wavelength, scaled per grain by an exact power of two, in FP32 and as
//        a bf16 hi+lo pair (both in MFMA fragment order); the solve weights K' c1 lam^-5; the emission
//        weights w C c1 lam^-5 (Eq. 10 without the mass); the wavelength
//        exponent table nu = -c2 log2(e) / lam.
//  ltab  (mixed mode): per grain, y_k = ln P'(T_k) at log-spaced T_k, in
//        FP64, with P'(T) = sum_l K'_l B(lam_l, T) the right side of Eq. 7 in
//        the plan's scaled units -- as an FP64 matrix product of the grains'
//        Planck weights with the Planck factors of the table temperatures.
//  inv   (mixed mode): the inverse function ln T(y) and its derivative at
//        uniform steps of y, from Newton in FP64 on the forward table's
//        piecewise cubic, stored as FP32 pairs of nodes (one 16-byte load
//        per lookup).
//  table-linear mode: the same matrix product gives P'(T_k) itself at evenly
//        spaced T_k (the production table of Sections 2 and 5); kidx gives,
//        at uniform steps of ln P', the last table point below, so that a
//        lookup searches only a few points.
#include "device_common.h"

namespace dust {
namespace {

__global__ __launch_bounds__(256) void prep_kernel(PlanView v, const double* __restrict__ lam,
                                                   const double* __restrict__ dlam,
                                                   const double* __restrict__ cabs,
                                                   const double* __restrict__ w,
                                                   const int* __restrict__ es, int ge,
                                                   float* nu, float* kf, __bf16* khi,
                                                   __bf16* klo, float* kb, float* ku, float* em,
                                                   double* kdb, double* c2l) {
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    const int s = blockIdx.y;
    if (l >= v.NLp) return;
    const int64_t o = (int64_t)s * v.NLp + l;
    // The heating weights are stored in MFMA fragment order, so that one
    // wave's fragment of one grain tile and k-step is a contiguous 1 KB.
    const int64_t ob = kfrag_bf16(v, s, l), of = kfrag_f32(v, s, l);
    if (s == 0) {
        nu[l] = (l < v.NL) ? (float)(-RAD_C2 * LOG2E / lam[l]) : -1.0f;
        if (l < v.NL) c2l[l] = RAD_C2 / lam[l];
    }
    if (s < v.S && l < v.NL) {
        const double C = cabs[(int64_t)s * v.NL + l];
        const double K = ldexp(C * dlam[l], es[s]);
        const double lm = lam[l];
        const double c1l5 = RAD_C1 / (lm * lm * lm * lm * lm);
        const float kff = (float)K;
        const __bf16 hi = (__bf16)kff;
        const __bf16 lo = (__bf16)(float)(K - (double)(float)hi);
        kf[of] = kff;
        khi[ob] = hi;
        klo[ob] = lo;
        kb[o] = (float)(K * c1l5);
        ku[o] = (float)(K * c1l5 * (RAD_C2 * LOG2E / lm));
        em[o] = (float)ldexp(w[s] * C * c1l5, -ge);
        kdb[(int64_t)s * v.NL + l] = K * c1l5;
    } else {
        kf[of] = 0.0f;
        khi[ob] = (__bf16)0.0f;
        klo[ob] = (__bf16)0.0f;
        kb[o] = 0.0f;
        ku[o] = 0.0f;
        em[o] = 0.0f;
    }
}

// The table is a matrix product:  P'[s,k] = sum_l W[s,l] F[k,l]  with
// W = K' c1 lam^-5 (per grain) and F[k,l] = 1 / (exp(c2 / (lam_l T_k)) - 1)
// (per table temperature, the same for every grain).  F takes N x NL
// exponentials once; the product is FP64 FMA work.

// F[k][l], one thread per element.
__global__ __launch_bounds__(256) void planck_factor_kernel(PlanView v, double* F) {
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    const int k = blockIdx.y;
    if (l >= v.NL) return;
    const double invT = (v.mode == DUST_TABLE_LINEAR) ? 1.0 / v.texp[k]
                                                      : exp(-(v.lnTmin + k * v.hstep));
    F[(int64_t)k * v.NL + l] = 1.0 / expm1_pos(v.c2l[l] * invT);  // 0 once e^x overflows
}

// y[s][k] = ln sum_l W[s][l] F[k][l] (table-linear: the sum itself): FP64
// GEMM on the matrix cores (v_mfma_f64_16x16x4_f64).  Each wave computes a
// 16-grain x 16-point block; a workgroup's four waves take four consecutive
// point blocks.  Lane (row = lane mod 16, q = lane / 16) supplies, for every
// 32-wavelength step, wavelengths l0 + 8 q .. l0 + 8 q + 7 to both operands
// (grain row of W, point row of F) -- contiguous 64-byte loads; MFMA t takes
// the t-th of them (any assignment of wavelengths to k-slots gives the same
// sum when both operands use it).  Element j of the accumulator of lane
// (col, q) holds row q + 4 j of column col (the FP64 form interleaves rows).
__global__ __launch_bounds__(256) void ltab_gemm_kernel(PlanView v, const double* __restrict__ F,
                                                        double* fwd) {
    typedef double f64x4 __attribute__((ext_vector_type(4)));
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int row = lane & 15, q = lane >> 4;
    const int s0 = blockIdx.y * 16;
    const int k0 = (blockIdx.x * 4 + wave) * 16;
    const int s = s0 + row, k = k0 + row;
    const double* wr = v.kdb + (int64_t)(s < v.S ? s : 0) * v.NL;
    const double* fr = F + (int64_t)(k < v.N ? k : 0) * v.NL;
    const bool s_ok = s < v.S, k_ok = k < v.N;
    f64x4 acc = {0.0, 0.0, 0.0, 0.0};
    for (int l0 = 0; l0 < v.NL; l0 += 32) {
        double a[8], b[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const int l = l0 + 8 * q + t;
            a[t] = (s_ok && l < v.NL) ? wr[l] : 0.0;
            b[t] = (k_ok && l < v.NL) ? fr[l] : 0.0;
        }
#pragma unroll
        for (int t = 0; t < 8; ++t) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[t], b[t], acc, 0, 0, 0);
    }
    const int kc = k0 + row;  // column of this lane's accumulator
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int sr = s0 + q + 4 * j;
        if (sr < v.S && kc < v.N)
            fwd[(int64_t)sr * v.N + kc] = (v.mode == DUST_TABLE_LINEAR) ? acc[j] : log(acc[j]);
    }
}

// Table-linear: one thread per (grain, node); node j sits at
// ln P' = ylo + j (yhi - ylo) / (M - 1) and kidx[s][j] is the largest k in
// [0, N-2] with ln P'_k <= that value (0 if none).
__global__ __launch_bounds__(256) void kidx_kernel(PlanView v, const double* __restrict__ fwd,
                                                   int* kidx, double* ylo, double* yhi,
                                                   double* dyinv) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int s = blockIdx.y;
    if (j >= v.M) return;
    const int N = v.N;
    const double* P = fwd + (int64_t)s * N;
    const double y0 = log(P[0]), y1 = log(P[N - 1]);
    const double dinv = (v.M - 1) / (y1 - y0);
    if (j == 0) {
        ylo[s] = y0;
        yhi[s] = y1;
        dyinv[s] = dinv;
    }
    const double yj = (j == v.M - 1) ? y1 : y0 + j / dinv;
    int lo = 0, hi = N - 2;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (log(P[mid]) <= yj) lo = mid; else hi = mid - 1;
    }
    kidx[(int64_t)s * v.M + j] = lo;
}

// One thread per (grain, inverse node): ln T at y_j = ylo + j dy, by Newton
// on the forward table's cubic, and dy * d ln T / dy there.
__global__ __launch_bounds__(256) void inv_kernel(PlanView v, const double* __restrict__ fwd,
                                                  double* ylo, double* yhi,
                                                  double* dyinv, float2* invf, float* ylof,
                                                  float* dyinvf) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int s = blockIdx.y;
    if (j >= v.M) return;
    const int N = v.N;
    const double* f = fwd + (int64_t)s * N;
    const double y0 = f[0], y1 = f[N - 1];
    const double dinv = (v.M - 1) / (y1 - y0);
    if (j == 0) {
        ylo[s] = y0;
        yhi[s] = y1;
        dyinv[s] = dinv;
        ylof[s] = (float)y0;
        dyinvf[s] = (float)dinv;
    }
    const double yj = (j == v.M - 1) ? y1 : y0 + j / dinv;
    // largest k in [0, N-2] with y_k <= yj
    int lo = 0, hi = N - 2;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (f[mid] <= yj) lo = mid; else hi = mid - 1;
    }
    const int j0 = stencil_start(lo, N);
    const double a0 = f[j0], a1 = f[j0 + 1], a2 = f[j0 + 2], a3 = f[j0 + 3];
    double x = lo - j0 + ((f[lo + 1] > f[lo]) ? (yj - f[lo]) / (f[lo + 1] - f[lo]) : 0.0);
    double dp = 1.0;
    for (int it = 0; it < 4; ++it) {
        const double p = cubic4(x, a0, a1, a2, a3, &dp);
        x -= (p - yj) / dp;
    }
    cubic4(x, a0, a1, a2, a3, &dp);
    // d lnT / dy = hstep / (dy/dx), scaled by the node spacing dy = 1/dinv
    const double lnTj = v.lnTmin + ((double)j0 + x) * v.hstep;
    const double mj = v.hstep / dp / dinv;
    // the FP32 entries of the two intervals this node bounds
    const float2 nf = make_float2((float)lnTj, (float)mj);
    float2* row = invf + (int64_t)s * (v.M - 1) * 2;
    if (j < v.M - 1) row[2 * j] = nf;
    if (j > 0) row[2 * (j - 1) + 1] = nf;
}

}  // namespace

hipError_t launch_prepare(const dust_plan* p, hipStream_t st) {
    const PlanView& v = p->view;
    dim3 g1((v.NLp + 255) / 256, v.Sp);
    hipLaunchKernelGGL(prep_kernel, g1, dim3(256), 0, st, v, p->d_lam, p->d_dlam, p->d_cabs,
                       p->d_w, p->d_es, p->ge, p->d_nu, p->d_kf, p->d_khi, p->d_klo, p->d_kb, p->d_ku,
                       p->d_em, p->d_kdb, p->d_c2l);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !table_mode(v.mode)) return e;
    dim3 gf((v.NL + 255) / 256, v.N);
    hipLaunchKernelGGL(planck_factor_kernel, gf, dim3(256), 0, st, v, p->d_F);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    dim3 g2((v.N + 63) / 64, (v.S + 15) / 16);
    hipLaunchKernelGGL(ltab_gemm_kernel, g2, dim3(256), 0, st, v, (const double*)p->d_F, p->d_fwd);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    dim3 g3((v.M + 255) / 256, v.S);
    if (v.mode == DUST_TABLE_LINEAR) {
        hipLaunchKernelGGL(kidx_kernel, g3, dim3(256), 0, st, v, (const double*)p->d_fwd,
                           p->d_kidx, p->d_ylo, p->d_yhi, p->d_dyinv);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(inv_kernel, g3, dim3(256), 0, st, v, (const double*)p->d_fwd,
                       p->d_ylo, p->d_yhi, p->d_dyinv, reinterpret_cast<float2*>(p->d_invf),
                       p->d_ylof, p->d_dyinvf);
    return hipGetLastError();
}

}  // namespace dust
