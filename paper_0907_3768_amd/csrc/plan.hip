// Plan-time kernels: the derived tables of a grid.
//
//  prep  (the paper's first kernel, Section 4.1): K = C dlam per grain and
//        wavelength, scaled per grain by an exact power of two, in FP32 and as
//        a bf16 hi+lo pair; the solve weights K' c1 lam^-5; the emission
//        weights w C c1 lam^-5 (Eq. 10 without the mass); the wavelength
//        exponent table nu = -c2 log2(e) / lam.
//  ltab  (mixed mode): per grain, y_k = ln P'(T_k) and d ln P'/d ln T at
//        log-spaced T_k, in FP64, with P'(T) = sum_l K'_l B(lam_l, T)
//        the right side of Eq. 7 in the plan's scaled units.
//  kidx  (mixed mode): for uniform steps of y, the table interval holding it,
//        so that a lookup needs no search.
#include "internal.h"

namespace dust {
namespace {

__global__ __launch_bounds__(256) void prep_kernel(PlanView v, const double* __restrict__ lam,
                                                   const double* __restrict__ dlam,
                                                   const double* __restrict__ cabs,
                                                   const double* __restrict__ w,
                                                   const int* __restrict__ es, int ge,
                                                   float* nu, float* kf, __bf16* khi,
                                                   __bf16* klo, float* kb, float* em,
                                                   double* kd) {
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    const int s = blockIdx.y;
    if (l >= v.NLp) return;
    const int64_t o = (int64_t)s * v.NLp + l;
    if (s == 0) nu[l] = (l < v.NL) ? (float)(-RAD_C2 * LOG2E / lam[l]) : -1.0f;
    if (s < v.S && l < v.NL) {
        const double C = cabs[(int64_t)s * v.NL + l];
        const double K = ldexp(C * dlam[l], es[s]);
        const double lm = lam[l];
        const double l5 = lm * lm * lm * lm * lm;
        const float kff = (float)K;
        const __bf16 hi = (__bf16)kff;
        const __bf16 lo = (__bf16)(float)(K - (double)(float)hi);
        kf[o] = kff;
        khi[o] = hi;
        klo[o] = lo;
        kb[o] = (float)(K * RAD_C1 / l5);
        em[o] = (float)ldexp(w[s] * C * RAD_C1 / l5, -ge);
        kd[(int64_t)s * v.NL + l] = K;
    } else {
        kf[o] = 0.0f;
        khi[o] = (__bf16)0.0f;
        klo[o] = (__bf16)0.0f;
        kb[o] = 0.0f;
        em[o] = 0.0f;
    }
}

__global__ __launch_bounds__(256) void ltab_kernel(PlanView v, const double* __restrict__ lam,
                                                   double* lty, double* ltd) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int s = blockIdx.y;
    if (k >= v.N) return;
    const double T = exp(v.lnTmin + k * v.hstep);
    const double* kd = v.kd + (int64_t)s * v.NL;
    double P = 0.0, D = 0.0;
    for (int l = 0; l < v.NL; ++l) {
        const double lm = lam[l];
        const double x = RAD_C2 / (lm * T);
        const double em1 = expm1(x);
        if (__builtin_isinf(em1)) continue;
        const double l2 = lm * lm;
        const double b = RAD_C1 / (l2 * l2 * lm) / em1;
        P += kd[l] * b;
        D += kd[l] * b * x * ((em1 + 1.0) / em1);
    }
    lty[(int64_t)s * v.N + k] = log(P);
    ltd[(int64_t)s * v.N + k] = D / P;
}

__global__ __launch_bounds__(256) void kidx_kernel(PlanView v, const double* __restrict__ lty,
                                                   uint16_t* kidx, double* ylo, double* yhi,
                                                   double* dyinv) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int s = blockIdx.y;
    if (j >= v.M) return;
    const double* ty = lty + (int64_t)s * v.N;
    const double y0 = ty[0], y1 = ty[v.N - 1];
    const double dinv = (v.M - 1) / (y1 - y0);
    if (j == 0) {
        ylo[s] = y0;
        yhi[s] = y1;
        dyinv[s] = dinv;
    }
    const double yj = y0 + j / dinv;
    // largest k in [0, N-2] with ty[k] <= yj
    int lo = 0, hi = v.N - 2;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (ty[mid] <= yj) lo = mid; else hi = mid - 1;
    }
    kidx[(int64_t)s * v.M + j] = (uint16_t)lo;
}

}  // namespace

hipError_t launch_prepare(const dust_plan* p, hipStream_t st) {
    const PlanView& v = p->view;
    dim3 g1((v.NLp + 255) / 256, v.Sp);
    hipLaunchKernelGGL(prep_kernel, g1, dim3(256), 0, st, v, p->d_lam, p->d_dlam, p->d_cabs,
                       p->d_w, p->d_es, p->ge, p->d_nu, p->d_kf, p->d_khi, p->d_klo, p->d_kb,
                       p->d_em, p->d_kd);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || v.mode != DUST_MIXED) return e;
    dim3 g2((v.N + 255) / 256, v.S);
    hipLaunchKernelGGL(ltab_kernel, g2, dim3(256), 0, st, v, p->d_lam, p->d_lty, p->d_ltd);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    dim3 g3((v.M + 255) / 256, v.S);
    hipLaunchKernelGGL(kidx_kernel, g3, dim3(256), 0, st, v, p->d_lty, p->d_kidx, p->d_ylo,
                       p->d_yhi, p->d_dyinv);
    return hipGetLastError();
}

}  // namespace dust
