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
//  inv   (mixed mode): the inverse function ln T(y) and its derivative at
//        uniform steps of y, from Newton on the cubic Hermite interpolant of
//        the forward table, so that a lookup starts next to its root.
#include "device_common.h"

namespace dust {
namespace {

__global__ __launch_bounds__(256) void prep_kernel(PlanView v, const double* __restrict__ lam,
                                                   const double* __restrict__ dlam,
                                                   const double* __restrict__ cabs,
                                                   const double* __restrict__ w,
                                                   const int* __restrict__ es, int ge,
                                                   float* nu, float* kf, __bf16* khi,
                                                   __bf16* klo, float* kb, float* em,
                                                   double* kdb, double* c2l) {
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    const int s = blockIdx.y;
    if (l >= v.NLp) return;
    const int64_t o = (int64_t)s * v.NLp + l;
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
        kf[o] = kff;
        khi[o] = hi;
        klo[o] = lo;
        kb[o] = (float)(K * c1l5);
        em[o] = (float)ldexp(w[s] * C * c1l5, -ge);
        kdb[(int64_t)s * v.NL + l] = K * c1l5;
    } else {
        kf[o] = 0.0f;
        khi[o] = (__bf16)0.0f;
        klo[o] = (__bf16)0.0f;
        kb[o] = 0.0f;
        em[o] = 0.0f;
    }
}

// One thread per (grain, table point).  Per term: one multiply, expm1, one
// division; B = c1 lam^-5 / (e^x - 1) and T dB/dT = B x e^x / (e^x - 1).
__global__ __launch_bounds__(256) void ltab_kernel(PlanView v, double2* fwd) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int s = blockIdx.y;
    if (k >= v.N) return;
    const double invT = exp(-(v.lnTmin + k * v.hstep));
    const double* kdb = v.kdb + (int64_t)s * v.NL;
    double P = 0.0, D = 0.0;
    for (int l = 0; l < v.NL; ++l) {
        const double x = v.c2l[l] * invT;
        const double r = 1.0 / expm1_pos(x);  // 0 once e^x overflows
        const double b = kdb[l] * r;
        P += b;
        D += b * x * (1.0 + r);
    }
    fwd[(int64_t)s * v.N + k] = make_double2(log(P), v.hstep * (D / P));
}

// One thread per (grain, inverse node): ln T at y_j = ylo + j dy.
__global__ __launch_bounds__(256) void inv_kernel(PlanView v, const double2* __restrict__ fwd,
                                                  double2* inv, double* ylo, double* yhi,
                                                  double* dyinv) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int s = blockIdx.y;
    if (j >= v.M) return;
    const double2* f = fwd + (int64_t)s * v.N;
    const double y0 = f[0].x, y1 = f[v.N - 1].x;
    const double dinv = (v.M - 1) / (y1 - y0);
    if (j == 0) {
        ylo[s] = y0;
        yhi[s] = y1;
        dyinv[s] = dinv;
    }
    const double yj = (j == v.M - 1) ? y1 : y0 + j / dinv;
    // largest k in [0, N-2] with y_k <= yj
    int lo = 0, hi = v.N - 2;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (f[mid].x <= yj) lo = mid; else hi = mid - 1;
    }
    const double2 a = f[lo], b = f[lo + 1];
    double th = (b.x > a.x) ? (yj - a.x) / (b.x - a.x) : 0.0;
    double dp = 1.0;
    for (int it = 0; it < 4; ++it) {
        const double t2 = th * th, t3 = t2 * th;
        const double p = (2.0 * t3 - 3.0 * t2 + 1.0) * a.x + (t3 - 2.0 * t2 + th) * a.y +
                         (3.0 * t2 - 2.0 * t3) * b.x + (t3 - t2) * b.y;
        dp = (6.0 * t2 - 6.0 * th) * a.x + (3.0 * t2 - 4.0 * th + 1.0) * a.y +
             (6.0 * th - 6.0 * t2) * b.x + (3.0 * t2 - 2.0 * th) * b.y;
        th -= (p - yj) / dp;
        th = th < 0.0 ? 0.0 : (th > 1.0 ? 1.0 : th);
    }
    // d lnT / dy = hstep / (dp/dth), scaled by the node spacing dy = 1/dinv
    inv[(int64_t)s * v.M + j] = make_double2(v.lnTmin + ((double)lo + th) * v.hstep,
                                             v.hstep / dp / dinv);
}

}  // namespace

hipError_t launch_prepare(const dust_plan* p, hipStream_t st) {
    const PlanView& v = p->view;
    dim3 g1((v.NLp + 255) / 256, v.Sp);
    hipLaunchKernelGGL(prep_kernel, g1, dim3(256), 0, st, v, p->d_lam, p->d_dlam, p->d_cabs,
                       p->d_w, p->d_es, p->ge, p->d_nu, p->d_kf, p->d_khi, p->d_klo, p->d_kb,
                       p->d_em, p->d_kdb, p->d_c2l);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || v.mode != DUST_MIXED) return e;
    dim3 g2((v.N + 255) / 256, v.S);
    hipLaunchKernelGGL(ltab_kernel, g2, dim3(256), 0, st, v, p->d_fwd);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    dim3 g3((v.M + 255) / 256, v.S);
    hipLaunchKernelGGL(inv_kernel, g3, dim3(256), 0, st, v, (const double2*)p->d_fwd, p->d_inv,
                       p->d_ylo, p->d_yhi, p->d_dyinv);
    return hipGetLastError();
}

}  // namespace dust
