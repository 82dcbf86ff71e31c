// Device building blocks shared by the solve, emit, fused and batched kernels.
#pragma once

#include "internal.h"

namespace dust {

// ---------------------------------------------------------------------------
// Planck factor in FP32.  With a = nu_l / T = -h c / (k lam_l T) log2(e),
// y = 2^a = exp(-h c / (k lam T)) and B(lam, T) = c1 lam^-5 y / (1 - y).
// Written in y (not e^{+x}) so that the deep Wien tail underflows to 0
// instead of producing inf * 0.  Costs one v_exp_f32 and one v_rcp_f32.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float planck_factor(float nu, float invT) {
    const float y = __builtin_amdgcn_exp2f(nu * invT);
    const float q = __builtin_amdgcn_rcpf(1.0f - y);
    return y * q;
}

// ---------------------------------------------------------------------------
// Eq. 11 initial guess (Section 4.3) in natural-log units of T, floored at
// 5 K.  hs is the scaled heating H' = H 2^es; gs folds log10(4 pi 2^-es)
// and the size terms alpha1 log a + alpha2 log^2 a.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float guess_lnT(float hs, float gs) {
    const float x = log10f(hs) + gs;
    const float lg = 1.86f + x * (0.189f + 3.41e-3f * x);
    const float lnT = lg * 2.302585093f;
    return fmaxf(lnT, 1.609437912f);  // ln 5
}

__device__ __forceinline__ void count(int64_t* field) {
    atomicAdd(reinterpret_cast<unsigned long long*>(field), 1ull);
}

// ---------------------------------------------------------------------------
// Plain FP32 solve of Eq. 7 for one pair (Section 4.3): Newton's method on
// ln P(T) = ln H in the variable ln T from the Eq. 11 guess, with a bracket
// safeguard.  Stops when |ln(P/H)| <= tol and then applies the Newton step
// already computed.  `kb` is the grain's row of K' c1 lam^-5 (stride 1);
// `nu` the wavelength table.  Returns T.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float solve_newton_f32(const float* __restrict__ kb,
                                                  const float* __restrict__ nu,
                                                  int NL, float hs, float gs,
                                                  float tol, int maxit,
                                                  dust_counters* cnt) {
    if (!(hs >= 0.0f) || __builtin_isinf(hs)) {
        if (cnt) count(&cnt->n_nonfinite);
        return __builtin_nanf("");
    }
    if (hs == 0.0f) return 0.0f;

    const float lnH = logf(hs);
    float lnT = guess_lnT(hs, gs);
    float lo = -INFINITY, hi = INFINITY;
    bool done = false;
    for (int it = 0; it < maxit; ++it) {
        const float invT = expf(-lnT);
        float p0 = 0.f, p1 = 0.f, d0 = 0.f, d1 = 0.f;
        int l = 0;
        for (; l + 1 < NL; l += 2) {
            {
                const float a = nu[l] * invT;
                const float y = __builtin_amdgcn_exp2f(a);
                const float q = __builtin_amdgcn_rcpf(1.0f - y);
                const float b = y * q;
                p0 = fmaf(kb[l], b, p0);
                d0 = fmaf(kb[l], b * q * a, d0);
            }
            {
                const float a = nu[l + 1] * invT;
                const float y = __builtin_amdgcn_exp2f(a);
                const float q = __builtin_amdgcn_rcpf(1.0f - y);
                const float b = y * q;
                p1 = fmaf(kb[l + 1], b, p1);
                d1 = fmaf(kb[l + 1], b * q * a, d1);
            }
        }
        if (l < NL) {
            const float a = nu[l] * invT;
            const float y = __builtin_amdgcn_exp2f(a);
            const float q = __builtin_amdgcn_rcpf(1.0f - y);
            const float b = y * q;
            p0 = fmaf(kb[l], b, p0);
            d0 = fmaf(kb[l], b * q * a, d0);
        }
        const float P = p0 + p1;
        const float D = d0 + d1;  // = -sum K' B x / (ln 2 (1 - e^-x))
        if (!(P > 0.0f)) {        // every term underflowed: T is far too low
            lo = lnT;
            lnT = (hi < INFINITY) ? 0.5f * (lo + hi) : lnT + 1.0f;
            continue;
        }
        const float r = logf(P) - lnH;           // ln(P / H)
        const float slope = -0.69314718f * D / P;  // d ln P / d ln T
        if (r < 0.0f) lo = lnT; else hi = lnT;
        float next = lnT - r / slope;
        if (fabsf(r) <= tol) {
            lnT = next;
            done = true;
            break;
        }
        if (!(next > lo && next < hi))
            next = (lo > -INFINITY && hi < INFINITY) ? 0.5f * (lo + hi)
                                                     : lnT - copysignf(1.0f, r);
        lnT = next;
    }
    if (!done && cnt) count(&cnt->n_unconverged);
    return expf(lnT);
}

// ---------------------------------------------------------------------------
// Exact FP64 solve of Eq. 7 for one pair, used by the mixed path when T lies
// outside the table: Newton on ln P = ln H in ln T with the bracket
// [lnlo, lnhi].  Rare, so it evaluates the sum directly.
// ---------------------------------------------------------------------------
__device__ inline double solve_exact_f64(const PlanView& v, int s, double hs,
                                         double lnlo, double lnhi, bool* ok) {
    const double* kd = v.kd + (int64_t)s * v.NL;
    const double lnH = log(hs);
    double lo = lnlo, hi = lnhi;
    double lnT = 0.5 * (lo + hi);
    for (int it = 0; it < 200; ++it) {
        const double T = exp(lnT);
        double P = 0.0, D = 0.0;
        for (int l = 0; l < v.NL; ++l) {
            const double lam = v.lamd[l];
            const double x = RAD_C2 / (lam * T);
            const double em1 = expm1(x);
            if (__builtin_isinf(em1)) continue;
            const double l2 = lam * lam;
            const double b = RAD_C1 / (l2 * l2 * lam) / em1;
            P += kd[l] * b;
            D += kd[l] * b * x * ((em1 + 1.0) / em1);
        }
        double next;
        if (!(P > 0.0)) {
            lo = lnT;
            next = 0.5 * (lo + hi);
        } else {
            const double r = log(P) - lnH;
            if (r < 0.0) lo = lnT; else hi = lnT;
            next = lnT - r * P / D;
            if (fabs(next - lnT) <= 1e-14) { *ok = true; return next; }
            if (!(next > lo && next < hi)) next = 0.5 * (lo + hi);
        }
        if (hi - lo <= 1e-14) { *ok = true; return 0.5 * (lo + hi); }
        lnT = next;
    }
    *ok = false;
    return lnT;
}

// ---------------------------------------------------------------------------
// Mixed solve of Eq. 7 for one pair from the FP64 table of y = ln P'(ln T):
// locate the table interval through the uniform-in-y index, then Newton in
// FP64 on the cubic Hermite interpolant of y(ln T) over that interval.
// Out-of-table pairs fall back to the exact FP64 solve.  Returns T.
// ---------------------------------------------------------------------------
__device__ inline float solve_table_f64(const PlanView& v, int s, double hs,
                                        dust_counters* cnt) {
    if (!(hs >= 0.0) || __builtin_isinf(hs)) {
        if (cnt) count(&cnt->n_nonfinite);
        return __builtin_nanf("");
    }
    if (hs == 0.0) return 0.0f;
    const double y = log(hs);
    const double ylo = v.ylo[s], yhi = v.yhi[s];
    const bool table_ok = __builtin_isfinite(ylo) && __builtin_isfinite(yhi);
    if (!table_ok || !(y >= ylo && y <= yhi)) {
        // Outside the table (or a grain whose power underflows at the table's
        // low end): exact FP64 solve on the matching side of the range.
        bool ok = false;
        const double lnTmax = v.lnTmin + (v.N - 1) * v.hstep;
        double lnT;
        if (table_ok && y < ylo)
            lnT = solve_exact_f64(v, s, hs, log(1e-3), v.lnTmin, &ok);
        else if (table_ok)
            lnT = solve_exact_f64(v, s, hs, lnTmax, log(1e7), &ok);
        else
            lnT = solve_exact_f64(v, s, hs, log(1e-3), log(1e7), &ok);
        if (cnt) {
            count(&cnt->n_out_of_table);
            if (!ok) count(&cnt->n_unconverged);
        }
        return (float)exp(lnT);
    }
    const int N = v.N, M = v.M;
    int j = (int)((y - ylo) * v.dyinv[s]);
    j = j < 0 ? 0 : (j > M - 1 ? M - 1 : j);
    int k = v.kidx[(int64_t)s * M + j];
    const double* ty = v.lty + (int64_t)s * N;
    const double* td = v.ltd + (int64_t)s * N;
    while (k < N - 2 && ty[k + 1] <= y) ++k;
    while (k > 0 && ty[k] > y) --k;
    const double y0 = ty[k], y1 = ty[k + 1];
    const double m0 = td[k] * v.hstep, m1 = td[k + 1] * v.hstep;
    double th = (y1 > y0) ? (y - y0) / (y1 - y0) : 0.0;
    for (int it = 0; it < 3; ++it) {
        const double t2 = th * th, t3 = t2 * th;
        const double p = (2.0 * t3 - 3.0 * t2 + 1.0) * y0 + (t3 - 2.0 * t2 + th) * m0 +
                         (3.0 * t2 - 2.0 * t3) * y1 + (t3 - t2) * m1;
        const double dp = (6.0 * t2 - 6.0 * th) * y0 + (3.0 * t2 - 4.0 * th + 1.0) * m0 +
                          (6.0 * th - 6.0 * t2) * y1 + (3.0 * t2 - 2.0 * th) * m1;
        th -= (p - y) / dp;
        th = th < 0.0 ? 0.0 : (th > 1.0 ? 1.0 : th);
    }
    return (float)exp(v.lnTmin + ((double)k + th) * v.hstep);
}

// ---------------------------------------------------------------------------
// Emission of TC cells at one wavelength (Eqs. 9-10, Section 4.4): the lane
// owns wavelength l and accumulates sum_s em[s,l] B-factor(nu_l / T[c,s])
// for each of its TC cells.  sInvT is the tile's 1/T in LDS, [TC][Sp]
// (wave-uniform addresses: broadcast reads).  em points at column l of the
// emission-weight table (stride NLp).
// ---------------------------------------------------------------------------
template <int TC>
__device__ __forceinline__ void emit_accumulate(const float* __restrict__ em, int NLp,
                                                float nu, const float* sInvT, int Sp,
                                                int S, float (&acc)[TC]) {
#pragma unroll
    for (int cc = 0; cc < TC; ++cc) acc[cc] = 0.0f;
    for (int s = 0; s < S; s += 4) {
        const float e0 = em[(int64_t)(s + 0) * NLp];
        const float e1 = em[(int64_t)(s + 1) * NLp];
        const float e2 = em[(int64_t)(s + 2) * NLp];
        const float e3 = em[(int64_t)(s + 3) * NLp];
#pragma unroll
        for (int cc = 0; cc < TC; ++cc) {
            const float4 it = *reinterpret_cast<const float4*>(sInvT + cc * Sp + s);
            float a = acc[cc];
            a = fmaf(e0, planck_factor(nu, it.x), a);
            a = fmaf(e1, planck_factor(nu, it.y), a);
            a = fmaf(e2, planck_factor(nu, it.z), a);
            a = fmaf(e3, planck_factor(nu, it.w), a);
            acc[cc] = a;
        }
    }
}

}  // namespace dust
