// Device building blocks shared by the solve, emit, fused and batched kernels.
#pragma once

#include "internal.h"

namespace dust {

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

// Adds the sum of `n` over the wave to a counter with one atomic.  Every lane
// of the wave must call it.
__device__ __forceinline__ void wave_count_add(int64_t* field, int n) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) n += __shfl_xor(n, off, 64);
    if ((threadIdx.x & 63) == 0 && n != 0)
        atomicAdd(reinterpret_cast<unsigned long long*>(field), (unsigned long long)n);
}

// ---------------------------------------------------------------------------
// Plain FP32 solve of Eq. 7 for one pair (Section 4.3): Newton's method on
// ln P(T) = ln H in the variable ln T from the Eq. 11 guess, with a bracket
// safeguard.  Stops when |ln(P/H)| <= tol and then applies the Newton step
// already computed.  `kb` is the grain's row of K' c1 lam^-5 (stride 1);
// `nu` the wavelength table.  A finite tstart > 0 (a previous solution)
// replaces the guess as the starting point.  Returns T; *evals receives the
// number of evaluations of the sum.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float solve_newton_f32(const float* __restrict__ kb,
                                                  const float* __restrict__ nu,
                                                  int NL, float hs, float gs,
                                                  float tol, int maxit, float tstart,
                                                  int* evals, dust_counters* cnt) {
    *evals = 0;
    if (!(hs >= 0.0f) || __builtin_isinf(hs)) {
        if (cnt) count(&cnt->n_nonfinite);
        return __builtin_nanf("");
    }
    if (hs == 0.0f) return 0.0f;

    const float lnH = logf(hs);
    float lnT = (tstart > 0.0f && tstart < INFINITY) ? logf(tstart) : guess_lnT(hs, gs);
    float lo = -INFINITY, hi = INFINITY;
    bool done = false;
    int it = 0;
    for (; it < maxit; ++it) {
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
        // A start far from the root (a warm start can be anywhere) may leave
        // the sum unusable; step towards the Eq. 11 guess, or bisect once
        // the other end of the bracket is known.
        if (!(P < INFINITY)) {    // inf or NaN (1 - 2^-t rounded to 0): T far too high
            hi = lnT;
            lnT = (lo > -INFINITY) ? 0.5f * (lo + hi) : fminf(lnT - 1.0f, guess_lnT(hs, gs));
            continue;
        }
        if (!(P > 0.0f)) {        // every term underflowed: T far too low
            lo = lnT;
            lnT = (hi < INFINITY) ? 0.5f * (lo + hi) : fmaxf(lnT + 1.0f, guess_lnT(hs, gs));
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
    *evals = done ? it + 1 : it;
    if (!done && cnt) count(&cnt->n_unconverged);
    return expf(lnT);
}

// ---------------------------------------------------------------------------
// ln x for a positive finite double x: x = 2^E M, M = c_i (1 + r) with
// c_i = 1 + i/256 from the top mantissa bits (M - c_i is exact: the two lie
// within a factor 2), and ln(1 + r) from its series to r^6 (|r| < 2^-8:
// truncation < 2e-18).  ln 2 enters as a two-part constant (Cody and Waite).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double ln_f32_value(double x, const double2* __restrict__ lntab) {
    const double m = __builtin_amdgcn_frexp_mant(x);        // [0.5, 1)
    const int e = __builtin_amdgcn_frexp_exp(x) - 1;
    const double M = 2.0 * m;                               // [1, 2)
    const int i = (int)((M - 1.0) * 256.0);
    const double2 t = lntab[i];
    const double r = (M - (1.0 + i * (1.0 / 256.0))) * t.y;  // M - c_i is exact
    const double lr = r * (1.0 + r * (-0.5 + r * (1.0 / 3.0 + r * (-0.25 + r * (0.2 - r * (1.0 / 6.0))))));
    return (double)e * 6.93147180369123816490e-01 + ((double)e * 1.90821492927058770002e-10 +
                                                     (t.x + lr));
}

// 1 / x with v_rcp_f64 and one Newton-Raphson refinement (finite, nonzero x:
// the refinement turns x = inf into NaN).
__device__ __forceinline__ double rcp_f64(double x) {
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    return r;
}

// ---------------------------------------------------------------------------
// Smallest value over the wave, the same in every lane (a scalar).
// ---------------------------------------------------------------------------
__device__ __forceinline__ float wave_min_f32(float x) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) x = fminf(x, __shfl_xor(x, off, 64));
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
}

// First wavelength index l with u_l < lim, where u_l = -nu[l] decreases with
// l (NL if none); lim is wave-uniform, so the search runs on scalar loads.
__device__ __forceinline__ int first_u_below(const float* __restrict__ nu, int NL, float lim) {
    int a = 0, b = NL;
    while (a < b) {
        const int mid = (a + b) >> 1;
        if (-nu[mid] < lim) b = mid; else a = mid + 1;
    }
    return a;
}

// ---------------------------------------------------------------------------
// Plain FP32 solve of Eq. 7 for one grain and up to 64 cells, one cell per
// lane: the iteration of solve_newton_f32 (Newton on ln P = ln H in ln T,
// bracket safeguard, stop at |ln(P/H)| <= tol after applying the step),
// with the grain's weights wave-uniform (scalar loads) and the sums of
// Eq. 7 split by wavelength at every evaluation from the wave's hottest
// active cell, t = u_l / T:
//   t >= 150 for every lane: the term is exactly 0 in FP32, skipped;
//   t >= 24 for every lane: 1/(2^t - 1) = 2^-t to FP32 rounding (one
//                           exponential, no reciprocal);
//   otherwise: the exact 1/(2^t - 1).
// The slope uses ku = kb u: T dP/dT = ln 2 / T sum_l ku_l r (1 + r).
// Every lane of the wave must call it (`live` false for a lane without a
// pair).  *evals receives the lane's number of evaluations.
// ---------------------------------------------------------------------------
__device__ inline float solve_newton_wave(const float* __restrict__ kb,
                                          const float* __restrict__ ku,
                                          const float* __restrict__ nu, int NL, bool live,
                                          float hs, float gs, float tol, int maxit, float tstart,
                                          int* evals, dust_counters* cnt) {
    int nev = 0;
    float result = 0.0f;
    bool active = false;
    float lnH = 0.0f, lnT = 0.0f;
    if (live) {
        if (!(hs >= 0.0f) || __builtin_isinf(hs)) {
            if (cnt) count(&cnt->n_nonfinite);
            result = __builtin_nanf("");
        } else if (hs > 0.0f) {
            active = true;
            lnH = logf(hs);
            lnT = (tstart > 0.0f && tstart < INFINITY) ? logf(tstart) : guess_lnT(hs, gs);
        }
    }
    const bool solving = active;
    float lo = -INFINITY, hi = INFINITY;
    bool done = false;
    for (int it = 0; it < maxit; ++it) {
        if (__ballot(active) == 0) break;
        const float invT = active ? expf(-lnT) : INFINITY;
        // hottest active cell; the split only chooses between forms that are
        // exact to FP32 rounding there, so an approximate reciprocal will do
        const float tinv = __builtin_amdgcn_rcpf(wave_min_f32(invT));
        const int l1 = first_u_below(nu, NL, 150.0f * tinv);
        const int l2 = first_u_below(nu, NL, 24.0f * tinv);
        float p = 0.0f, d = 0.0f;
#pragma unroll 4
        for (int l = l1; l < l2; ++l) {
            const float y = __builtin_amdgcn_exp2f(nu[l] * invT);
            p = fmaf(kb[l], y, p);
            d = fmaf(ku[l], y, d);
        }
#pragma unroll 4
        for (int l = l2; l < NL; ++l) {
            const float r = __builtin_amdgcn_rcpf(__builtin_amdgcn_exp2f(-(nu[l] * invT)) - 1.0f);
            p = fmaf(kb[l], r, p);
            d = fmaf(ku[l], fmaf(r, r, r), d);
        }
        if (active) {
            ++nev;
            // A start far from the root (a warm start can be anywhere) may
            // leave the sum unusable; step towards the Eq. 11 guess, or bisect
            // once the other end of the bracket is known.
            if (!(p < INFINITY)) {
                hi = lnT;
                lnT = (lo > -INFINITY) ? 0.5f * (lo + hi) : fminf(lnT - 1.0f, guess_lnT(hs, gs));
            } else if (!(p > 0.0f)) {
                lo = lnT;
                lnT = (hi < INFINITY) ? 0.5f * (lo + hi) : fmaxf(lnT + 1.0f, guess_lnT(hs, gs));
            } else {
                const float r = logf(p) - lnH;                 // ln(P / H)
                const float slope = 0.69314718f * invT * d / p;  // d ln P / d ln T
                if (r < 0.0f) lo = lnT; else hi = lnT;
                float next = lnT - r / slope;
                if (fabsf(r) <= tol) {
                    lnT = next;
                    done = true;
                    active = false;
                } else {
                    if (!(next > lo && next < hi))
                        next = (lo > -INFINITY && hi < INFINITY) ? 0.5f * (lo + hi)
                                                                 : lnT - copysignf(1.0f, r);
                    lnT = next;
                }
            }
        }
    }
    *evals = nev;
    if (solving) {
        if (!done && cnt) count(&cnt->n_unconverged);
        result = expf(lnT);
    }
    return result;
}

// ---------------------------------------------------------------------------
// e^x in FP64 with few registers: Cody-Waite reduction x = k ln 2 + r
// (|r| <= ln(2)/2, ln 2 in two parts so that k ln2_hi is exact), e^r from its
// Taylor series to r^12 (truncation < 2e-16 relative), then 2^k.  Overflow
// gives +inf, underflow 0 (through subnormals).
// ---------------------------------------------------------------------------
constexpr double EXP_F64_OVERFLOW = 709.782712893384;  // ln of the largest double

__device__ __forceinline__ double exp_f64(double x) {
    if (x > EXP_F64_OVERFLOW) return __builtin_inf();
    if (x < -745.1332191019412) return 0.0;
    const double k = __builtin_rint(x * 1.4426950408889634);
    double r = fma(-k, 6.93147180369123816490e-01, x);
    r = fma(-k, 1.90821492927058770002e-10, r);
    double p = 1.0 / 479001600.0;
    p = fma(p, r, 1.0 / 39916800.0);
    p = fma(p, r, 1.0 / 3628800.0);
    p = fma(p, r, 1.0 / 362880.0);
    p = fma(p, r, 1.0 / 40320.0);
    p = fma(p, r, 1.0 / 5040.0);
    p = fma(p, r, 1.0 / 720.0);
    p = fma(p, r, 1.0 / 120.0);
    p = fma(p, r, 1.0 / 24.0);
    p = fma(p, r, 1.0 / 6.0);
    p = fma(p, r, 0.5);
    p = fma(p, r, 1.0);
    p = fma(p, r, 1.0);
    return ldexp(p, (int)k);
}

// ---------------------------------------------------------------------------
// e^x - 1 in FP64 for x >= 0: e^x - 1 where that loses at most a few units
// in the last place relative (x >= 0.01: <= 2.3e-14), the Taylor series to
// x^7 below (truncation x^8/8! < 3e-21 relative).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double expm1_pos(double x) {
    if (x >= 0.01) return exp_f64(x) - 1.0;
    const double p = 1.0 + x * (1.0 / 2 + x * (1.0 / 6 + x * (1.0 / 24 + x * (1.0 / 120 +
                     x * (1.0 / 720 + x * (1.0 / 5040))))));
    return x * p;
}

// ---------------------------------------------------------------------------
// Exact FP64 power of grain s at T and T dP/dT (Eq. 7's right side), summed
// over wavelengths by the whole wave: lane i takes wavelengths i, i+64, ...
// from l0 (a multiple of 64) on; a butterfly reduction leaves both totals in
// every lane.  Every lane of the wave must call it with the same (s, T, l0).
// The wavelengths below l0 must hold only terms that are exactly zero at T
// (see exact_first_chunk), so the sums are those over the whole grid.
// ---------------------------------------------------------------------------
__device__ inline void wave_power_f64(const PlanView& v, int s, double T, int l0, double* P,
                                      double* D) {
    const int lane = threadIdx.x & 63;
    const double* kdb = v.kdb + (int64_t)s * v.NL;
    const double invT = rcp_f64(T);
    double p = 0.0, d = 0.0;
    // (no test per chunk: the loads of successive chunks can be in flight together)
#pragma unroll 2
    for (int c0 = l0; c0 < v.NL; c0 += 64) {
        const int l = c0 + lane;
        if (l < v.NL) {
            const double x = v.c2l[l] * invT;
            const double em = expm1_pos(x);
            const double r = (em < __builtin_inf()) ? rcp_f64(em) : 0.0;  // 0 once e^x overflows
            const double b = kdb[l] * r;
            p += b;
            d += b * x * (1.0 + r);
        }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        p += __shfl_xor(p, off, 64);
        d += __shfl_xor(d, off, 64);
    }
    *P = p;
    *D = d;
}

// First wavelength (a multiple of 64) from which the exact power at any
// T <= Thi can hold a nonzero term.  The wavelengths increase, so x =
// c2 / (lam T) falls with l, and a 64-wavelength chunk whose last x is past
// the overflow point of e^x (with a margin of 1 for the rounding of T) holds
// only terms that are exactly zero: skipping such chunks leaves the sums
// unchanged bit for bit (cold grains skip the short half of the grid).  A
// binary search over the chunks, once per pair.
__device__ inline int exact_first_chunk(const PlanView& v, double Thi) {
    const double invT = rcp_f64(Thi);
    int a = 0, b = (v.NL + 63) >> 6;  // the answer lies in [a, b]
    while (a < b) {
        const int mid = (a + b) >> 1;
        const int last = (64 * mid + 63 < v.NL) ? 64 * mid + 63 : v.NL - 1;
        if (v.c2l[last] * invT > EXP_F64_OVERFLOW + 1.0) a = mid + 1;
        else b = mid;
    }
    return 64 * a;
}

// Exact FP64 solve of Eq. 7 for one pair, by the whole wave (uniform
// arguments): Newton on ln P = ln H in ln T from lnT0, safeguarded by the
// bracket [lnlo, lnhi].  Used by the mixed path for pairs outside the table.
__device__ inline double wave_solve_exact_f64(const PlanView& v, int s, double hs, double lnlo,
                                              double lnhi, double lnT0, bool* ok) {
    const double lnH = ln_f32_value(hs, v.lntab);
    double lo = lnlo, hi = lnhi;
    double lnT = (lnT0 > lo && lnT0 < hi) ? lnT0 : 0.5 * (lo + hi);
    // every iterate stays at or below the bracket's top
    const int l0 = exact_first_chunk(v, exp_f64(lnhi));
    for (int it = 0; it < 100; ++it) {
        double P, D;
        wave_power_f64(v, s, exp_f64(lnT), l0, &P, &D);
        double next;
        if (!(P > 0.0 && P < __builtin_inf())) {
            if (P > 0.0) hi = lnT; else lo = lnT;  // inf: T far too high; 0: far too low
            next = 0.5 * (lo + hi);
        } else {
            const double r = ln_f32_value(P, v.lntab) - lnH;
            if (r < 0.0) lo = lnT; else hi = lnT;
            next = lnT - r * P / D;
            // a step below 1e-9 leaves an error near its square: done
            if (fabs(next - lnT) <= 1e-9) { *ok = true; return next; }
            if (!(next > lo && next < hi)) next = 0.5 * (lo + hi);
        }
        if (hi - lo <= 1e-14) { *ok = true; return 0.5 * (lo + hi); }
        lnT = next;
    }
    *ok = false;
    return lnT;
}

// ---------------------------------------------------------------------------
// Cubic through four consecutive FP64 table values y0..y3 at unit-spaced
// nodes 0..3, in Newton's divided-difference form, at x; *dp = d/dx.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double cubic4(double x, double y0, double y1, double y2, double y3,
                                         double* dp) {
    const double d1 = y1 - y0;
    const double d2 = 0.5 * (y2 - 2.0 * y1 + y0);
    const double d3 = (y3 - 3.0 * (y2 - y1) - y0) * (1.0 / 6.0);
    const double xm1 = x - 1.0, xm2 = x - 2.0;
    *dp = d1 + (x + xm1) * d2 + (x * xm1 + x * xm2 + xm1 * xm2) * d3;
    return y0 + x * (d1 + xm1 * (d2 + xm2 * d3));
}

// First node of the 4-point stencil for interval [k, k+1] of an N-point table.
__device__ __forceinline__ int stencil_start(int k, int N) {
    const int j0 = k - 1;
    return j0 < 0 ? 0 : (j0 > N - 4 ? N - 4 : j0);
}


// Position u = (ln H' - y_0) / dy of ln H' on the grain's inverse-table grid
// (FP32), and the cubic Hermite of that table at u in node interval j.
__device__ __forceinline__ float inv_pos_f32(const PlanView& v, int s, float hs) {
    return (logf(hs) - v.ylof[s]) * v.dyinvf[s];
}

__device__ __forceinline__ float inv_hermite_f32(const PlanView& v, int s, float u, int j) {
    const float4 g = v.invf[(int64_t)s * (v.M - 1) + j];
    const float t = u - (float)j;
    const float t2 = t * t, t3 = t2 * t;
    const float lnT = (2.0f * t3 - 3.0f * t2 + 1.0f) * g.x + (t3 - 2.0f * t2 + t) * g.y +
                      (3.0f * t2 - 2.0f * t3) * g.z + (t3 - t2) * g.w;
    return expf(lnT);
}

// ---------------------------------------------------------------------------
// FP32 mixed solve of Eq. 7: the grain's inverse table ln T(y), y = ln H',
// as a cubic Hermite in FP32 between the two nodes around y (one 16-byte
// entry holds both).  FP32 rounding of y (|y| up to about 50) and of the
// table leaves a relative T error of about 2e-6; the Hermite itself is far
// below that.  Returns 0 with *T set, or nonzero for a pair outside the
// table (then solved exactly).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int table_lookup_f32(const PlanView& v, int s, float hs, float* T,
                                                dust_counters* cnt) {
    if (!(hs >= 0.0f) || __builtin_isinf(hs)) {
        if (cnt) count(&cnt->n_nonfinite);
        *T = __builtin_nanf("");
        return 0;
    }
    if (hs == 0.0f) { *T = 0.0f; return 0; }
    const float u = inv_pos_f32(v, s, hs);
    if (!(u >= 0.0f && u <= (float)(v.M - 1))) return 1;  // outside, or the table is not finite
    const int j = (int)u < v.M - 2 ? (int)u : v.M - 2;
    *T = inv_hermite_f32(v, s, u, j);
    return 0;
}

// ---------------------------------------------------------------------------
// ln x of a positive normal FP32 value, as an FP64 value with an absolute
// error of about 4e-8: the binary exponent enters exactly and only log2 of
// the mantissa (in [0.5, 1)) goes through v_log_f32.  The temperature step
// needs y = ln H' to a small absolute error (T moves by about dy / 5), which
// the FP32 rounding of y itself (|y| up to about 80) would not give.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double ln_normal_f32(float x) {
    const float m = __builtin_amdgcn_frexp_mantf(x);
    const int e = __builtin_amdgcn_frexp_expf(x);
    return ((double)e + (double)__builtin_amdgcn_logf(m)) * LN2;
}

// Position u = (ln H' - y_0) / dy of ln H' on the grain's FP64 inverse-table
// grid, and the cubic Hermite of that table at u in node interval j, with T
// leaving in FP32 as e^head (1 + tail) from the FP32 head of ln T.
__device__ __forceinline__ double inv_pos_f64(const PlanView& v, int s, float hs) {
    return (ln_normal_f32(hs) - v.ylo[s]) * v.dyinv[s];
}

__device__ __forceinline__ float inv_hermite_f64(const PlanView& v, int s, double u, int j) {
    const double2* g = v.invd + (int64_t)s * v.M + j;
    const double2 g0 = g[0], g1 = g[1];
    const double t = u - (double)j;
    const double d = g1.x - g0.x;
    const double c2 = 3.0 * d - 2.0 * g0.y - g1.y;
    const double c3 = g0.y + g1.y - 2.0 * d;
    const double lnT = g0.x + t * (g0.y + t * (c2 + t * c3));
    const float head = (float)lnT;
    return expf(head) * (1.0f + (float)(lnT - (double)head));
}

// ---------------------------------------------------------------------------
// Default mixed solve of Eq. 7: the grain's inverse table ln T(y), y = ln H',
// at uniform steps of y (no search), as a cubic Hermite evaluated in FP64
// between the FP64 nodes around y.  With 256 nodes the interpolation error
// is about 1e-9 in T; T leaves in FP32 as e^head (1 + tail) from the FP32
// head of ln T and its small tail (relative error about 1.5e-7).  Returns 0
// with *T set, or nonzero for a pair outside the table (or with a subnormal
// H'), which the exact FP64 solve then takes.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int table_lookup_f64(const PlanView& v, int s, float hs, float* T,
                                                dust_counters* cnt) {
    if (!(hs >= 0.0f) || __builtin_isinf(hs)) {
        if (cnt) count(&cnt->n_nonfinite);
        *T = __builtin_nanf("");
        return 0;
    }
    if (hs == 0.0f) { *T = 0.0f; return 0; }
    if (hs < 1.17549435e-38f) return 1;  // subnormal
    const double u = inv_pos_f64(v, s, hs);
    if (!(u >= 0.0 && u <= (double)(v.M - 1))) return 1;  // outside, or not finite
    const int j = (int)u < v.M - 2 ? (int)u : v.M - 2;
    *T = inv_hermite_f64(v, s, u, j);
    return 0;
}

// ---------------------------------------------------------------------------
// The two lookups above without branches, for kernels that take several pairs
// per thread: the node loads are made at a clamped index whatever the pair,
// so that the loads of all the thread's pairs can be in flight together, and
// the outcome is selected at the end.  *T and the status agree with the
// branching forms pair for pair (the nonfinite count is left to the caller).
// ---------------------------------------------------------------------------
constexpr int LOOKUP_OK = 0, LOOKUP_PENDING = 1, LOOKUP_NONFINITE = 2;

__device__ __forceinline__ int table_lookup_f64_nb(const PlanView& v, int s, float hs, float* T) {
    const double u = inv_pos_f64(v, s, hs);
    const bool in = u >= 0.0 && u <= (double)(v.M - 1);
    const double uc = in ? u : 0.0;
    const int j = (int)uc < v.M - 2 ? (int)uc : v.M - 2;
    const float t = inv_hermite_f64(v, s, uc, j);
    const bool bad = !(hs >= 0.0f) || __builtin_isinf(hs);
    const bool zero = hs == 0.0f;
    *T = bad ? __builtin_nanf("") : (zero ? 0.0f : t);
    return bad ? LOOKUP_NONFINITE
               : (zero ? LOOKUP_OK
                       : ((hs < 1.17549435e-38f || !in) ? LOOKUP_PENDING : LOOKUP_OK));
}

__device__ __forceinline__ int table_lookup_f32_nb(const PlanView& v, int s, float hs, float* T) {
    const float u = inv_pos_f32(v, s, hs);
    const bool in = u >= 0.0f && u <= (float)(v.M - 1);
    const float uc = in ? u : 0.0f;
    const int j = (int)uc < v.M - 2 ? (int)uc : v.M - 2;
    const float t = inv_hermite_f32(v, s, uc, j);
    const bool bad = !(hs >= 0.0f) || __builtin_isinf(hs);
    const bool zero = hs == 0.0f;
    *T = bad ? __builtin_nanf("") : (zero ? 0.0f : t);
    return bad ? LOOKUP_NONFINITE : (zero ? LOOKUP_OK : (!in ? LOOKUP_PENDING : LOOKUP_OK));
}

// ---------------------------------------------------------------------------
// Mixed solve with the FP64 Newton polish of Eq. 7 on the grain's forward
// table (dust_options.newton_polish): the inverse-table lookup above gives
// ln T0; the four forward-table values around the interval it falls in are
// read at once, the interval whose powers bracket H' is taken among the
// stencil's three (a step to a neighbour if rounding put ln T0 across a
// node), and a Newton step in FP64 on y(ln T) = ln P'(T) -- the cubic through
// the four values -- refines ln T inside that bracket (a step that would
// leave it bisects it instead).  The start lies within about 1e-9 of the
// cubic's root, so one step reaches FP64 rounding; what remains is the
// cubic's own interpolation error (about 1e-11 in ln T at 4096 table points
// over 2.7-3000 K).  Returns 0 with *T set, or nonzero for a pair outside the
// table (solved exactly instead).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int table_lookup_polish(const PlanView& v, int s, float hs, float* T,
                                                   dust_counters* cnt) {
    if (!(hs >= 0.0f) || __builtin_isinf(hs)) {
        if (cnt) count(&cnt->n_nonfinite);
        *T = __builtin_nanf("");
        return 0;
    }
    if (hs == 0.0f) { *T = 0.0f; return 0; }
    if (hs < 1.17549435e-38f) return 1;  // subnormal
    const double y = ln_normal_f32(hs);
    const double u = (y - v.ylo[s]) * v.dyinv[s];
    if (!(u >= 0.0 && u <= (double)(v.M - 1))) return 1;  // outside, or not finite
    const int j = (int)u < v.M - 2 ? (int)u : v.M - 2;
    const double2* g = v.invd + (int64_t)s * v.M + j;
    const double2 g0 = g[0], g1 = g[1];
    const double t = u - (double)j;
    const double d = g1.x - g0.x;
    const double c2 = 3.0 * d - 2.0 * g0.y - g1.y;
    const double c3 = g0.y + g1.y - 2.0 * d;
    const double lnT0 = g0.x + t * (g0.y + t * (c2 + t * c3));
    // the stencil around the interval of ln T0, and the bracketing interval in it
    const int N = v.N;
    const double xk = (lnT0 - v.lnTmin) / v.hstep;
    int k = (int)xk;
    k = k < 0 ? 0 : (k > N - 2 ? N - 2 : k);
    const int j0 = stencil_start(k, N);
    const double* f = v.fwd + (int64_t)s * N + j0;
    const double a0 = f[0], a1 = f[1], a2 = f[2], a3 = f[3];
    int kk = k - j0;  // 0, 1 or 2
    const double ylo_k = kk == 0 ? a0 : (kk == 1 ? a1 : a2);
    const double yhi_k = kk == 0 ? a1 : (kk == 1 ? a2 : a3);
    if (y < ylo_k && kk > 0) --kk;
    else if (y > yhi_k && kk < 2) ++kk;
    const double lo = (double)kk, hi = lo + 1.0;
    double x = xk - (double)j0;
    x = x < lo ? lo : (x > hi ? hi : x);
    double dp;
    const double r = cubic4(x, a0, a1, a2, a3, &dp) - y;
    if (r != 0.0) {
        const double xn = x - r / dp;
        x = (xn >= lo && xn <= hi) ? xn : (r > 0.0 ? 0.5 * (lo + x) : 0.5 * (x + hi));
    }
    const double lnT = v.lnTmin + ((double)j0 + x) * v.hstep;
    const float head = (float)lnT;
    *T = expf(head) * (1.0f + (float)(lnT - (double)head));
    return 0;
}

// The lookup of a mixed kernel form.
template <int MODE>
__device__ __forceinline__ int mixed_lookup(const PlanView& v, int s, float hs, float* T,
                                            dust_counters* cnt) {
    if constexpr (MODE == MODE_MIXED_F32) {
        return table_lookup_f32(v, s, hs, T, cnt);
    } else if constexpr (MODE == MODE_MIXED_POLISH) {
        return table_lookup_polish(v, s, hs, T, cnt);
    } else {
        return table_lookup_f64(v, s, hs, T, cnt);
    }
}

// Bracket [*lo, *hi] and start *lnT0 (ln T) of the exact solve of a pair
// the table lookup did not take, y = ln H': below the table (T < T_0), above
// it, a grain whose table is not finite, or a pair on the table's edge that
// FP32 rounding put outside.  Starts extrapolate the end interval's slope
// (in 1/T below the table, in ln T above it).
__device__ inline void pending_bracket(const PlanView& v, int s, double y, double* lo,
                                       double* hi, double* lnT0) {
    const double ylo = v.ylo[s], yhi = v.yhi[s];
    const int N = v.N;
    const double lnTmax = v.lnTmin + (N - 1) * v.hstep;
    const double* f = v.fwd + (int64_t)s * N;
    *lo = -6.907755278982137;  // ln 1e-3
    *hi = 16.11809565095832;   // ln 1e7
    if (!(__builtin_isfinite(ylo) && __builtin_isfinite(yhi) && yhi > ylo)) {
        *lnT0 = 0.5 * (*lo + *hi);
    } else if (y < ylo) {
        // Wien side: ln P' is close to linear in 1/T there, so extrapolate the
        // first interval's slope in u = 1/T (one Newton step fewer below 1.5 K)
        *hi = v.lnTmin;
        const double u0 = exp_f64(-v.lnTmin), u1 = exp_f64(-(v.lnTmin + v.hstep));
        const double u = u0 + (y - ylo) * (u1 - u0) / (f[1] - f[0]);
        *lnT0 = (u > u0 && u < 1e300) ? -ln_f32_value(u, v.lntab) : 0.5 * (*lo + *hi);
    } else if (y > yhi) {
        *lo = lnTmax;
        *lnT0 = lnTmax + (y - yhi) * v.hstep / (f[N - 1] - f[N - 2]);
    } else {
        *lnT0 = v.lnTmin + (y - ylo) / (yhi - ylo) * (lnTmax - v.lnTmin);
    }
}

// Exact FP64 solve of one pair the table lookup did not take, by the whole
// wave: every lane calls it with the same arguments and receives T.  Counts
// the pair as out of table.
__device__ inline float wave_solve_pending(const PlanView& v, int s, double hs,
                                           dust_counters* cnt) {
    double lo, hi, lnT0;
    pending_bracket(v, s, ln_f32_value(hs, v.lntab), &lo, &hi, &lnT0);
    bool ok = false;
    const double lnT = wave_solve_exact_f64(v, s, hs, lo, hi, lnT0, &ok);
    if (cnt && (threadIdx.x & 63) == 0) {
        count(&cnt->n_out_of_table);
        if (!ok) count(&cnt->n_unconverged);
    }
    return (float)exp_f64(lnT);
}

// ---------------------------------------------------------------------------
// Table-linear solve for one pair (the production variant of Sections 2 and
// 5): with P'_k the grain's FP64 table at T_k = tmin + k tstep, find k with
// P'_k <= H' < P'_{k+1} and interpolate T linearly between T_k and T_{k+1}.
// The search starts from the bracket [kidx[j], kidx[j+1] + 1] of the ln P'
// node j below ln H' (a few table points wide) and falls back to the whole
// table if rounding put H' outside it.  H' outside the table gives the end
// temperature (counted).  hs is an FP32 value in the plan's scaled units.
// ---------------------------------------------------------------------------
__device__ inline float table_linear_T(const PlanView& v, int s, float hs, dust_counters* cnt) {
    if (!(hs >= 0.0f) || __builtin_isinf(hs)) {
        if (cnt) count(&cnt->n_nonfinite);
        return __builtin_nanf("");
    }
    if (hs == 0.0f) return 0.0f;
    const int N = v.N;
    const double* P = v.fwd + (int64_t)s * N;
    const double h = (double)hs;
    const double p0 = P[0], pn = P[N - 1];
    if (!(h >= p0 && h < pn)) {
        if (cnt && h != pn) count(&cnt->n_out_of_table);
        return (float)(h < p0 ? v.texp[0] : v.texp[N - 1]);
    }
    // the position only chooses the bracket (a miss falls back to the whole
    // table), so the table-free ln of the FP32 value is enough
    const double u = (ln_normal_f32(hs) - v.ylo[s]) * v.dyinv[s];
    const int j = (u > 0.0) ? (u < (double)(v.M - 2) ? (int)u : v.M - 2) : 0;
    const int* kx = v.kidx + (int64_t)s * v.M;
    int a = kx[j], b = kx[j + 1] + 1;  // kidx <= N - 2, so b <= N - 1
    double pa = P[a], pb = P[b];
    if (!(pa <= h && h < pb)) {
        a = 0;
        b = N - 1;
        pa = p0;
        pb = pn;
    }
    while (b - a > 1) {  // invariant: P'_a <= h < P'_b
        const int mid = (a + b) >> 1;
        const double pm = P[mid];
        if (pm <= h) { a = mid; pa = pm; } else { b = mid; pb = pm; }
    }
    return (float)(v.texp[a] + (h - pa) * rcp_f64(pb - pa) * v.tstep);
}

// Capacity of a block's LDS list of pending pairs.
constexpr int PENDING_CAP = 256;

// ---------------------------------------------------------------------------
// Emission of TC cells at one wavelength (Eqs. 9-10, Section 4.4).
//
// The lane owns wavelength l and accumulates, for each of its TC cells,
//   sum_s em[s,l] / (2^t - 1),   t = u_l / T[c,s],  u_l = h c log2(e) / (k lam_l)
// (em already holds w_s C[s,l] c1 lam_l^-5).  nu = -u_l.
//
// LDS tile (filled by the caller):
//   sInvT  [TC][Sp]  1/T per cell and grain (+inf for T = 0, NaN for bad T);
//   sChunk [Sp/8][TC] bits of the smallest 1/T over each group of 8 grains
//                     (0 when the group holds a NaN).
// Both are read with wave-uniform addresses (LDS broadcast).
//
// For each (8-grain group, cell) the wave picks one evaluation, uniformly, by
// comparing the group's hottest grain at the wave's longest wavelength
// (smallest t over the wave's lanes) with three thresholds.  With y = 2^-t,
// 1/(2^t - 1) = y / (1 - y) = y + y^2 + ..., and cutting the series after
// y^n leaves the relative error y^n / (1 - y):
//   t >= 150      every term is exactly 0 in FP32 (2^-150 underflows): skip;
//   24 <= t       use y (relative error <= 2^-24);
//   12 <= t < 24  use y + y^2 (relative error <= 2^-24 (1 + 2^-12));
//   otherwise     the exact form rcp(2^t - 1).
// The comparisons are on the float bit patterns of non-negative values (their
// order is that of unsigned integers), so they run on the scalar unit.
// Costs per term: 0, 2 VALU + 1 exp, 3 VALU + 1 exp, 3 VALU + exp + rcp.
// ---------------------------------------------------------------------------
constexpr int EMIT_GROUP = 8;  // grains per class decision

__device__ __forceinline__ bool any_nan8(const float4& a, const float4& b) {
    return __builtin_isnan(a.x) || __builtin_isnan(a.y) || __builtin_isnan(a.z) ||
           __builtin_isnan(a.w) || __builtin_isnan(b.x) || __builtin_isnan(b.y) ||
           __builtin_isnan(b.z) || __builtin_isnan(b.w);
}

// LDS bytes of an emission tile of TC cells: sInvT, sChunk and sPair.
__host__ __device__ constexpr size_t emit_lds_bytes(int TC, int Sp) {
    return (size_t)TC * (size_t)Sp * sizeof(float) +
           (size_t)(Sp / EMIT_GROUP) * TC * sizeof(uint32_t) +
           (size_t)(Sp / (2 * EMIT_GROUP)) * TC * sizeof(uint32_t);
}

// Fill sChunk from sInvT (all threads of the block; caller synchronises).
template <int TC>
__device__ __forceinline__ void fill_chunk_min(const float* sInvT, uint32_t* sChunk, int Sp) {
    const int SC = Sp / EMIT_GROUP;
    for (int i = threadIdx.x; i < TC * SC; i += blockDim.x) {
        const int ch = i / TC, cc = i - ch * TC;
        const float4 a = *reinterpret_cast<const float4*>(sInvT + cc * Sp + EMIT_GROUP * ch);
        const float4 b = *reinterpret_cast<const float4*>(sInvT + cc * Sp + EMIT_GROUP * ch + 4);
        const float m = fminf(fminf(fminf(a.x, a.y), fminf(a.z, a.w)),
                              fminf(fminf(b.x, b.y), fminf(b.z, b.w)));
        // a NaN forces the exact form, which propagates it
        sChunk[i] = any_nan8(a, b) ? 0u : __float_as_uint(m);
    }
    // sPair [Sp/16][TC], right after sChunk: the same over each 16 grains
    // (a pair of groups), for the block emission's choices
    uint32_t* sPair = sChunk + SC * TC;
    for (int i = threadIdx.x; i < TC * (SC / 2); i += blockDim.x) {
        const int pr = i / TC, cc = i - pr * TC;
        const float* row = sInvT + cc * Sp + 2 * EMIT_GROUP * pr;
        const float4 a = *reinterpret_cast<const float4*>(row);
        const float4 b = *reinterpret_cast<const float4*>(row + 4);
        const float4 c = *reinterpret_cast<const float4*>(row + 8);
        const float4 d = *reinterpret_cast<const float4*>(row + 12);
        const float m = fminf(fminf(fminf(fminf(a.x, a.y), fminf(a.z, a.w)),
                                    fminf(fminf(b.x, b.y), fminf(b.z, b.w))),
                              fminf(fminf(fminf(c.x, c.y), fminf(c.z, c.w)),
                                    fminf(fminf(d.x, d.y), fminf(d.z, d.w))));
        sPair[i] = (any_nan8(a, b) || any_nan8(c, d)) ? 0u : __float_as_uint(m);
    }
}

// 1/u_min for the thresholds on 1/T (t >= t0 <=> 1/T >= t0 / u_min), with
// v_rcp_f32 instead of a correctly rounded division and a relative margin
// of 2^-20 that only raises the thresholds, so that each form keeps its
// guarantee (its rounding error is far below the margin).
__device__ __forceinline__ float emit_threshold_scale(float u_min) {
    return __builtin_amdgcn_rcpf(u_min) * (1.0f + 0x1p-20f);
}

// TC cells from sInvT rows 0..TC-1 and sChunk columns 0..TC-1 (TCS, the
// row stride of sChunk, is the whole tile's cell count).
template <int TC, int TCS = TC>
__device__ __forceinline__ void emit_accumulate(const float* __restrict__ em, int NLp,
                                                float nu, float u_wave_min,
                                                const float* sInvT, const uint32_t* sChunk,
                                                int Sp, int S, float (&acc)[TC]) {
    static_assert(TC % 4 == 0, "cells per tile must be a multiple of 4");
    // Thresholds on 1/T for this wave (uniform).
    const float ru = emit_threshold_scale(u_wave_min);
    const uint32_t thr_skip = (uint32_t)__builtin_amdgcn_readfirstlane(__float_as_uint(150.0f * ru));
    const uint32_t thr_y = (uint32_t)__builtin_amdgcn_readfirstlane(__float_as_uint(24.0f * ru));
    const uint32_t thr_y2 = (uint32_t)__builtin_amdgcn_readfirstlane(__float_as_uint(12.0f * ru));
#pragma unroll
    for (int cc = 0; cc < TC; ++cc) acc[cc] = 0.0f;
    for (int s = 0; s < S; s += EMIT_GROUP) {
        float e[EMIT_GROUP];
#pragma unroll
        for (int g = 0; g < EMIT_GROUP; ++g) e[g] = em[(int64_t)(s + g) * NLp];
        const uint32_t* cmrow = sChunk + (s / EMIT_GROUP) * TCS;
#pragma unroll
        for (int c4 = 0; c4 < TC; c4 += 4) {
            const uint4 cm4 = *reinterpret_cast<const uint4*>(cmrow + c4);
            float4 ia[4], ib[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                ia[k] = *reinterpret_cast<const float4*>(sInvT + (c4 + k) * Sp + s);
                ib[k] = *reinterpret_cast<const float4*>(sInvT + (c4 + k) * Sp + s + 4);
            }
            const uint32_t cms[4] = {(uint32_t)__builtin_amdgcn_readfirstlane(cm4.x),
                                     (uint32_t)__builtin_amdgcn_readfirstlane(cm4.y),
                                     (uint32_t)__builtin_amdgcn_readfirstlane(cm4.z),
                                     (uint32_t)__builtin_amdgcn_readfirstlane(cm4.w)};
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const uint32_t cm = cms[k];
                if (cm >= thr_skip) continue;
                const float it[EMIT_GROUP] = {ia[k].x, ia[k].y, ia[k].z, ia[k].w,
                                              ib[k].x, ib[k].y, ib[k].z, ib[k].w};
                // each branch updates the accumulator in place (no copy at the merge)
                if (cm >= thr_y) {
#pragma unroll
                    for (int g = 0; g < EMIT_GROUP; ++g)
                        acc[c4 + k] = fmaf(e[g], __builtin_amdgcn_exp2f(nu * it[g]), acc[c4 + k]);
                } else if (cm >= thr_y2) {
#pragma unroll
                    for (int g = 0; g < EMIT_GROUP; ++g) {
                        const float y = __builtin_amdgcn_exp2f(nu * it[g]);
                        acc[c4 + k] = fmaf(e[g], fmaf(y, y, y), acc[c4 + k]);
                    }
                } else {
#pragma unroll
                    for (int g = 0; g < EMIT_GROUP; ++g)
                        acc[c4 + k] = fmaf(
                            e[g], __builtin_amdgcn_rcpf(__builtin_amdgcn_exp2f(-(nu * it[g])) - 1.0f),
                            acc[c4 + k]);
                }
            }
        }
    }
}

// 1/T as the emission tile stores it: T < 0 or NaN gives NaN (the cell's SED
// becomes NaN), T = 0 gives +inf (the grain emits nothing).
__device__ __forceinline__ float inv_temperature(float t) {
    // v_rcp_f32 (1 ulp): 1/T only enters the FP32 emission exponent
    return (t >= 0.0f) ? __builtin_amdgcn_rcpf(t) : __builtin_nanf("");
}

// Smallest u = -nu over the valid wavelengths of the wave that owns
// wavelengths [l_wave0, l_wave0 + 64): the one at its longest wavelength.
__device__ __forceinline__ float wave_u_min(const float* nu, int l_wave0, int NL) {
    const int lw = (l_wave0 + 63 < NL) ? l_wave0 + 63 : NL - 1;
    return -nu[lw];
}

// Emission of a grid with nch <= 2 wavelength chunks of 64: wave w takes
// chunk w mod nch and CW = TC nch / 4 cells starting at (w / nch) CW.
template <int CW, int TC>
__device__ __forceinline__ void emit_cell_part(const PlanView& v, int64_t c0, int64_t C,
                                               const float* __restrict__ m,
                                               float* __restrict__ L, int64_t ldl,
                                               const float* sInvT, const uint32_t* sChunk,
                                               int nch) {
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int chunk = wave % nch;
    const int cbase = (wave / nch) * CW;
    const int l = chunk * 64 + (threadIdx.x & 63);
    const bool lv = l < v.NL;
    const float nu = v.nu[lv ? l : 0];
    const float uw = wave_u_min(v.nu, chunk * 64, v.NL);
    float acc[CW];
    emit_accumulate<CW, TC>(v.em + (lv ? l : 0), v.NLp, nu, uw, sInvT + cbase * v.Sp,
                            sChunk + cbase, v.Sp, v.S, acc);
    if (lv) {
#pragma unroll
        for (int cc = 0; cc < CW; ++cc) {
            const int64_t c = c0 + cbase + cc;
            if (c < C) L[c * ldl + l] = acc[cc] * ((m ? m[c] : 1.0f) * v.escale);
        }
    }
}


// ---------------------------------------------------------------------------
// Emission of 16 cells over one block of LW = 64 / ROWS wavelengths by one
// wave: lane (row r = lane / LW, i = lane mod LW) takes wavelength LW lb + i
// and, of every 16 grains, grains 16p + GR r .. 16p + GR r + GR - 1
// (GR = 16 / ROWS); the rows' partial sums are added across lanes at the end:
// with two rows, row r then holds the sum of cell 2k + r in acc[2k], with
// more rows every lane holds all 16 sums.
// A block of fewer than 64 wavelengths spans a smaller range of t, so more
// (16 grains, cell) choices take a cheap form.  The form is chosen as in
// emit_accumulate, per 16 grains, from their smallest 1/T (sPair; the odd
// last group of TAIL from sChunk; TCS the row stride of both, already offset
// to the first of the 16 cells) and the block's smallest u.  Requires
// LW lb < NLp.
// ---------------------------------------------------------------------------
constexpr int EMIT_ROWS = 2;  // rows of a wave in the block emission

// One choice step of emit_block: the calling lane's GRr grains starting at
// its row's first grain (emp, itp already offset to it), all 16 cells, the
// form chosen from the smallest 1/T bits cmA[c] (and cmB[c] when given).
template <int GRr>
__device__ __forceinline__ void emit_step(const float* emp, int NLp, const float* itp, int Sp,
                                          float nu, const uint32_t* cmA, const uint32_t* cmB,
                                          uint32_t thr_skip, uint32_t thr_y, uint32_t thr_y2,
                                          float (&acc)[16]) {
    float e[GRr];
#pragma unroll
    for (int g = 0; g < GRr; ++g) e[g] = emp[(int64_t)g * NLp];
#pragma unroll
    for (int c4 = 0; c4 < 16; c4 += 4) {
        uint4 a4 = *reinterpret_cast<const uint4*>(cmA + c4);
        if (cmB) {
            // uint min: a NaN group (0) forces the exact form for both groups
            const uint4 b4 = *reinterpret_cast<const uint4*>(cmB + c4);
            a4.x = a4.x < b4.x ? a4.x : b4.x;
            a4.y = a4.y < b4.y ? a4.y : b4.y;
            a4.z = a4.z < b4.z ? a4.z : b4.z;
            a4.w = a4.w < b4.w ? a4.w : b4.w;
        }
        float it[4][GRr];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
#pragma unroll
            for (int q = 0; q < GRr; q += 4) {
                const float4 x = *reinterpret_cast<const float4*>(itp + (c4 + k) * Sp + q);
                it[k][q] = x.x; it[k][q + 1] = x.y; it[k][q + 2] = x.z; it[k][q + 3] = x.w;
            }
        }
        const uint32_t cms[4] = {(uint32_t)__builtin_amdgcn_readfirstlane(a4.x),
                                 (uint32_t)__builtin_amdgcn_readfirstlane(a4.y),
                                 (uint32_t)__builtin_amdgcn_readfirstlane(a4.z),
                                 (uint32_t)__builtin_amdgcn_readfirstlane(a4.w)};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint32_t cm = cms[k];
            if (cm >= thr_skip) continue;
            // each branch updates the accumulator in place (no copy at the merge)
            if (cm >= thr_y) {
#pragma unroll
                for (int g = 0; g < GRr; ++g)
                    acc[c4 + k] = fmaf(e[g], __builtin_amdgcn_exp2f(nu * it[k][g]), acc[c4 + k]);
            } else if (cm >= thr_y2) {
#pragma unroll
                for (int g = 0; g < GRr; ++g) {
                    const float y = __builtin_amdgcn_exp2f(nu * it[k][g]);
                    acc[c4 + k] = fmaf(e[g], fmaf(y, y, y), acc[c4 + k]);
                }
            } else {
#pragma unroll
                for (int g = 0; g < GRr; ++g)
                    acc[c4 + k] = fmaf(
                        e[g], __builtin_amdgcn_rcpf(__builtin_amdgcn_exp2f(-(nu * it[k][g])) - 1.0f),
                        acc[c4 + k]);
            }
        }
    }
}

template <int ROWS, int TCS, bool TAIL>
__device__ __forceinline__ void emit_block(const PlanView& v, int lb, const float* sInvT,
                                           const uint32_t* sChunk, const uint32_t* sPair,
                                           float (&acc)[16]) {
    constexpr int LW = 64 / ROWS, GR = 16 / ROWS;
    static_assert(GR % 8 == 0 || GR == 4, "a row takes whole float4s of grains");
    const int lane = threadIdx.x & 63;
    const int r = lane / LW;
    const int l = lb * LW + (lane % LW);
    const float nu = v.nu[l];
    const int lw = (lb * LW + LW - 1 < v.NL) ? lb * LW + LW - 1 : v.NL - 1;
    const float umin = -v.nu[lw];
    const float ru = emit_threshold_scale(umin);
    const uint32_t thr_skip = (uint32_t)__builtin_amdgcn_readfirstlane(__float_as_uint(150.0f * ru));
    const uint32_t thr_y = (uint32_t)__builtin_amdgcn_readfirstlane(__float_as_uint(24.0f * ru));
    const uint32_t thr_y2 = (uint32_t)__builtin_amdgcn_readfirstlane(__float_as_uint(12.0f * ru));
    const float* emp = v.em + (int64_t)(GR * r) * v.NLp + l;
    const float* itp = sInvT + GR * r;
#pragma unroll
    for (int cc = 0; cc < 16; ++cc) acc[cc] = 0.0f;
    // 16-grain steps over the groups that hold real grains; with TAIL an odd
    // last group is left to the step below instead of being paired with
    // padding (a separate instantiation: the tail's code alone costs the
    // main loop registers)
    const int G = (v.S + EMIT_GROUP - 1) / EMIT_GROUP;
    const int s_pairs = TAIL ? (G & ~1) * EMIT_GROUP : v.S;
    for (int s = 0; s < s_pairs; s += 2 * EMIT_GROUP) {
        float e[GR];
#pragma unroll
        for (int g = 0; g < GR; ++g) e[g] = emp[(int64_t)(s + g) * v.NLp];
        const uint32_t* cmp = sPair + (s / (2 * EMIT_GROUP)) * TCS;
#pragma unroll
        for (int c4 = 0; c4 < 16; c4 += 4) {
            const uint4 a4 = *reinterpret_cast<const uint4*>(cmp + c4);
            float it[4][GR];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
#pragma unroll
                for (int q = 0; q < GR; q += 4) {
                    const float4 x = *reinterpret_cast<const float4*>(itp + (c4 + k) * v.Sp + s + q);
                    it[k][q] = x.x; it[k][q + 1] = x.y; it[k][q + 2] = x.z; it[k][q + 3] = x.w;
                }
            }
            const uint32_t cms[4] = {(uint32_t)__builtin_amdgcn_readfirstlane(a4.x),
                                     (uint32_t)__builtin_amdgcn_readfirstlane(a4.y),
                                     (uint32_t)__builtin_amdgcn_readfirstlane(a4.z),
                                     (uint32_t)__builtin_amdgcn_readfirstlane(a4.w)};
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const uint32_t cm = cms[k];
                if (cm >= thr_skip) continue;
                // each branch updates the accumulator in place (no copy at the merge)
                if (cm >= thr_y) {
#pragma unroll
                    for (int g = 0; g < GR; ++g)
                        acc[c4 + k] = fmaf(e[g], __builtin_amdgcn_exp2f(nu * it[k][g]), acc[c4 + k]);
                } else if (cm >= thr_y2) {
#pragma unroll
                    for (int g = 0; g < GR; ++g) {
                        const float y = __builtin_amdgcn_exp2f(nu * it[k][g]);
                        acc[c4 + k] = fmaf(e[g], fmaf(y, y, y), acc[c4 + k]);
                    }
                } else {
#pragma unroll
                    for (int g = 0; g < GR; ++g)
                        acc[c4 + k] = fmaf(
                            e[g],
                            __builtin_amdgcn_rcpf(__builtin_amdgcn_exp2f(-(nu * it[k][g])) - 1.0f),
                            acc[c4 + k]);
                }
            }
        }
    }
    // an odd last group: its 8 grains split over the rows, so that no row
    // works on grains past the last group
    if (TAIL && (G & 1)) {
        constexpr int GT = EMIT_GROUP / ROWS;
        const int s_row = s_pairs + GT * r;
        emit_step<GT>(v.em + l + (int64_t)s_row * v.NLp, v.NLp, sInvT + s_row, v.Sp, nu,
                      sChunk + (s_pairs / EMIT_GROUP) * TCS, nullptr, thr_skip, thr_y, thr_y2,
                      acc);
    }
    // the rows hold partial sums over different grains
    if constexpr (ROWS == 2) {
        // v_permlane32_swap of cells 2k and 2k + 1 leaves row 0's and row 1's
        // partial sums of cell 2k in the two registers of lanes 0-31 and
        // those of cell 2k + 1 in lanes 32-63: one add gives row r the sum of
        // cell 2k + r in acc[2k], with no trip through LDS
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const auto sw = __builtin_amdgcn_permlane32_swap(
                __float_as_uint(acc[2 * k]), __float_as_uint(acc[2 * k + 1]), false, false);
            acc[2 * k] = __uint_as_float(sw[0]) + __uint_as_float(sw[1]);
        }
    } else {
#pragma unroll
        for (int off = 32; off >= LW; off >>= 1) {
#pragma unroll
            for (int cc = 0; cc < 16; ++cc) acc[cc] += __shfl_xor(acc[cc], off, 64);
        }
    }
}

// SED of a tile of TC cells (a multiple of 16) over the blocks of
// LW = 64 / ROWS wavelengths lb_first, lb_first + lb_step, ... < lb_end of
// the calling wave, from the tile's LDS (sInvT [TC][Sp], then sChunk [Sp/8][TC]
// and sPair [Sp/16][TC] as fill_chunk_min writes them).
// Row r of the wave stores the cells cc with cc mod ROWS = r.
template <int ROWS, int TC, bool TAIL>
__device__ __forceinline__ void emit_tile(const PlanView& v, int64_t c0, int64_t C,
                                          const float* __restrict__ m, float* __restrict__ L,
                                          int64_t ldl, const float* sInvT, const uint32_t* sChunk,
                                          int lb_first, int lb_step, int lb_end) {
    static_assert(TC % 16 == 0, "cells per tile must be a multiple of 16");
    constexpr int LW = 64 / ROWS;
    const int lane = threadIdx.x & 63;
    const int r = lane / LW;
    const uint32_t* sPair = sChunk + (v.Sp / EMIT_GROUP) * TC;
    for (int lb = lb_first; lb < lb_end; lb += lb_step) {
        const int l = lb * LW + (lane % LW);
#pragma unroll 1
        for (int h = 0; h < TC; h += 16) {
            float acc[16];
            emit_block<ROWS, TC, TAIL>(v, lb, sInvT + h * v.Sp, sChunk + h, sPair + h, acc);
            if (l >= v.NL) continue;
            if constexpr (ROWS == 2) {
                // row r holds the sum of cell 2k + r in acc[2k]; the two cells'
                // masses are wave-uniform loads (clamped to the last cell)
                const int64_t cb = c0 + h;
                float* Lp = L + (cb + r) * ldl + l;  // cell cb + r; cells 2k further on
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const int64_t ce = cb + 2 * k < C ? cb + 2 * k : C - 1;
                    const int64_t co = cb + 2 * k + 1 < C ? cb + 2 * k + 1 : C - 1;
                    const float me = m ? m[ce] : 1.0f, mo = m ? m[co] : 1.0f;
                    if (cb + 2 * k + r < C)
                        Lp[2 * k * ldl] = acc[2 * k] * ((r ? mo : me) * v.escale);
                }
            } else {
                // a branch per row keeps the accumulator indices static
#pragma unroll
                for (int rr = 0; rr < ROWS; ++rr) {
                    if (r != rr) continue;
#pragma unroll
                    for (int k = 0; k < 16 / ROWS; ++k) {
                        const int64_t c = c0 + h + ROWS * k + rr;
                        if (c < C)
                            L[c * ldl + l] = acc[ROWS * k + rr] * ((m ? m[c] : 1.0f) * v.escale);
                    }
                }
            }
        }
    }
}

}  // namespace dust
