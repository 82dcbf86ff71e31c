/*
 * dust_ref.c -- plain FP64 CPU oracle (test infrastructure only; see
 * dust_ref.h).  Written for a reader checking it against the paper by eye:
 * one function per equation, no blocking, no fusion, no reordering.
 * The loops over cells run under OpenMP; that changes no arithmetic.
 */
#include "dust_ref.h"

#include <float.h>
#include <math.h>
#include <stddef.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* Exact SI constants (2019 redefinition of the SI). */
static const double PLANCK_H = 6.62607015e-34;  /* J s   */
static const double LIGHT_C = 299792458.0;      /* m/s   */
static const double BOLTZ_K = 1.380649e-23;     /* J/K   */

/* Fit constants of the initial guess, Section 4.3, Eq. 11. */
static const double GUESS_K = 1.86;
static const double GUESS_B1 = 0.189;
static const double GUESS_B2 = 3.41e-3;
static const double GUESS_A1 = -1.39;
static const double GUESS_A2 = 0.126;
static const double GUESS_FLOOR_K = 5.0; /* Section 4.3: guesses below 5 K use 5 K */

#define ORACLE_MAX_EVALS 400

/* B_lambda(lam, T) = 2 h c^2 / lam^5 / (exp(h c / (k lam T)) - 1)   (Eq. 1) */
double dust_ref_planck(double lam, double T)
{
    if (!(T > 0.0)) return (T == 0.0) ? 0.0 : NAN;
    double x = PLANCK_H * LIGHT_C / (BOLTZ_K * lam * T);
    double em1 = expm1(x);
    if (isinf(em1)) return 0.0;
    double lam5 = lam * lam * lam * lam * lam;
    return 2.0 * PLANCK_H * LIGHT_C * LIGHT_C / lam5 / em1;
}

/* dB/dT = B * x e^x / ((e^x - 1) T),  x = h c / (k lam T) */
double dust_ref_planck_dT(double lam, double T)
{
    if (!(T > 0.0)) return 0.0;
    double x = PLANCK_H * LIGHT_C / (BOLTZ_K * lam * T);
    double em1 = expm1(x);
    if (isinf(em1)) return 0.0;
    double b = dust_ref_planck(lam, T);
    return b * x * ((em1 + 1.0) / em1) / T;
}

/* Power radiated by one grain at temperature T: right side of Eq. 7. */
double dust_ref_grain_power(int32_t NL, const double* lam, const double* dlam,
                            const double* c_row, double T)
{
    double sum = 0.0;
    for (int32_t l = 0; l < NL; ++l)
        sum += c_row[l] * dlam[l] * dust_ref_planck(lam[l], T);
    return sum;
}

static double grain_power_dT(int32_t NL, const double* lam, const double* dlam,
                             const double* c_row, double T)
{
    double sum = 0.0;
    for (int32_t l = 0; l < NL; ++l)
        sum += c_row[l] * dlam[l] * dust_ref_planck_dT(lam[l], T);
    return sum;
}

/* Eq. 11 (Section 4.3). */
double dust_ref_guess(double lh_watt, double a_m)
{
    if (!(lh_watt > 0.0) || !(a_m > 0.0)) return GUESS_FLOOR_K;
    double la = log10(a_m);
    double x = log10(lh_watt) + GUESS_A1 * la + GUESS_A2 * la * la;
    double logt = GUESS_K + GUESS_B1 * x + GUESS_B2 * x * x;
    double t = pow(10.0, logt);
    return (t < GUESS_FLOOR_K) ? GUESS_FLOOR_K : t;
}

/* Eq. 6: the heating of grain s in cell c, summed in ascending wavelength
 * with Neumaier's compensated summation (a running correction term carries
 * the low-order bits each addition drops, whichever operand is larger), so
 * that the sum is correct to about one rounding whatever the spread of the
 * terms. */
void dust_ref_heating(int64_t n_cells, int32_t NL, int32_t S,
                      const double* J, int64_t ldj, const double* c_abs,
                      const double* dlam, double* H)
{
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < n_cells; ++c) {
        for (int32_t s = 0; s < S; ++s) {
            double sum = 0.0, comp = 0.0;
            for (int32_t l = 0; l < NL; ++l) {
                double term = J[c * ldj + l] * c_abs[(int64_t)s * NL + l] * dlam[l];
                double t = sum + term;
                if (fabs(sum) >= fabs(term)) comp += (sum - t) + term;
                else comp += (term - t) + sum;
                sum = t;
            }
            H[c * S + s] = sum + comp;
        }
    }
}

/*
 * Eq. 7 for one (cell, grain) pair.  F(T) = P(T) - H with P the grain power
 * is strictly increasing from -H (T -> 0) to +infinity, so for H > 0 it has
 * exactly one root.  Newton's method from the Eq. 11 guess, taken on the
 * equivalent equation ln P(T) = ln H in the variable ln T (same root; the
 * log-log form is close to linear, so it needs few steps), safeguarded by a
 * bracket [lo, hi] with F(lo) < 0 < F(hi): a step that leaves the bracket is
 * replaced by doubling (upper end still unknown) or a geometric bisection.
 * Stops when the step falls below 4 units of the last place or the bracket
 * closes.
 */
static double solve_pair(double H, double a, int32_t NL, const double* lam,
                         const double* dlam, const double* c_row, int32_t* evals)
{
    *evals = 0;
    if (isnan(H) || isinf(H) || H < 0.0) return NAN;
    if (H == 0.0) return 0.0;

    double T = dust_ref_guess(4.0 * M_PI * H, a);
    double lo = 0.0, hi = INFINITY;
    for (int32_t it = 1; it <= ORACLE_MAX_EVALS; ++it) {
        double P = dust_ref_grain_power(NL, lam, dlam, c_row, T);
        double dF = grain_power_dT(NL, lam, dlam, c_row, T);
        double F = P - H;
        *evals = it;
        if (F == 0.0) return T;
        if (F < 0.0) lo = T;
        else hi = T;

        double Tn = NAN;
        if (P > 0.0 && dF > 0.0)
            Tn = T * exp(log(H / P) * P / (T * dF));
        if (fabs(Tn - T) <= 4.0 * DBL_EPSILON * T) return Tn;
        if (!(Tn > lo && Tn < hi)) {
            if (isinf(hi)) Tn = 2.0 * lo;
            else if (lo > 0.0) Tn = sqrt(lo * hi);
            else Tn = 0.5 * hi;
        }

        if (!isinf(hi) && hi - lo <= 4.0 * DBL_EPSILON * hi) return 0.5 * (lo + hi);
        T = Tn;
    }
    return T;
}

void dust_ref_temperature(int64_t n_cells, int32_t NL, int32_t S,
                          const double* lam, const double* dlam,
                          const double* c_abs, const double* size,
                          const double* H, double* T, int32_t* iters)
{
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t c = 0; c < n_cells; ++c) {
        for (int32_t s = 0; s < S; ++s) {
            int32_t evals;
            T[c * S + s] = solve_pair(H[c * S + s], size[s], NL, lam, dlam,
                                      c_abs + (int64_t)s * NL, &evals);
            if (iters) iters[c * S + s] = evals;
        }
    }
}

/* Eqs. 9-10: the SED of cell c summed over grains, times the dust mass. */
void dust_ref_emission(int64_t n_cells, int32_t NL, int32_t S,
                       const double* lam, const double* c_abs,
                       const double* weight, const double* m_dust,
                       const double* T, double* L)
{
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < n_cells; ++c) {
        double md = m_dust ? m_dust[c] : 1.0;
        for (int32_t l = 0; l < NL; ++l) {
            double sum = 0.0;
            for (int32_t s = 0; s < S; ++s)
                sum += weight[s] * c_abs[(int64_t)s * NL + l] *
                       dust_ref_planck(lam[l], T[c * S + s]);
            L[c * NL + l] = md * sum;
        }
    }
}

/*
 * The production variant of the temperature step (Sections 2 and 5): per
 * grain, the power P_s(T_k) of Eq. 7 at n_T temperatures evenly spaced from
 * t_min to t_max, T_k = t_min + k (t_max - t_min) / (n_T - 1).
 */
void dust_ref_table_build(int32_t NL, int32_t S, const double* lam,
                          const double* dlam, const double* c_abs,
                          int32_t n_T, double t_min, double t_max, double* P)
{
    const double step = (t_max - t_min) / (double)(n_T - 1);
#pragma omp parallel for schedule(static)
    for (int32_t s = 0; s < S; ++s)
        for (int32_t k = 0; k < n_T; ++k)
            P[(int64_t)s * n_T + k] =
                dust_ref_grain_power(NL, lam, dlam, c_abs + (int64_t)s * NL,
                                     t_min + k * step);
}

/*
 * T(H) from the table by linear interpolation between the two table points
 * whose powers bracket H: P_k <= H < P_{k+1} gives
 *   T = T_k + (H - P_k) / (P_{k+1} - P_k) * (T_{k+1} - T_k).
 * H = 0 gives 0; H < 0 or non-finite gives NaN.  H below the table gives
 * t_min and H above it t_max; those pairs are counted (return value).
 */
int64_t dust_ref_table_temperature(int64_t n_cells, int32_t S, int32_t n_T,
                                   double t_min, double t_max, const double* P,
                                   const double* H, double* T)
{
    const double step = (t_max - t_min) / (double)(n_T - 1);
    int64_t clamped = 0;
#pragma omp parallel for schedule(static) reduction(+:clamped)
    for (int64_t c = 0; c < n_cells; ++c) {
        for (int32_t s = 0; s < S; ++s) {
            const double h = H[c * S + s];
            const double* row = P + (int64_t)s * n_T;
            double t;
            if (isnan(h) || isinf(h) || h < 0.0) {
                t = NAN;
            } else if (h == 0.0) {
                t = 0.0;
            } else if (h < row[0]) {
                t = t_min;
                ++clamped;
            } else if (h >= row[n_T - 1]) {
                t = t_max;
                if (h > row[n_T - 1]) ++clamped;
            } else {
                int32_t lo = 0, hi = n_T - 1;   /* row[lo] <= h < row[hi] */
                while (hi - lo > 1) {
                    const int32_t mid = lo + (hi - lo) / 2;
                    if (row[mid] <= h) lo = mid;
                    else hi = mid;
                }
                t = (t_min + lo * step) + (h - row[lo]) / (row[lo + 1] - row[lo]) * step;
            }
            T[c * S + s] = t;
        }
    }
    return clamped;
}

int dust_ref_get_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void dust_ref_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
