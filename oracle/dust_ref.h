/*
 * dust_ref.h -- plain FP64 CPU oracle for the dust equilibrium-temperature
 * and emission calculation of Jonsson & Primack, "Accelerating Dust
 * Temperature Calculations with Graphics Processing Units" (New Astronomy).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes
 * or calls this code; it shares no source, header, table or constant with
 * the GPU path.  Only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark use it.
 *
 * What it computes (Section 4, Eqs. 6-10), all in IEEE double precision:
 *   heating      H[c,s] = sum_l J[c,l] * C[s,l] * dlam[l]                (Eq. 6)
 *   temperature  T[c,s] = the unique root of
 *                sum_l C[s,l] dlam[l] B(lam_l, T) = H[c,s]                (Eq. 7)
 *   emission     L[c,l] = m[c] * sum_s w[s] C[s,l] B(lam_l, T[c,s])       (Eqs. 8-10)
 * with the Planck function B(lam,T) = 2hc^2 lam^-5 / (exp(hc/(k lam T)) - 1)
 * (Eq. 1) and the exact SI values of h, c and k.
 *
 * J is the mean intensity; the heating and emission sums carry no 4 pi (both
 * sides of the balance drop the same factor, so T is unaffected).  The only
 * place 4 pi appears is the initial-guess fit of Eq. 11, whose L_h is read
 * as a luminosity in watts (4 pi H) with the grain size in metres and
 * base-10 logarithms.
 *
 * Arrays are row-major.  Sizes: C cells, NL wavelengths, S grains.
 * No function allocates on behalf of the caller; all are thread-safe.
 */
#ifndef DUST_REF_H
#define DUST_REF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Planck function B_lambda(lam [m], T [K]) in W m^-2 m^-1 sr^-1 (Eq. 1).
 * T <= 0 gives 0; an exponent too large for double gives 0. */
double dust_ref_planck(double lam, double T);

/* dB/dT at (lam, T); 0 where B underflows. */
double dust_ref_planck_dT(double lam, double T);

/* Right-hand side of Eq. 7 for one grain: sum_l C[l] dlam[l] B(lam_l, T). */
double dust_ref_grain_power(int32_t NL, const double* lam, const double* dlam,
                            const double* c_row, double T);

/* Initial guess of Eq. 11: log10 T = k + b1 x + b2 x^2 with
 * x = log10 Lh + a1 log10 a + a2 (log10 a)^2, floored at 5 K.
 * Lh in W, a in m.  Lh <= 0 gives the floor. */
double dust_ref_guess(double lh_watt, double a_m);

/* Eq. 6.  J[c*ldj + l], C[s*NL + l], H[c*S + s]. */
void dust_ref_heating(int64_t n_cells, int32_t NL, int32_t S,
                      const double* J, int64_t ldj, const double* c_abs,
                      const double* dlam, double* H);

/* Eq. 7 solved for every (c,s) to machine precision.
 * H = 0 gives T = 0; H < 0 or non-finite gives NaN.
 * iters (nullable) receives the number of power evaluations per pair. */
void dust_ref_temperature(int64_t n_cells, int32_t NL, int32_t S,
                          const double* lam, const double* dlam,
                          const double* c_abs, const double* size,
                          const double* H, double* T, int32_t* iters);

/* Eqs. 9-10.  m_dust may be NULL (all ones).  L[c*NL + l]. */
void dust_ref_emission(int64_t n_cells, int32_t NL, int32_t S,
                       const double* lam, const double* c_abs,
                       const double* weight, const double* m_dust,
                       const double* T, double* L);

/* Production variant of the temperature step (Sections 2 and 5): the table
 * P[s*n_T + k] = grain power of grain s at T_k = t_min + k (t_max - t_min) /
 * (n_T - 1), n_T >= 2. */
void dust_ref_table_build(int32_t NL, int32_t S, const double* lam,
                          const double* dlam, const double* c_abs,
                          int32_t n_T, double t_min, double t_max, double* P);

/* T[c*S + s] by linear interpolation in that table between the two points
 * that bracket H.  H = 0 gives 0, H < 0 or non-finite NaN; H outside the
 * table gives the end temperature (t_min or t_max).  Returns the number of
 * pairs outside the table. */
int64_t dust_ref_table_temperature(int64_t n_cells, int32_t S, int32_t n_T,
                                   double t_min, double t_max, const double* P,
                                   const double* H, double* T);

/* Thermally fluctuating grains (fluct_ref.c): the steady-state probability
 * distribution over a grain's M >= 2 enthalpy levels (E_0 = 0 < E_1 < ...,
 * temperatures T_0 = 0 < T_1 < ...) under single-photon heating and
 * continuous cooling, and the emission averaged over it.
 * One pair: J[NL] of the cell, c_row[NL] of the grain, lev_T/lev_E[M] of the
 * grain; P[M] receives the distribution (NaN when J holds a negative or
 * non-finite value). */
void dust_ref_fluct_pair(int32_t NL, int32_t M, const double* lam, const double* dlam,
                         const double* c_row, const double* lev_T, const double* lev_E,
                         const double* J, double* P);

/* Every pair: lev_T/lev_E [S][M], J[c*ldj + l], P[(c*S + s)*M + j]. */
void dust_ref_fluct_distribution(int64_t n_cells, int32_t NL, int32_t S, int32_t M,
                                 const double* lam, const double* dlam, const double* c_abs,
                                 const double* lev_T, const double* lev_E, const double* J,
                                 int64_t ldj, double* P);

/* L[c*NL + l] = m[c] sum_s w_s C[s,l] sum_j P[c,s,j] B(lam_l, T_sj); m_dust
 * may be NULL. */
void dust_ref_fluct_emission(int64_t n_cells, int32_t NL, int32_t S, int32_t M,
                             const double* lam, const double* c_abs, const double* weight,
                             const double* lev_T, const double* m_dust, const double* P,
                             double* L);

/* OpenMP thread control (the oracle parallelises over cells only). */
int dust_ref_get_threads(void);
void dust_ref_set_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
