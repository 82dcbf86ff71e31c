/*
 * fluct_ref.c -- plain FP64 CPU oracle of thermally fluctuating grains
 * (test infrastructure only; see dust_ref.h).
 *
 * The paper (Section 2, and its discussion of future work in Section 6)
 * names the calculation for grains too small to hold an equilibrium
 * temperature: per cell and grain, the probability distribution over the
 * grain's temperature levels, which takes solving a linear system built from
 * the full matrix of transitions between the levels (the transition-matrix
 * method of the work it cites, Guhathakurta & Draine 1989), and the emission
 * averaged over that distribution.  The paper gives no algorithm of its own;
 * this file follows that method in its continuous-cooling form, step by step:
 *
 *   levels      E_0 = 0 < E_1 < ... < E_{M-1} (grain enthalpy, J) at
 *               temperatures T_0 = 0 < T_1 < ... (caller-supplied: they come
 *               from the grain's heat capacity, which is not a paper input);
 *   heating     a photon of wavelength bin l has energy eps_l = h c / lam_l
 *               and arrives at rate R_l = J_l C_l dlam_l / eps_l (the energy
 *               rate of Eq. 6 counted in photons; the common factor 4 pi of
 *               heating and cooling is dropped as in Eq. 7).  From level i it
 *               lifts the grain to E = E_i + eps_l, shared between the two
 *               levels around E in proportion to linear interpolation, so
 *               that the mean energy gained is eps_l; above the top level it
 *               goes to the top level;
 *   cooling     from level j > 0 only to level j - 1, at the rate that drains
 *               the grain's radiated power (the sum of Eq. 7 at T_j):
 *               A[j-1][j] = P(T_j) / (E_j - E_{j-1});
 *   steady      sum_i A[f][i] X_i = X_f sum_k A[k][f] for every f; with
 *   state       cooling one level at a time the balance of the flux across
 *               the boundary below level j gives X_j exactly from the levels
 *               under it:  X_j A[j-1][j] = sum_{i<j} X_i sum_{f>=j} A[f][i];
 *               X_0 = 1 and P = X / sum X;
 *   emission    L[c,l] = m[c] sum_s w_s C[s,l] sum_j P[c,s,j] B(lam_l, T_j)
 *               (Eq. 10 averaged over the distribution).
 *
 * One function per step; no blocking, no fusion.  The loops over cells run
 * under OpenMP, which changes no arithmetic.
 */
#include <math.h>
#include <stdlib.h>

#include "dust_ref.h"

static const double PLANCK_H = 6.62607015e-34;
static const double LIGHT_C = 299792458.0;

/* Photon rates R_l of one (cell, grain) pair. */
static void photon_rates(int32_t NL, const double* lam, const double* dlam, const double* c_row,
                         const double* J, double* R)
{
    for (int32_t l = 0; l < NL; ++l) {
        double eps = PLANCK_H * LIGHT_C / lam[l];
        R[l] = J[l] * c_row[l] * dlam[l] / eps;
    }
}

/* Largest f with E[f] <= e (E ascending, E[0] <= e). */
static int32_t level_below(int32_t M, const double* E, double e)
{
    int32_t lo = 0, hi = M - 1;
    while (lo < hi) {
        int32_t mid = (lo + hi + 1) / 2;
        if (E[mid] <= e) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

/* Upward rates A[f*M + i] (f > i) of one pair: every photon from every level,
 * split between the two levels around its landing energy. */
static void upward_rates(int32_t NL, int32_t M, const double* lam, const double* E,
                         const double* R, double* A)
{
    for (int32_t k = 0; k < M * M; ++k) A[k] = 0.0;
    for (int32_t i = 0; i < M - 1; ++i) {
        for (int32_t l = 0; l < NL; ++l) {
            double eps = PLANCK_H * LIGHT_C / lam[l];
            double e = E[i] + eps;
            if (e >= E[M - 1]) {
                A[(M - 1) * M + i] += R[l];
                continue;
            }
            int32_t f = level_below(M, E, e);
            double w = (e - E[f]) / (E[f + 1] - E[f]);
            if (f > i) A[f * M + i] += (1.0 - w) * R[l];
            A[(f + 1) * M + i] += w * R[l];
        }
    }
}

void dust_ref_fluct_pair(int32_t NL, int32_t M, const double* lam, const double* dlam,
                         const double* c_row, const double* lev_T, const double* lev_E,
                         const double* J, double* P)
{
    int bad = 0;
    for (int32_t l = 0; l < NL; ++l)
        if (!(J[l] >= 0.0) || isinf(J[l])) bad = 1;
    if (bad) {
        for (int32_t j = 0; j < M; ++j) P[j] = NAN;
        return;
    }
    double* R = (double*)malloc(sizeof(double) * (size_t)NL);
    double* A = (double*)malloc(sizeof(double) * (size_t)M * (size_t)M);
    double* X = (double*)malloc(sizeof(double) * (size_t)M);
    photon_rates(NL, lam, dlam, c_row, J, R);
    upward_rates(NL, M, lam, lev_E, R, A);
    /* cooling, one level down */
    for (int32_t j = 1; j < M; ++j)
        A[(j - 1) * M + j] = dust_ref_grain_power(NL, lam, dlam, c_row, lev_T[j]) /
                             (lev_E[j] - lev_E[j - 1]);
    /* the flux balance across each level boundary, level by level upwards */
    X[0] = 1.0;
    for (int32_t j = 1; j < M; ++j) {
        double up = 0.0;
        for (int32_t i = 0; i < j; ++i) {
            double Bji = 0.0;
            for (int32_t f = j; f < M; ++f) Bji += A[f * M + i];
            up += Bji * X[i];
        }
        X[j] = up / A[(j - 1) * M + j];
        if (X[j] > 0x1p500) /* keep the running values in range (exact: P is a ratio) */
            for (int32_t i = 0; i <= j; ++i) X[i] = ldexp(X[i], -500);
    }
    double total = 0.0;
    for (int32_t j = 0; j < M; ++j) total += X[j];
    for (int32_t j = 0; j < M; ++j) P[j] = X[j] / total;
    free(R);
    free(A);
    free(X);
}

void dust_ref_fluct_distribution(int64_t n_cells, int32_t NL, int32_t S, int32_t M,
                                 const double* lam, const double* dlam, const double* c_abs,
                                 const double* lev_T, const double* lev_E, const double* J,
                                 int64_t ldj, double* P)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t c = 0; c < n_cells; ++c)
        for (int32_t s = 0; s < S; ++s)
            dust_ref_fluct_pair(NL, M, lam, dlam, c_abs + (int64_t)s * NL,
                                lev_T + (int64_t)s * M, lev_E + (int64_t)s * M, J + c * ldj,
                                P + (c * S + s) * M);
}

void dust_ref_fluct_emission(int64_t n_cells, int32_t NL, int32_t S, int32_t M,
                             const double* lam, const double* c_abs, const double* weight,
                             const double* lev_T, const double* m_dust, const double* P,
                             double* L)
{
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < n_cells; ++c) {
        double m = m_dust ? m_dust[c] : 1.0;
        for (int32_t l = 0; l < NL; ++l) {
            double sum = 0.0;
            for (int32_t s = 0; s < S; ++s) {
                double avg = 0.0;
                for (int32_t j = 0; j < M; ++j)
                    avg += P[(c * S + s) * M + j] *
                           dust_ref_planck(lam[l], lev_T[(int64_t)s * M + j]);
                sum += weight[s] * c_abs[(int64_t)s * NL + l] * avg;
            }
            L[c * NL + l] = m * sum;
        }
    }
}
