/*
 * Driver of the C oracle for a sanitizer build (AddressSanitizer and
 * UndefinedBehaviorSanitizer, host only): every entry point of dust_ref.h on
 * a small synthetic problem, with invariants checked, so that an
 * out-of-bounds access, a use of freed memory, a leak or undefined
 * arithmetic anywhere in the oracle fails the run.  Built and run by
 * tests/test_oracle_sanitize.py.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "dust_ref.h"

#define NL 64
#define S 5
#define C 7
#define M 24

static int fail(const char* what)
{
    fprintf(stderr, "oracle sanitize driver: %s\n", what);
    return 1;
}

int main(void)
{
    double lam[NL], dlam[NL], cabs[S * NL], w[S], a[S];
    const double h = 6.62607015e-34, c = 299792458.0, k = 1.380649e-23;
    double dln = log(1000.0 / 0.09) / (NL - 1);
    for (int l = 0; l < NL; ++l) {
        lam[l] = 0.09e-6 * exp(l * dln);
        dlam[l] = lam[l] * dln * ((l == 0 || l == NL - 1) ? 0.5 : 1.0);
    }
    for (int s = 0; s < S; ++s) {
        a[s] = 1e-9 * pow(10.0, 0.6 * s);
        w[s] = 1.0 / (s + 1.0);
        for (int l = 0; l < NL; ++l) {
            double x = 2.0 * M_PI * a[s] / lam[l];
            cabs[s * NL + l] = M_PI * a[s] * a[s] * (-expm1(-1.0 * pow(x, 1.5)));
        }
    }
    double J[C * NL], m[C];
    for (int ci = 0; ci < C; ++ci) {
        double Ts = 5000.0 + 3000.0 * ci, W = pow(10.0, -14.0 + 0.5 * ci);
        m[ci] = 1.0 + ci;
        for (int l = 0; l < NL; ++l)
            J[ci * NL + l] = W * 2.0 * h * c * c / pow(lam[l], 5) / expm1(h * c / (k * lam[l] * Ts));
    }
    double* H = malloc(sizeof(double) * C * S);
    double* T = malloc(sizeof(double) * C * S);
    double* L = malloc(sizeof(double) * C * NL);
    int32_t* it = malloc(sizeof(int32_t) * C * S);
    dust_ref_heating(C, NL, S, J, NL, cabs, dlam, H);
    dust_ref_temperature(C, NL, S, lam, dlam, cabs, a, H, T, it);
    dust_ref_emission(C, NL, S, lam, cabs, w, m, T, L);
    int bad = 0;
    for (int ci = 0; ci < C; ++ci) {
        double lhs = 0.0, rhs = 0.0;
        for (int l = 0; l < NL; ++l) lhs += L[ci * NL + l] * dlam[l];
        for (int s = 0; s < S; ++s) {
            double P = dust_ref_grain_power(NL, lam, dlam, cabs + s * NL, T[ci * S + s]);
            if (!(fabs(P / H[ci * S + s] - 1.0) < 1e-12)) bad |= fail("balance of Eq. 7");
            rhs += m[ci] * w[s] * H[ci * S + s];
        }
        if (!(fabs(lhs / rhs - 1.0) < 1e-12)) bad |= fail("SED energy identity");
    }
    /* the production table */
    double* Ptab = malloc(sizeof(double) * S * 200);
    double* Tt = malloc(sizeof(double) * C * S);
    dust_ref_table_build(NL, S, lam, dlam, cabs, 200, 3.0, 1500.0, Ptab);
    (void)dust_ref_table_temperature(C, S, 200, 3.0, 1500.0, Ptab, H, Tt);
    for (int i = 0; i < C * S; ++i)
        if (!(Tt[i] <= T[i] * (1.0 + 1e-12) || Tt[i] == 3.0 || Tt[i] == 1500.0))
            bad |= fail("table temperature above the root");
    /* fluctuating grains */
    double levT[S * M], levE[S * M];
    for (int s = 0; s < S; ++s) {
        levT[s * M] = 0.0;
        levE[s * M] = 0.0;
        for (int j = 1; j < M; ++j) {
            levT[s * M + j] = 2.0 * pow(2500.0 / 2.0, (j - 1.0) / (M - 2.0));
            levE[s * M + j] = 1e-24 * pow(10.0, 0.3 * s) * pow(levT[s * M + j], 4.0) /
                              (1.0 + pow(levT[s * M + j] / 300.0, 3.0));
        }
    }
    double* P = malloc(sizeof(double) * C * S * M);
    double* Lf = malloc(sizeof(double) * C * NL);
    dust_ref_fluct_distribution(C, NL, S, M, lam, dlam, cabs, levT, levE, J, NL, P);
    dust_ref_fluct_emission(C, NL, S, M, lam, cabs, w, levT, m, P, Lf);
    for (int i = 0; i < C * S; ++i) {
        double sum = 0.0;
        for (int j = 0; j < M; ++j) sum += P[i * M + j];
        if (!(fabs(sum - 1.0) < 1e-12)) bad |= fail("distribution sums to one");
    }
    for (int i = 0; i < C * NL; ++i)
        if (!(Lf[i] >= 0.0)) bad |= fail("averaged emission non-negative");
    free(H); free(T); free(L); free(it); free(Ptab); free(Tt); free(P); free(Lf);
    if (!bad) printf("oracle sanitize driver: ok\n");
    return bad;
}
