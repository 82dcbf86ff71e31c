// Internal declarations of libdust (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "dust.h"

namespace dust {

// Padding of the kernel tables.  Wavelengths pad to the K depth of one
// bf16 MFMA step (16x16x32); grains pad to the MFMA N width.
constexpr int PAD_L = 32;
constexpr int PAD_S = 16;

// Exact SI constants (2019 SI) and the derived radiation constants.
constexpr double PLANCK_H = 6.62607015e-34;
constexpr double LIGHT_C = 299792458.0;
constexpr double BOLTZ_K = 1.380649e-23;
constexpr double RAD_C1 = 2.0 * PLANCK_H * LIGHT_C * LIGHT_C;  // 2 h c^2
constexpr double RAD_C2 = PLANCK_H * LIGHT_C / BOLTZ_K;        // h c / k
constexpr double LOG2E = 1.4426950408889634;
constexpr double LN2 = 0.6931471805599453;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Everything a kernel needs from a plan, passed by value.
struct PlanView {
    int NL, S, NLp, Sp;
    int mode;
    int maxit;
    float tol;
    // wavelength tables [NLp]
    const float* nu;       // -c2 log2(e) / lam  (0 on padding)
    // per-grain tables [Sp]
    const float* hscale;   // 2^es: H' = H * hscale (exact)
    const float* hinv;     // 2^-es
    const float* gs;       // Eq. 11 offset: log10 of 4 pi 2^-es, plus the size terms
    // [Sp][NLp] tables
    const float* kf;       // K' = C dlam 2^es (FP32), fragment order (kfrag_f32)
    const __bf16* khi;     // bf16(K'), fragment order (kfrag_bf16)
    const __bf16* klo;     // bf16(K' - khi), fragment order
    const float* kb;       // K' c1 lam^-5 (FP32): the solve's Planck weights
    const float* ku;       // kb * c2 log2(e) / lam: weights of the solve's slope
    const float* em;       // w C c1 lam^-5 2^-ge (FP32): the emission weights
    float escale;          // 2^ge
    // float64 tables of the mixed solve
    const double* kdb;     // [S][NL] K' c1 lam^-5 (FP64): exact power weights
    const double* c2l;     // [NL] c2 / lam (FP64)
    const double* fwd;     // [S][N] y_k = ln P'(T_k), T_k = exp(lnTmin + k hstep)
    const double* ylo;     // [S] y_0
    const double* yhi;     // [S] y_{N-1}
    const double* dyinv;   // [S] (M - 1) / (yhi - ylo)
    // inverse table ln T(y) at M uniform steps of y, computed in FP64 from
    // the forward table: node j holds (ln T_j, m_j), m = dy d ln T / dy
    const double2* invd;   // [S][M] FP64 nodes (default mixed lookup)
    // the same in FP32, per interval j (ln T_j, m_j, ln T_{j+1}, m_{j+1}) in
    // one 16-byte entry (the FP32 lookup)
    const float4* invf;    // [S][M-1]
    const float* ylof;     // [S] float(ylo)
    const float* dyinvf;   // [S] float(dyinv)
    int f32_lookup;        // mixed: FP32 inverse-table lookup instead of the FP64 one
    int polish;            // mixed: FP64 Newton polish on the forward table after the lookup
    int N, M;
    double lnTmin, hstep;  // ln T_k = lnTmin + k hstep
    const double* texp;    // [N] T_k: exp(lnTmin + k hstep) (mixed),
                           //      tmin + k tstep (table-linear)
    const double2* lntab;  // [256] (ln c_i, 1 / c_i), c_i = 1 + i / 256
    // table-linear: fwd holds P'_s(T_k) itself; ylo/yhi/dyinv describe
    // M uniform nodes in ln P' and kidx[s][j] the last table point whose
    // ln P' is <= node j (a bracket for the search)
    const int* kidx;       // [S][M]
    double tstep;          // T_{k+1} - T_k
    // Per-call inputs of the temperature step (dust_solve_ext); zero in the
    // plan's own copy.
    const float* q;        // [C][ldq] extra heating (unscaled units of H), or null
    int64_t ldq;
    int warm;              // plain: start Newton from the T already in the output
};

// Positions of K'[s][l] (s < Sp, l < NLp) in the fragment-ordered weight
// tables.  Grain tile t = s / 16, k-step j = l / 32; the 64 lanes of a wave
// (lane = 16 q + row) hold row s = 16 t + row and wavelengths
// 32 j + 8 q .. 32 j + 8 q + 7.  bf16: 8 values per lane, one fragment of
// 64 x 8 values per (t, j).  FP32: the same 8 values as two halves of 4, each
// half a contiguous 64 x 4 block.
__host__ __device__ inline int64_t kfrag_bf16(const PlanView& v, int s, int l) {
    const int t = s >> 4, row = s & 15, j = l >> 5, q = (l >> 3) & 3, e = l & 7;
    return (((int64_t)t * (v.NLp >> 5) + j) * 64 + (q * 16 + row)) * 8 + e;
}
__host__ __device__ inline int64_t kfrag_f32(const PlanView& v, int s, int l) {
    const int t = s >> 4, row = s & 15, j = l >> 5, q = (l >> 3) & 3, e = l & 7;
    return ((((int64_t)t * (v.NLp >> 5) + j) * 2 + (e >> 2)) * 64 + (q * 16 + row)) * 4 + (e & 3);
}

}  // namespace dust

struct dust_plan {
    int device;
    dust_options opt;
    int NL, S, NLp, Sp;
    int N, M;
    double lnTmin, hstep;
    int ge;
    // device float64 copies of the grid
    double *d_lam, *d_dlam, *d_cabs, *d_w, *d_size;
    int* d_es;
    // derived device tables
    float *d_nu, *d_hscale, *d_hinv, *d_gs, *d_kf, *d_kb, *d_ku, *d_em;
    __bf16 *d_khi, *d_klo;
    double *d_kdb, *d_c2l, *d_ylo, *d_yhi, *d_dyinv, *d_fwd, *d_texp;
    double2* d_lntab;
    double2* d_invd;
    float4* d_invf;
    float *d_ylof, *d_dyinvf;
    int* d_kidx;  // table-linear search brackets [S][M]
    dust::PlanView view;
};

namespace dust {

// Thread-local error text; returns `code` for convenience.
dust_status set_error(dust_status code, const std::string& msg);
// Clears the calling thread's last error (every entry point starts with it).
void clear_error();
dust_status hip_error(hipError_t e, const char* what);

// Kernel launchers (each in its own translation unit).
hipError_t launch_prepare(const dust_plan* p, hipStream_t st);

// Everything the four refresh stages of one plan read and write, with each
// stage's grid (gx, gy; gy = 0 where the plan has no such stage).
struct RefreshJob {
    PlanView v;
    const double *lam, *dlam, *cabs, *w;
    const int* es;
    int ge;
    float *nu, *kf, *kb, *ku, *em;
    __bf16 *khi, *klo;
    double *kdb, *c2l, *fwd, *ylo, *yhi, *dyinv;
    int* kidx;
    double2* invd;
    float2* invf;
    float *ylof, *dyinvf;
    int gx[4], gy[4];
};
void make_refresh_job(const dust_plan* p, RefreshJob* j);
// The refresh of many plans as four launches (one per stage); d_starts[k]
// holds, per plan, the first block of its range in stage k (ascending).
hipError_t launch_prepare_batched(const RefreshJob* d_jobs, const int* const d_starts[4],
                                  int n_jobs, const int blocks[4], hipStream_t st);
hipError_t launch_absorb(const PlanView& v, int64_t C, const float* J, int64_t ldj,
                         float* H, int64_t ldh, hipStream_t st);
hipError_t launch_solve(const PlanView& v, int64_t C, const float* H, int64_t ldh,
                        float* T, int64_t ldt, dust_counters* cnt, hipStream_t st);
// Kernel forms: the public modes, plus the mixed mode with the FP32
// inverse-table lookup in place of the FP64 one (a separate instantiation,
// so that it carries none of the FP64 code and registers).
constexpr int MODE_MIXED_F32 = 3;
// The default mixed lookup followed by the FP64 Newton polish on the forward
// table (dust_options.newton_polish).
constexpr int MODE_MIXED_POLISH = 4;
// Forms whose heating runs on bf16 hi+lo MFMA and whose T comes from a table.
__host__ __device__ constexpr bool table_mode(int mode) { return mode != DUST_PLAIN_FP32; }
__host__ __device__ constexpr bool mixed_mode(int mode) {
    return mode == DUST_MIXED || mode == MODE_MIXED_F32 || mode == MODE_MIXED_POLISH;
}
inline int kernel_mode(const PlanView& v) {
    if (v.mode == DUST_MIXED && v.f32_lookup) return MODE_MIXED_F32;
    if (v.mode == DUST_MIXED && v.polish) return MODE_MIXED_POLISH;
    return v.mode;
}
hipError_t launch_emit(const PlanView& v, int64_t C, const float* T, int64_t ldt,
                       const float* m, float* L, int64_t ldl, hipStream_t st);
hipError_t launch_absorb_solve(const PlanView& v, int64_t C, const float* J, int64_t ldj,
                               float* T, int64_t ldt, dust_counters* cnt, hipStream_t st);
hipError_t launch_fused(const PlanView& v, int64_t C, const float* J, int64_t ldj,
                        const float* m, float* T, int64_t ldt, float* L, int64_t ldl,
                        dust_counters* cnt, hipStream_t st);

}  // namespace dust
