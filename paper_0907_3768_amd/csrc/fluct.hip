// Thermally fluctuating grains (the calculation Sections 2 and 6 name; see
// dust.h): the steady-state probability of every enthalpy level of every
// (cell, grain) pair under single-photon heating and continuous cooling, and
// the emission averaged over it.
//
// Distribution (one wave per pair, FP64).  With photons ordered from the
// shortest wavelength (largest energy eps) on, the upward rate from level i
// to any level >= j is
//   B[j][i] = sum_l R_l clamp((E_i + eps_l - E_{j-1}) / (E_j - E_{j-1}), 0, 1)
// (a photon landing between E_{j-1} and E_j counts with the fraction of it
// shared to level j).  With the prefix sums F0[n] = sum_{l<n} R_l and
// F1[n] = sum_{l<n} R_l eps_l in LDS and n(x) = #{l : eps_l >= x} from a
// per-grain table built with the plan, that is
//   B[j][i] = F0[n2] + ((F1[n1] - F1[n2]) - a (F0[n1] - F0[n2])) / d,
//   a = E_{j-1} - E_i, d = E_j - E_{j-1}, n1 = n(a), n2 = n(a + d):
// two LDS reads and a few FP64 operations per (j, i) instead of a pass over
// the wavelengths.  The flux balance across each level boundary then gives
// the levels one by one, X_j = sum_{i<j} B[j][i] X_i / cool_j: the lanes
// hold the upper levels j and collect their sums as the levels below them
// become final (no wave reduction); the running values are rescaled by exact
// powers of two when they grow large, and P = X / sum X.
//
// Emission: L[c,l] = m_c sum_k P[c,k] Etab[k,l] over k = (grain, level), a
// dense contraction (K = S M) on v_mfma_f32_16x16x4_f32 with a per-grain
// emission table w_s C[s,l] B(lam_l, T_sj) built with the plan.

#include <math.h>
#include <string.h>

#include <string>
#include <vector>

#include "device_common.h"

namespace dust {

dust_status validate_grid(const dust_grid_desc* g);  // api.hip

namespace fluct {

constexpr int MAX_LEVELS = 256;
constexpr int MAX_LDS = 65536;          // bytes of one workgroup's prefix sums
constexpr double TOP_PROBABILITY = 1e-6;  // counted when the top level holds more

struct View {
    int NL, S, M;
    int K, Kp, NLp;       // K = S M; Kp = K rounded up to 32; NLp = NL rounded up to 128
    const double* eps;    // [NL] photon energies h c / lam (J)
    const double* kr;     // [S][NL] C dlam / eps: J times it is the photon rate
    const double* E;      // [S][M] level enthalpies
    const double* rcool;  // [S][M] (E_j - E_{j-1}) / P(T_j): 1 / the cooling rate, 0 at j = 0
    const double* invd;   // [S][M] 1 / (E_j - E_{j-1}), 0 at j = 0
    const int* cnt;       // [S][M][M] cnt[s][i][k] = #{l : eps_l >= E_k - E_i} (NL for k <= i)
    const float* etab;    // [Kp][NLp] w_s C[s,l] B(lam_l, T_sj) 2^-ge, zero padded
    float escale;         // 2^ge
};

__device__ __forceinline__ double wave_sum_f64(double x) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

// ---------------------------------------------------------------------------
// Plan tables.
// ---------------------------------------------------------------------------
struct Prep {
    View v;
    const double *lam, *dlam, *cabs, *w, *T;
    double *eps, *kr, *rcool, *invd;
    int* cnt;
    float* etab;
    int ge;
};

// eps and kr: one thread per (grain, wavelength).
__global__ __launch_bounds__(256) void prep_rates_kernel(Prep p) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= (int64_t)p.v.S * p.v.NL) return;
    const int s = (int)(i / p.v.NL), l = (int)(i - (int64_t)s * p.v.NL);
    const double eps = PLANCK_H * LIGHT_C / p.lam[l];
    if (s == 0) p.eps[l] = eps;
    p.kr[i] = p.cabs[i] * p.dlam[l] / eps;
}

// Cooling rates (their reciprocals): one wave per (grain, level), the grain
// power of Eq. 7 at T_j summed over the wavelengths by the lanes.
__global__ __launch_bounds__(64) void prep_cool_kernel(Prep p) {
    const int s = blockIdx.y, j = blockIdx.x;
    const int M = p.v.M, NL = p.v.NL;
    const double T = p.T[(int64_t)s * M + j];
    double sum = 0.0;
    if (j > 0) {
        const double invT = rcp_f64(T);
        for (int l = threadIdx.x; l < NL; l += 64) {
            const double lam = p.lam[l];
            const double em = expm1_pos(RAD_C2 / lam * invT);
            const double lam2 = lam * lam;
            const double b = (em < __builtin_inf()) ? RAD_C1 / (lam2 * lam2 * lam) / em : 0.0;
            sum += p.cabs[(int64_t)s * NL + l] * p.dlam[l] * b;
        }
    }
    sum = wave_sum_f64(sum);
    if (threadIdx.x == 0) {
        const int64_t o = (int64_t)s * M + j;
        if (j == 0) {
            p.rcool[o] = 0.0;
            p.invd[o] = 0.0;
        } else {
            const double d = p.v.E[o] - p.v.E[o - 1];
            p.rcool[o] = d / sum;  // inf when the level radiates nothing (refused by the host)
            p.invd[o] = 1.0 / d;
        }
    }
}

// Photon counts: one thread per (grain, i, k); eps decreases with l, so the
// count of eps_l >= x is the first l with eps_l < x.
__global__ __launch_bounds__(256) void prep_count_kernel(Prep p) {
    const int M = p.v.M, NL = p.v.NL;
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= (int64_t)p.v.S * M * M) return;
    const int s = (int)(t / ((int64_t)M * M));
    const int r = (int)(t - (int64_t)s * M * M);
    const int i = r / M, k = r - i * M;
    int n = NL;
    if (i < k) {
        const double x = p.v.E[(int64_t)s * M + k] - p.v.E[(int64_t)s * M + i];
        int lo = 0, hi = NL;  // first l in [0, NL] with eps_l < x
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (p.eps[mid] < x) hi = mid; else lo = mid + 1;
        }
        n = lo;
    }
    p.cnt[t] = n;
}

// Emission table: one thread per (wavelength, (grain, level)).
__global__ __launch_bounds__(256) void prep_etab_kernel(Prep p) {
    const View& v = p.v;
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= (int64_t)v.NLp * v.Kp) return;
    const int k = (int)(t / v.NLp), l = (int)(t - (int64_t)k * v.NLp);
    float val = 0.0f;
    if (l < v.NL && k < v.K) {
        const int s = k / v.M;
        const double T = p.T[k];  // [S][M] flattened: k = s M + j
        if (T > 0.0) {
            const double lam = p.lam[l];
            const double em = expm1_pos(RAD_C2 / lam * rcp_f64(T));
            const double lam2 = lam * lam;
            const double b = (em < __builtin_inf()) ? RAD_C1 / (lam2 * lam2 * lam) / em : 0.0;
            val = (float)ldexp(p.w[s] * p.cabs[(int64_t)s * v.NL + l] * b, -p.ge);
        }
    }
    p.etab[t] = val;
}

// ---------------------------------------------------------------------------
// The distribution of one pair per wave; Q = levels per lane (M <= 64 Q).
//
// Lanes over the upper level j: acc_j collects sum_{i<j} B[j][i] X_i.  Level
// i is final once every level below it has been added, so the levels are
// taken in order: X_i = acc_i / cool_i is read from lane i, and every lane
// j > i adds B[j][i] X_i.  No wave reduction is needed; the rates of a step
// depend only on the plan and the pair's prefix sums, not on X.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double readlane_f64(double x, int lane) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(x), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(x), lane);
    return __hiloint2double(hi, lo);
}

template <int Q>
__device__ __forceinline__ double pick(const double (&a)[Q], int q) {
    double r = a[0];
#pragma unroll
    for (int k = 1; k < Q; ++k)
        if (q == k) r = a[k];
    return r;
}

template <int Q>
__global__ __launch_bounds__(64) void solve_kernel(View v, int64_t C, const float* __restrict__ J,
                                                   int64_t ldj, float* __restrict__ P, int64_t ldp,
                                                   dust_counters* cnt) {
    extern __shared__ double2 sF[];  // [NL + 1]: (F0, F1) prefix sums
    const int lane = threadIdx.x;
    const int64_t pair = blockIdx.x;
    const int s = (int)(pair % v.S);
    const int64_t c = pair / v.S;
    const int NL = v.NL, M = v.M;
    // 1. photon rates and their prefix sums, shortest wavelength first
    const float* jr = J + c * ldj;
    const double* kr = v.kr + (int64_t)s * NL;
    double carry0 = 0.0, carry1 = 0.0;
    bool bad = false;
    if (lane == 0) sF[0] = make_double2(0.0, 0.0);
    for (int l0 = 0; l0 < NL; l0 += 64) {
        const int l = l0 + lane;
        double r = 0.0, re = 0.0;
        if (l < NL) {
            const float jv = jr[l];
            if (!(jv >= 0.0f) || __builtin_isinf(jv)) bad = true;
            r = (double)jv * kr[l];
            re = r * v.eps[l];
        }
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const double a = __shfl_up(r, d, 64), b = __shfl_up(re, d, 64);
            if (lane >= d) {
                r += a;
                re += b;
            }
        }
        if (l < NL) sF[l + 1] = make_double2(carry0 + r, carry1 + re);
        carry0 += readlane_f64(r, 63);
        carry1 += readlane_f64(re, 63);
    }
    const bool any_bad = __ballot(bad) != 0;
    __syncthreads();
    // 2. levels in order; lane holds upper levels j = lane + 64 q
    const double* Es = v.E + (int64_t)s * M;
    const double* rcool = v.rcool + (int64_t)s * M;
    const int* cn = v.cnt + (int64_t)s * M * M;
    double acc[Q], X[Q], Ejm1[Q], dinv[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int j = lane + 64 * q;
        const bool ok = j >= 1 && j < M;
        acc[q] = 0.0;
        X[q] = 0.0;
        Ejm1[q] = ok ? Es[j - 1] : 0.0;
        dinv[q] = ok ? v.invd[(int64_t)s * M + j] : 0.0;
    }
    double xi = 1.0;  // X_0
    for (int i = 0; i < M; ++i) {
        if (i > 0) {
            xi = readlane_f64(pick<Q>(acc, i >> 6), i & 63) * rcool[i];
            if (xi > 0x1p500) {  // uniform: keep the running values in range (exact)
                xi = ldexp(xi, -500);
#pragma unroll
                for (int q = 0; q < Q; ++q) {
                    acc[q] = ldexp(acc[q], -500);
                    X[q] = ldexp(X[q], -500);
                }
            }
        }
#pragma unroll
        for (int q = 0; q < Q; ++q)
            if ((i >> 6) == q && lane == (i & 63)) X[q] = xi;
        if (i == M - 1) break;
        const double Ei = Es[i];
        const int* row = cn + (int64_t)i * M;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            if (64 * q + 63 <= i) continue;  // uniform: every level of this chunk is at or below i
            const int j = lane + 64 * q;
            if (j > i && j < M) {
                const int n1 = row[j - 1];  // eps >= E_{j-1} - E_i (NL when j - 1 = i)
                const int n2 = row[j];      // eps >= E_j - E_i
                const double2 f1 = sF[n1], f2 = sF[n2];
                const double a = Ejm1[q] - Ei;
                const double B = f2.x + ((f1.y - f2.y) - a * (f1.x - f2.x)) * dinv[q];
                acc[q] = fma(B, xi, acc[q]);
            }
        }
    }
    // 3. normalise
    double tot = 0.0;
#pragma unroll
    for (int q = 0; q < Q; ++q) tot += X[q];
    tot = wave_sum_f64(tot);
    const double inv = 1.0 / tot;
    float* pr = P + c * ldp + (int64_t)s * M;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int i = lane + 64 * q;
        if (i < M) {
            const double pv = X[q] * inv;
            pr[i] = any_bad ? __builtin_nanf("") : (float)pv;
            if (cnt && !any_bad && i == M - 1 && pv > TOP_PROBABILITY) count(&cnt->n_out_of_table);
        }
    }
    if (cnt && any_bad && lane == 0) count(&cnt->n_nonfinite);
}

// ---------------------------------------------------------------------------
// The same distribution for grains of at most 64 levels (one level per lane),
// several cells of one grain per workgroup (a wave per cell).  The grain's
// tables go through LDS once per workgroup: the photon counts as byte offsets
// into a wave's prefix sums ([M][M] ints) and (E_i, 1 / cooling rate_i)
// ([M] pairs).  Per level step a wave then issues only LDS reads and VALU
// work: the lower level's value X_i = acc_i / cool_i is read from lane i of
// the product acc * (1 / cool), its enthalpy is one broadcast LDS read, the
// rescale test is a scalar branch on X_i's exponent word, and X is not kept
// per level but read off the sums at the end (X_j = acc_j / cool_j, every
// sum having taken the same rescales; X_0 = 2^(-500 rescales)).  The
// arithmetic of every sum is the one of solve_kernel.
// ---------------------------------------------------------------------------
constexpr int STAGED_MAX_LEVELS = 64;
constexpr int STAGED_MAX_WAVES = 8;

// LDS of the grain's tables: the offsets [M + 1][M] (a zero row after the
// last, read by the steps past the end), then (E, 1 / cooling rate) [M].
__host__ __device__ inline int staged_offsets_bytes(int M) {
    return (4 * (M + 1) * M + 15) / 16 * 16;
}
__host__ __device__ inline int staged_table_bytes(int M) {
    return staged_offsets_bytes(M) + 16 * M;
}

__global__ __launch_bounds__(64 * STAGED_MAX_WAVES) void solve_staged_kernel(
    View v, int64_t C, const float* __restrict__ J, int64_t ldj, float* __restrict__ P,
    int64_t ldp, dust_counters* cnt) {
    extern __shared__ __align__(16) char smem[];
    const int NL = v.NL, M = v.M, S = v.S;
    const int W = (int)(blockDim.x >> 6);
    int* sOff = reinterpret_cast<int*>(smem);  // [M + 1][M] 16 * count
    double2* sLev = reinterpret_cast<double2*>(smem + staged_offsets_bytes(M));  // [M]
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    char* sFb = smem + staged_table_bytes(M) + (size_t)wave * (NL + 1) * sizeof(double2);
    double2* sF = reinterpret_cast<double2*>(sFb);
    const int s = (int)(blockIdx.x % (unsigned)S);
    const int64_t c_raw = (int64_t)(blockIdx.x / (unsigned)S) * W + wave;
    const bool live = c_raw < C;
    const int64_t c = live ? c_raw : C - 1;  // a wave past the end repeats the last cell, unwritten
    // 0. the grain's tables
    {
        const int* cn = v.cnt + (int64_t)s * M * M;
        for (int e = threadIdx.x; e < M * M; e += blockDim.x) sOff[e] = cn[e] * (int)sizeof(double2);
        for (int e = threadIdx.x; e < M; e += blockDim.x) sOff[M * M + e] = 0;
        for (int e = threadIdx.x; e < M; e += blockDim.x)
            sLev[e] = make_double2(v.E[(int64_t)s * M + e], v.rcool[(int64_t)s * M + e]);
    }
    // 1. photon rates and their prefix sums, shortest wavelength first: lane
    //    l takes the wavelengths [l G, (l + 1) G), G = ceil(NL / 64); one
    //    wave scan of the lanes' totals gives each lane its start, then the
    //    lane runs through its wavelengths again writing the sums.
    const float* jr = J + c * ldj;
    const double* kr = v.kr + (int64_t)s * NL;
    const int G = (NL + 63) >> 6;
    const int lb = lane * G;
    bool bad = false;
    double t0 = 0.0, t1 = 0.0;
    for (int q = 0; q < G; ++q) {
        const int l = lb + q;
        if (l < NL) {
            const float jv = jr[l];
            if (!(jv >= 0.0f) || __builtin_isinf(jv)) bad = true;
            const double r = (double)jv * kr[l];
            t0 += r;
            t1 += r * v.eps[l];
        }
    }
    // exclusive scan of the totals: the lane below's total, then an inclusive scan
    double e0 = __shfl_up(t0, 1, 64), e1 = __shfl_up(t1, 1, 64);
    if (lane == 0) e0 = e1 = 0.0;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const double a = __shfl_up(e0, d, 64), b = __shfl_up(e1, d, 64);
        if (lane >= d) {
            e0 += a;
            e1 += b;
        }
    }
    if (lane == 0) sF[0] = make_double2(0.0, 0.0);
    for (int q = 0; q < G; ++q) {
        const int l = lb + q;
        if (l < NL) {
            const double r = (double)jr[l] * kr[l];
            e0 += r;
            e1 += r * v.eps[l];
            sF[l + 1] = make_double2(e0, e1);
        }
    }
    const bool any_bad = __ballot(bad) != 0;
    __syncthreads();
    // 2. levels in order; lane j holds level j.  The LDS reads are issued
    //    ahead of their use, so the chain from one level to the next is only
    //    acc -> X_i -> acc: at step i the offsets of step i + 2 and the prefix
    //    sums of step i + 1 are read, and B[j][i] is formed from the sums read
    //    at step i - 1.  Lanes with j <= i read valid addresses and drop the
    //    values.
    const int j = lane;
    const bool jok = j >= 1 && j < M;
    const double Ejm1 = jok ? sLev[j - 1].x : 0.0;
    const double Ej = j < M ? sLev[j].x : 0.0;
    const double dinv = jok ? v.invd[(int64_t)s * M + j] : 0.0;
    const double rc = j < M ? sLev[j].y : 0.0;  // 0 at j = 0
    // offset of step r <= M for this lane: the count of eps >= E_j - E_r
    // (column j of row r; column M - 1 for lanes past the last level; row M
    // is zeros).  The other bound of B[j][r], eps >= E_{j-1} - E_r, is the
    // next lane down's: its sums come from that lane by a one-lane shift of
    // the wave (DPP), one LDS gather per step instead of two.
    const int* col = sOff + (j < M ? j : M - 1);
    auto offset = [&](int r) { return col[r * M]; };
    auto sums = [&](int o) { return *reinterpret_cast<const double2*>(sFb + o); };
    auto from_lane_below = [](const double2& a) {
        auto sh = [](double x) {  // lane l gets lane l - 1's x (lane 0: 0)
            const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), 0x138, 0xf, 0xf, false);
            const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), 0x138, 0xf, 0xf, false);
            return __hiloint2double(hi, lo);
        };
        return make_double2(sh(a.x), sh(a.y));
    };
    int o2 = offset(0);
    double2 f2 = sums(o2);  // step 0
    o2 = offset(1);         // step 1
    double acc = 0.0;
    int rescales = 0;
    double xi = 1.0;  // X_0
    double Ei = sLev[0].x;
    // one step: B[j][i] from the sums a2 read at the step before (and the
    // lane below's), the sums of step i + 1 into b2, the offset of step
    // i + 2 and E_{i+1}, then X_i (from readlane in both branches of the
    // rescale, so it stays in scalar registers)
    auto step = [&](int i, const double2& a2, double2& b2) {
        const double2 a1 = from_lane_below(a2);
        const double B = a2.x + ((a1.y - a2.y) - (Ejm1 - Ei) * (a1.x - a2.x)) * dinv;
        // the offset first: LDS reads complete in order, and the next step
        // needs it before the sums
        const int n2 = offset(i + 2);
        b2 = sums(o2);
        o2 = n2;
        Ei = sLev[i + 1 < M ? i + 1 : i].x;
        if (i > 0) {
            xi = readlane_f64(acc * rc, i);
            if (__double2hiint(xi) > 0x5F2FFFFF) {  // X_i >= 2^500 (uniform): rescale, exactly
                // (the empty asm keeps this a scalar branch: without it the
                // compiler computes the rescale at every step and selects)
                asm volatile("");
                acc = ldexp(acc, -500);
                ++rescales;
                xi = readlane_f64(acc * rc, i);
            }
        }
        if (j > i) {
            asm volatile("");  // (an exec-masked branch, not a select after the FMA)
            acc = fma(B, xi, acc);
        }
    };
    // two steps per pass, the sums alternating between two register sets
    // (a copy from one to the other would wait for the reads at once)
    double2 g2;
    int i = 0;
    for (; i + 1 < M - 1; i += 2) {
        step(i, f2, g2);
        step(i + 1, g2, f2);
    }
    if (i < M - 1) step(i, f2, g2);
    // 3. normalise
    const double X = j == 0 ? ldexp(1.0, -500 * rescales) : (j < M ? acc * rc : 0.0);
    const double tot = wave_sum_f64(X);
    const double inv = 1.0 / tot;
    if (live && j < M) {
        const double pv = X * inv;
        P[c * ldp + (int64_t)s * M + j] = any_bad ? __builtin_nanf("") : (float)pv;
        if (cnt && !any_bad && j == M - 1 && pv > TOP_PROBABILITY) count(&cnt->n_out_of_table);
    }
    if (live && cnt && any_bad && lane == 0) count(&cnt->n_nonfinite);
}

// ---------------------------------------------------------------------------
// Emission: L[c,l] = m_c sum_k P[c,k] Etab[k,l] on v_mfma_f32_16x16x4_f32.  A
// workgroup of four waves takes 64 cells x 128 wavelengths, each wave 16
// cells x all 128 (eight 16x16 accumulator blocks sharing the cells' P
// values).  The table goes through LDS in chunks of 32 k x 128 wavelengths,
// double-buffered, rows of 130 floats (the four k-rows one B read touches fall
// on distinct bank groups); the next chunk and the next P values load during
// the MFMAs of the current one.  Within a chunk MFMA sub-step s takes, in
// k-slot q (lane = 16 q + row), the k = k0 + 8 q + s: one permutation of the
// chunk's k for both operands, so a lane's eight P values of a chunk are
// consecutive.  VW: P load width in floats (rows and P aligned to it).
// ---------------------------------------------------------------------------
constexpr int E_KC = 32;
constexpr int E_ROW = 130;
constexpr int E_CELLS = 64;

template <int VW>
__global__ __launch_bounds__(256) void emit_kernel(View v, int64_t C, const float* __restrict__ P,
                                                   int64_t ldp, const float* __restrict__ m,
                                                   float* __restrict__ L, int64_t ldl,
                                                   int accumulate) {
    __shared__ __align__(16) float sE[2][E_KC][E_ROW];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int row = lane & 15, q = lane >> 4;
    const int nlb = v.NLp / 128;
    const int64_t b = blockIdx.x;
    const int lb = (int)(b % nlb);
    const int64_t c0 = (b / nlb) * E_CELLS + 16 * wave;
    const int l0 = lb * 128;
    const int64_t cr = c0 + row;
    const bool c_ok = cr < C;
    const float* pr = P + (c_ok ? cr : 0) * ldp;
    const int nch = v.Kp / E_KC;
    // table loader: thread t takes k-row t / 8 of the chunk, wavelengths 16 (t mod 8) .. + 16
    const int ek = tid >> 3, el = (tid & 7) * 16;
    auto load_e = [&](int ch, float4 (&e)[4]) {
        const float* src = v.etab + (int64_t)(ch * E_KC + ek) * v.NLp + l0 + el;
#pragma unroll
        for (int i = 0; i < 4; ++i) e[i] = *reinterpret_cast<const float4*>(src + 4 * i);
    };
    auto store_e = [&](int buf, const float4 (&e)[4]) {
        float* dst = &sE[buf][ek][el];  // 8-byte aligned (rows of 520 bytes)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            *reinterpret_cast<float2*>(dst + 4 * i) = make_float2(e[i].x, e[i].y);
            *reinterpret_cast<float2*>(dst + 4 * i + 2) = make_float2(e[i].z, e[i].w);
        }
    };
    auto load_p = [&](int ch, float (&a)[8]) {
        const int k = ch * E_KC + 8 * q;
        if (VW == 4 && c_ok && k + 8 <= v.K) {
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const float4 f = *reinterpret_cast<const float4*>(pr + k + 4 * i);
                a[4 * i] = f.x;
                a[4 * i + 1] = f.y;
                a[4 * i + 2] = f.z;
                a[4 * i + 3] = f.w;
            }
        } else if (VW == 2 && c_ok && k + 8 <= v.K) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float2 f = *reinterpret_cast<const float2*>(pr + k + 2 * i);
                a[2 * i] = f.x;
                a[2 * i + 1] = f.y;
            }
        } else {
#pragma unroll
            for (int i = 0; i < 8; ++i) a[i] = (c_ok && k + i < v.K) ? pr[k + i] : 0.0f;
        }
    };
    f32x4 acc[8];
#pragma unroll
    for (int blk = 0; blk < 8; ++blk) acc[blk] = f32x4{0.f, 0.f, 0.f, 0.f};
    float4 e[4];
    float a[8], an[8];
    load_e(0, e);
    load_p(0, a);
    store_e(0, e);
    __syncthreads();
    for (int ch = 0; ch < nch; ++ch) {
        const int buf = ch & 1;
        const bool more = ch + 1 < nch;
        if (more) {
            load_e(ch + 1, e);
            load_p(ch + 1, an);
        }
#pragma unroll
        for (int s = 0; s < 8; ++s)
#pragma unroll
            for (int blk = 0; blk < 8; ++blk)
                acc[blk] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[s], sE[buf][8 * q + s][16 * blk + row],
                                                                acc[blk], 0, 0, 0);
        if (more) {
            store_e(buf ^ 1, e);
#pragma unroll
            for (int i = 0; i < 8; ++i) a[i] = an[i];
        }
        __syncthreads();
    }
    // accumulator element r of lane (row, q): cell c0 + 4 q + r, wavelength l0 + 16 blk + row
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int64_t cc = c0 + 4 * q + r;
        if (cc >= C) continue;
        const float scale = (m ? m[cc] : 1.0f) * v.escale;
#pragma unroll
        for (int blk = 0; blk < 8; ++blk) {
            const int l = l0 + 16 * blk + row;
            if (l < v.NL) {
                const float val = acc[blk][r] * scale;
                float* dst = L + cc * ldl + l;
                *dst = accumulate ? *dst + val : val;
            }
        }
    }
}

int round_up(int x, int mlt) { return (x + mlt - 1) / mlt * mlt; }

}  // namespace fluct
}  // namespace dust

struct dust_fluct_plan {
    int device;
    double *d_lam, *d_dlam, *d_cabs, *d_w, *d_T;
    double *d_E, *d_eps, *d_kr, *d_rcool, *d_invd;
    int* d_cnt;
    float* d_etab;
    dust::fluct::View view;
};

namespace dust {
namespace fluct {

void free_plan(dust_fluct_plan* p) {
    if (!p) return;
    void* ptrs[] = {p->d_lam, p->d_dlam, p->d_cabs, p->d_w, p->d_T, p->d_E,
                    p->d_eps, p->d_kr, p->d_rcool, p->d_invd, p->d_cnt, p->d_etab};
    for (void* x : ptrs)
        if (x) (void)hipFree(x);
    delete p;
}

dust_status validate_levels(const dust_levels* lv, int S) {
    if (!lv) return set_error(DUST_EINVAL, "levels descriptor is NULL");
    const int M = lv->n_levels;
    if (M < 2 || M > MAX_LEVELS) return set_error(DUST_EINVAL, "n_levels must be in [2, 256]");
    if (!lv->T || !lv->E) return set_error(DUST_EINVAL, "a level table pointer is NULL");
    for (int s = 0; s < S; ++s) {
        const double* T = lv->T + (int64_t)s * M;
        const double* E = lv->E + (int64_t)s * M;
        if (T[0] != 0.0 || E[0] != 0.0)
            return set_error(DUST_EINVAL, "level 0 must be the ground state (T = 0, E = 0)");
        for (int j = 1; j < M; ++j) {
            if (!isfinite(T[j]) || !isfinite(E[j]) || !(T[j] > T[j - 1]) || !(E[j] > E[j - 1]))
                return set_error(DUST_EINVAL,
                                 "level temperatures and enthalpies must be finite and strictly "
                                 "increasing");
        }
    }
    return DUST_OK;
}

}  // namespace fluct
}  // namespace dust

using namespace dust;
using namespace dust::fluct;

extern "C" {

dust_status dust_fluct_plan_create(const dust_grid_desc* g, const dust_levels* lv,
                                   dust_fluct_plan** out) {
    clear_error();
    if (!out) return set_error(DUST_EINVAL, "out is NULL");
    *out = nullptr;
    dust_status st = validate_grid(g);
    if (st != DUST_OK) return st;
    if ((st = validate_levels(lv, g->n_grains)) != DUST_OK) return st;
    const int NL = g->n_lambda, S = g->n_grains, M = lv->n_levels;
    if ((size_t)(NL + 1) * sizeof(double2) > (size_t)MAX_LDS)
        return set_error(DUST_EUNSUPPORTED,
                         "fluctuating grains take at most 4095 wavelengths (one workgroup's "
                         "prefix sums in LDS)");
    if ((int64_t)S * M > (1 << 20))
        return set_error(DUST_EUNSUPPORTED, "n_grains x n_levels above 2^20");
    // one power of two for the emission table: with B(lam, T) <= c1 lam^-4 T / c2
    // (Rayleigh-Jeans) its entries stay below 2^0
    double emax = 0.0;
    for (int s = 0; s < S; ++s) {
        const double tmax = lv->T[(int64_t)s * M + M - 1];
        for (int l = 0; l < NL; ++l) {
            const double lam = g->lambda[l];
            emax = fmax(emax, g->weight[s] * g->c_abs[(int64_t)s * NL + l] * RAD_C1 * tmax /
                                  (RAD_C2 * lam * lam * lam * lam));
        }
    }
    int ge = 0;
    if (emax > 0.0) (void)frexp(emax, &ge);
    if (ge < -120 || ge > 120)
        return set_error(DUST_EUNSUPPORTED, "emission table outside the FP32 range");

    hipError_t e;
    int dev = 0;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return hip_error(e, "hipGetDevice");
    dust_fluct_plan* p = new dust_fluct_plan;
    memset(p, 0, sizeof *p);
    p->device = dev;
    View& v = p->view;
    v.NL = NL;
    v.S = S;
    v.M = M;
    v.K = S * M;
    v.Kp = round_up(v.K, 32);
    v.NLp = round_up(NL, 128);
    v.escale = ldexpf(1.0f, ge);
    const size_t nSM = (size_t)S * M;
#define FALLOC(ptr, n)                                                     \
    if ((e = hipMalloc((void**)&(ptr), sizeof(*(ptr)) * (n))) != hipSuccess) { \
        free_plan(p);                                                      \
        return hip_error(e, "hipMalloc (" #ptr ")");                       \
    }
    FALLOC(p->d_lam, NL);
    FALLOC(p->d_dlam, NL);
    FALLOC(p->d_cabs, (size_t)S * NL);
    FALLOC(p->d_w, S);
    FALLOC(p->d_T, nSM);
    FALLOC(p->d_E, nSM);
    FALLOC(p->d_eps, NL);
    FALLOC(p->d_kr, (size_t)S * NL);
    FALLOC(p->d_rcool, nSM);
    FALLOC(p->d_invd, nSM);
    FALLOC(p->d_cnt, nSM * M);
    FALLOC(p->d_etab, (size_t)v.NLp * v.Kp);
#undef FALLOC
    struct Up { void* d; const void* h; size_t n; } ups[] = {
        {p->d_lam, g->lambda, sizeof(double) * NL},
        {p->d_dlam, g->dlambda, sizeof(double) * NL},
        {p->d_cabs, g->c_abs, sizeof(double) * S * (size_t)NL},
        {p->d_w, g->weight, sizeof(double) * S},
        {p->d_T, lv->T, sizeof(double) * nSM},
        {p->d_E, lv->E, sizeof(double) * nSM},
    };
    for (const Up& u : ups) {
        if ((e = hipMemcpy(u.d, u.h, u.n, hipMemcpyHostToDevice)) != hipSuccess) {
            free_plan(p);
            return hip_error(e, "hipMemcpy (fluctuating-grain plan)");
        }
    }
    v.eps = p->d_eps;
    v.kr = p->d_kr;
    v.E = p->d_E;
    v.rcool = p->d_rcool;
    v.invd = p->d_invd;
    v.cnt = p->d_cnt;
    v.etab = p->d_etab;
    Prep pr{v, p->d_lam, p->d_dlam, p->d_cabs, p->d_w, p->d_T,
            p->d_eps, p->d_kr, p->d_rcool, p->d_invd, p->d_cnt, p->d_etab, ge};
    const int64_t n_rates = (int64_t)S * NL, n_cnt = (int64_t)nSM * M,
                  n_etab = (int64_t)v.NLp * v.Kp;
    hipLaunchKernelGGL(prep_rates_kernel, dim3((unsigned)((n_rates + 255) / 256)), dim3(256), 0,
                       nullptr, pr);
    e = hipGetLastError();
    if (e == hipSuccess) {
        hipLaunchKernelGGL(prep_cool_kernel, dim3(M, S), dim3(64), 0, nullptr, pr);
        e = hipGetLastError();
    }
    if (e == hipSuccess) {  // after the rates: the counts read eps
        hipLaunchKernelGGL(prep_count_kernel, dim3((unsigned)((n_cnt + 255) / 256)), dim3(256), 0,
                           nullptr, pr);
        e = hipGetLastError();
    }
    if (e == hipSuccess) {
        hipLaunchKernelGGL(prep_etab_kernel, dim3((unsigned)((n_etab + 255) / 256)), dim3(256), 0,
                           nullptr, pr);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        free_plan(p);
        return hip_error(e, "fluctuating-grain plan kernels");
    }
    // every level above the ground must radiate (the solve multiplies by
    // 1 / its cooling rate)
    std::vector<double> rcool(nSM);
    if ((e = hipMemcpy(rcool.data(), p->d_rcool, sizeof(double) * nSM, hipMemcpyDeviceToHost)) !=
        hipSuccess) {
        free_plan(p);
        return hip_error(e, "hipMemcpy (cooling rates)");
    }
    for (int s = 0; s < S; ++s)
        for (int j = 1; j < M; ++j)
            if (!(rcool[(size_t)s * M + j] > 0.0) || !isfinite(rcool[(size_t)s * M + j])) {
                free_plan(p);
                return set_error(DUST_EINVAL,
                                 "grain " + std::to_string(s) + " level " + std::to_string(j) +
                                     ": the grain radiates no power at that temperature in FP64 "
                                     "(too cold for the wavelength grid)");
            }
    *out = p;
    return DUST_OK;
}

dust_status dust_fluct_plan_destroy(dust_fluct_plan* p) {
    clear_error();
    if (!p) return DUST_OK;
    const hipError_t e = hipDeviceSynchronize();
    free_plan(p);
    return e == hipSuccess ? DUST_OK : hip_error(e, "hipDeviceSynchronize");
}

dust_status dust_fluct_solve_P(dust_fluct_plan* p, int64_t C, const float* J, int64_t ldj,
                               float* P, int64_t ldp, dust_counters* cnt, void* stream) {
    clear_error();
    if (!p) return set_error(DUST_EINVAL, "plan is NULL");
    if (C < 0) return set_error(DUST_EINVAL, "n_cells must be >= 0");
    const View& v = p->view;
    if (C * (int64_t)v.S > INT32_MAX)
        return set_error(DUST_EUNSUPPORTED, "n_cells x n_grains above 2^31 - 1");
    if (cnt && ((uintptr_t)cnt & 7u)) return set_error(DUST_EINVAL, "counters must be 8-byte aligned");
    if (C == 0) return DUST_OK;
    if (!J || !P) return set_error(DUST_EINVAL, "J or P is NULL");
    if ((((uintptr_t)J) | ((uintptr_t)P)) & 3u)
        return set_error(DUST_EINVAL, "J and P must be 4-byte aligned");
    if (ldj < v.NL) return set_error(DUST_EINVAL, "leading dimension of J is smaller than its row");
    if (ldp < (int64_t)v.K)
        return set_error(DUST_EINVAL, "leading dimension of P is smaller than n_grains x n_levels");
    const hipStream_t st = (hipStream_t)stream;
    const size_t lds = sizeof(double2) * (size_t)(v.NL + 1);
    if (v.M <= STAGED_MAX_LEVELS) {
        // as many cells per workgroup (up to eight) as the LDS allows
        int w = STAGED_MAX_WAVES;
        while (w > 1 && (size_t)staged_table_bytes(v.M) + w * lds > (size_t)MAX_LDS) w >>= 1;
        if ((size_t)staged_table_bytes(v.M) + w * lds <= (size_t)MAX_LDS) {
            const int64_t groups = (C + w - 1) / w;
            hipLaunchKernelGGL(solve_staged_kernel, dim3((unsigned)(groups * v.S)), dim3(64 * w),
                               (size_t)staged_table_bytes(v.M) + w * lds, st, v, C, J, ldj, P,
                               ldp, cnt);
            const hipError_t e = hipGetLastError();
            return e == hipSuccess ? DUST_OK
                                   : hip_error(e, "fluctuating-grain distribution launch");
        }
    }
    const dim3 grid((unsigned)(C * v.S));
    if (v.M <= 64)
        hipLaunchKernelGGL(solve_kernel<1>, grid, dim3(64), lds, st, v, C, J, ldj, P, ldp, cnt);
    else if (v.M <= 128)
        hipLaunchKernelGGL(solve_kernel<2>, grid, dim3(64), lds, st, v, C, J, ldj, P, ldp, cnt);
    else
        hipLaunchKernelGGL(solve_kernel<4>, grid, dim3(64), lds, st, v, C, J, ldj, P, ldp, cnt);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? DUST_OK : hip_error(e, "fluctuating-grain distribution launch");
}

dust_status dust_fluct_emit_sed(dust_fluct_plan* p, int64_t C, const float* P, int64_t ldp,
                                const float* m, float* L, int64_t ldl, int32_t accumulate,
                                void* stream) {
    clear_error();
    if (!p) return set_error(DUST_EINVAL, "plan is NULL");
    if (C < 0) return set_error(DUST_EINVAL, "n_cells must be >= 0");
    const View& v = p->view;
    if (C == 0) return DUST_OK;
    if (!P || !L) return set_error(DUST_EINVAL, "P or L is NULL");
    if ((((uintptr_t)P) | ((uintptr_t)L) | ((uintptr_t)m)) & 3u)
        return set_error(DUST_EINVAL, "P, L and m_dust must be 4-byte aligned");
    if (ldp < (int64_t)v.K)
        return set_error(DUST_EINVAL, "leading dimension of P is smaller than n_grains x n_levels");
    if (ldl < v.NL) return set_error(DUST_EINVAL, "leading dimension of L is smaller than its row");
    const int64_t blocks = (C + E_CELLS - 1) / E_CELLS * (v.NLp / 128);
    if (blocks > INT32_MAX) return set_error(DUST_EUNSUPPORTED, "too many cells");
    const hipStream_t st = (hipStream_t)stream;
    const int acc_flag = accumulate ? 1 : 0;
    if ((ldp % 4) == 0 && ((uintptr_t)P & 15u) == 0)
        hipLaunchKernelGGL(emit_kernel<4>, dim3((unsigned)blocks), dim3(256), 0, st, v, C, P, ldp,
                           m, L, ldl, acc_flag);
    else if ((ldp % 2) == 0 && ((uintptr_t)P & 7u) == 0)
        hipLaunchKernelGGL(emit_kernel<2>, dim3((unsigned)blocks), dim3(256), 0, st, v, C, P, ldp,
                           m, L, ldl, acc_flag);
    else
        hipLaunchKernelGGL(emit_kernel<1>, dim3((unsigned)blocks), dim3(256), 0, st, v, C, P, ldp,
                           m, L, ldl, acc_flag);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? DUST_OK : hip_error(e, "fluctuating-grain emission launch");
}

}  // extern "C"
