// Plan-time kernels: the derived tables of a grid.
//
//  prep  (the paper's first kernel, Section 4.1): K = C dlam per grain and
//        wavelength, scaled per grain by an exact power of two, in FP32 and as
//        a bf16 hi+lo pair (both in MFMA fragment order); the solve weights K' c1 lam^-5; the emission
//        weights w C c1 lam^-5 (Eq. 10 without the mass); the wavelength
//        exponent table nu = -c2 log2(e) / lam.
//  ltab  (mixed mode): per grain, y_k = ln P'(T_k) at log-spaced T_k, in
//        FP64, with P'(T) = sum_l K'_l B(lam_l, T) the right side of Eq. 7 in
//        the plan's scaled units -- as an FP64 matrix product (MFMA) of the
//        grains' Planck weights with the Planck factors of the table
//        temperatures, which the product computes as it goes.
//  inv   (mixed mode): the inverse function ln T(y) and its derivative at
//        uniform steps of y, from Newton in FP64 on the forward table's
//        piecewise cubic, stored as FP32 pairs of nodes (one 16-byte load
//        per lookup).
//  table-linear mode: the same matrix product gives P'(T_k) itself at evenly
//        spaced T_k (the production table of Sections 2 and 5); kidx gives,
//        at uniform steps of ln P', the last table point below, so that a
//        lookup searches only a few points.
#include "device_common.h"

namespace dust {
namespace {

__device__ __forceinline__ void prep_body(const RefreshJob& j, int bx, int by) {
    const PlanView& v = j.v;
    const double* __restrict__ lam = j.lam;
    const double* __restrict__ dlam = j.dlam;
    const double* __restrict__ cabs = j.cabs;
    const double* __restrict__ w = j.w;
    const int* __restrict__ es = j.es;
    const int ge = j.ge;
    float* nu = j.nu; float* kf = j.kf; float* kb = j.kb; float* ku = j.ku; float* em = j.em;
    __bf16* khi = j.khi; __bf16* klo = j.klo;
    double* kdb = j.kdb; double* c2l = j.c2l;
    const int l = bx * blockDim.x + threadIdx.x;
    const int s = by;
    if (l >= v.NLp) return;
    const int64_t o = (int64_t)s * v.NLp + l;
    // The heating weights are stored in MFMA fragment order, so that one
    // wave's fragment of one grain tile and k-step is a contiguous 1 KB.
    const int64_t ob = kfrag_bf16(v, s, l), of = kfrag_f32(v, s, l);
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
        kf[of] = kff;
        khi[ob] = hi;
        klo[ob] = lo;
        kb[o] = (float)(K * c1l5);
        ku[o] = (float)(K * c1l5 * (RAD_C2 * LOG2E / lm));
        em[o] = (float)ldexp(w[s] * C * c1l5, -ge);
        kdb[(int64_t)s * v.NL + l] = K * c1l5;
    } else {
        kf[of] = 0.0f;
        khi[ob] = (__bf16)0.0f;
        klo[ob] = (__bf16)0.0f;
        kb[o] = 0.0f;
        ku[o] = 0.0f;
        em[o] = 0.0f;
    }
}

// The table is a matrix product:  P'[s,k] = sum_l W[s,l] F[k,l]  with
// W = K' c1 lam^-5 (per grain) and F[k,l] = 1 / (exp(c2 / (lam_l T_k)) - 1)
// (per table temperature, the same for every grain).

// y[s][k] = ln sum_l W[s][l] F[k][l] (table-linear: the sum itself): an FP64
// product on the matrix cores (v_mfma_f64_16x16x4_f64) whose F operand is
// computed in registers and never stored.  Each wave owns 16 table points
// (a workgroup's four waves take four consecutive blocks of them) and up to
// LT_SG grain tiles of 16.  Per 32-wavelength step, lane (row = lane mod 16,
// q = lane / 16) computes F for point row and wavelengths l0 + 8 q .. + 7
// (eight FP64 exponentials), loads the same wavelengths of each grain tile's
// row of W (contiguous 64 bytes) and issues eight MFMAs per tile; MFMA t
// takes the t-th wavelength of both operands (any assignment of wavelengths
// to k-slots gives the same sum when both operands use it).  Element j of a
// tile's accumulator in lane (col, q) holds grain row q + 4 j of point col
// (the FP64 form interleaves rows).
// Grain tiles per wave when many plans share a launch: four (the product's
// exponentials are spent once per four tiles).  A single plan takes the
// split form below instead (LT_SG_SINGLE only instantiates the other stages).
constexpr int LT_SG_BATCHED = 4, LT_SG_SINGLE = 1;

template <int LT_SG>
__device__ __forceinline__ void ltab_gemm_body(const RefreshJob& j, int bx, int by) {
    typedef double f64x4 __attribute__((ext_vector_type(4)));
    const PlanView& v = j.v;
    double* fwd = j.fwd;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int row = lane & 15, q = lane >> 4;
    const int k0 = (bx * 4 + wave) * 16;
    const int sg0 = by * LT_SG * 16;
    const int k = k0 + row;
    const bool k_ok = k < v.N;
    const double invT = !k_ok ? 0.0
                        : (v.mode == DUST_TABLE_LINEAR ? 1.0 / v.texp[k]
                                                       : exp(-(v.lnTmin + k * v.hstep)));
    f64x4 acc[LT_SG];
#pragma unroll
    for (int t = 0; t < LT_SG; ++t) acc[t] = f64x4{0.0, 0.0, 0.0, 0.0};
    for (int l0 = 0; l0 < v.NL; l0 += 32) {
        double f[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const int l = l0 + 8 * q + t;
            double x = 0.0;
            if (k_ok && l < v.NL) {
                const double em = expm1_pos(v.c2l[l] * invT);
                x = (em < __builtin_inf()) ? rcp_f64(em) : 0.0;  // 0 once e^x overflows
            }
            f[t] = x;
        }
#pragma unroll
        for (int st = 0; st < LT_SG; ++st) {
            const int s_tile = sg0 + st * 16;
            if (s_tile >= v.S) break;  // uniform
            const int s = s_tile + row;
            const double* wr = v.kdb + (int64_t)(s < v.S ? s : 0) * v.NL;
            double a[8];
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const int l = l0 + 8 * q + t;
                a[t] = (s < v.S && l < v.NL) ? wr[l] : 0.0;
            }
#pragma unroll
            for (int t = 0; t < 8; ++t)
                acc[st] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[t], f[t], acc[st], 0, 0, 0);
        }
    }
#pragma unroll
    for (int st = 0; st < LT_SG; ++st) {
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
            const int sr = sg0 + st * 16 + q + 4 * jj;
            if (sr < v.S && k < v.N)
                fwd[(int64_t)sr * v.N + k] =
                    (v.mode == DUST_TABLE_LINEAR) ? acc[st][jj] : log(acc[st][jj]);
        }
    }
}

// The product for a single plan: a workgroup takes one block of 16 points
// and one grain tile, its four waves split the wavelength steps (wave w
// takes steps w, w + 4, ...) and the partial accumulators meet in LDS.  A
// single grid has too few (point block, grain tile) pairs to fill the GPU
// with one wave each, and each wave's chain of FP64 exponentials is then the
// whole wavelength range.
__device__ __forceinline__ void ltab_gemm_split_body(const RefreshJob& j, int bx, int by) {
    typedef double f64x4 __attribute__((ext_vector_type(4)));
    __shared__ f64x4 part[3][64];
    const PlanView& v = j.v;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int row = lane & 15, q = lane >> 4;
    const int k = bx * 16 + row;
    const int s = by * 16 + row;
    const bool k_ok = k < v.N;
    const double invT = !k_ok ? 0.0
                        : (v.mode == DUST_TABLE_LINEAR ? 1.0 / v.texp[k]
                                                       : exp(-(v.lnTmin + k * v.hstep)));
    const double* wr = v.kdb + (int64_t)(s < v.S ? s : 0) * v.NL;
    f64x4 acc = f64x4{0.0, 0.0, 0.0, 0.0};
    for (int l0 = 32 * wave; l0 < v.NL; l0 += 128) {
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const int l = l0 + 8 * q + t;
            double f = 0.0, a = 0.0;
            if (l < v.NL) {
                if (k_ok) {
                    const double em = expm1_pos(v.c2l[l] * invT);
                    f = (em < __builtin_inf()) ? rcp_f64(em) : 0.0;  // 0 once e^x overflows
                }
                if (s < v.S) a = wr[l];
            }
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, f, acc, 0, 0, 0);
        }
    }
    if (wave > 0) part[wave - 1][lane] = acc;
    __syncthreads();
    if (wave == 0) {
        acc += part[0][lane] + part[1][lane] + part[2][lane];
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
            const int sr = by * 16 + q + 4 * jj;
            if (sr < v.S && k_ok)
                j.fwd[(int64_t)sr * v.N + k] = (v.mode == DUST_TABLE_LINEAR) ? acc[jj] : log(acc[jj]);
        }
    }
}

// Table-linear: one thread per (grain, node); node j sits at
// ln P' = ylo + j (yhi - ylo) / (M - 1) and kidx[s][j] is the largest k in
// [0, N-2] with ln P'_k <= that value (0 if none).
__device__ __forceinline__ void kidx_body(const RefreshJob& job, int bx, int by) {
    const PlanView& v = job.v;
    const double* __restrict__ fwd = job.fwd;
    int* kidx = job.kidx;
    double* ylo = job.ylo; double* yhi = job.yhi; double* dyinv = job.dyinv;
    const int j = bx * blockDim.x + threadIdx.x;
    const int s = by;
    if (j >= v.M) return;
    const int N = v.N;
    const double* P = fwd + (int64_t)s * N;
    const double y0 = log(P[0]), y1 = log(P[N - 1]);
    const double dinv = (v.M - 1) / (y1 - y0);
    if (j == 0) {
        ylo[s] = y0;
        yhi[s] = y1;
        dyinv[s] = dinv;
    }
    const double yj = (j == v.M - 1) ? y1 : y0 + j / dinv;
    int lo = 0, hi = N - 2;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (log(P[mid]) <= yj) lo = mid; else hi = mid - 1;
    }
    kidx[(int64_t)s * v.M + j] = lo;
}

// One thread per (grain, inverse node): ln T at y_j = ylo + j dy, by Newton
// on the forward table's cubic, and dy * d ln T / dy there.
__device__ __forceinline__ void inv_body(const RefreshJob& job, int bx, int by) {
    const PlanView& v = job.v;
    const double* __restrict__ fwd = job.fwd;
    double* ylo = job.ylo; double* yhi = job.yhi; double* dyinv = job.dyinv;
    double2* invd = job.invd;
    float2* invf = job.invf; float* ylof = job.ylof; float* dyinvf = job.dyinvf;
    const int j = bx * blockDim.x + threadIdx.x;
    const int s = by;
    if (j >= v.M) return;
    const int N = v.N;
    const double* f = fwd + (int64_t)s * N;
    const double y0 = f[0], y1 = f[N - 1];
    const double dinv = (v.M - 1) / (y1 - y0);
    if (j == 0) {
        ylo[s] = y0;
        yhi[s] = y1;
        dyinv[s] = dinv;
        ylof[s] = (float)y0;
        dyinvf[s] = (float)dinv;
    }
    const double yj = (j == v.M - 1) ? y1 : y0 + j / dinv;
    // largest k in [0, N-2] with y_k <= yj
    int lo = 0, hi = N - 2;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (f[mid] <= yj) lo = mid; else hi = mid - 1;
    }
    const int j0 = stencil_start(lo, N);
    const double a0 = f[j0], a1 = f[j0 + 1], a2 = f[j0 + 2], a3 = f[j0 + 3];
    double x = lo - j0 + ((f[lo + 1] > f[lo]) ? (yj - f[lo]) / (f[lo + 1] - f[lo]) : 0.0);
    double dp = 1.0;
    for (int it = 0; it < 4; ++it) {
        const double p = cubic4(x, a0, a1, a2, a3, &dp);
        x -= (p - yj) / dp;
    }
    cubic4(x, a0, a1, a2, a3, &dp);
    // d lnT / dy = hstep / (dy/dx), scaled by the node spacing dy = 1/dinv
    const double lnTj = v.lnTmin + ((double)j0 + x) * v.hstep;
    const double mj = v.hstep / dp / dinv;
    invd[(int64_t)s * v.M + j] = make_double2(lnTj, mj);
    // the FP32 entries of the two intervals this node bounds
    const float2 nf = make_float2((float)lnTj, (float)mj);
    float2* row = invf + (int64_t)s * (v.M - 1) * 2;
    if (j < v.M - 1) row[2 * j] = nf;
    if (j > 0) row[2 * (j - 1) + 1] = nf;
}

// The stages of a refresh (0 prep, 2 table product, 3 inverse table or search
// brackets; stage 1 is empty since the product computes its Planck factors
// itself): one block of a stage's grid.
template <int STAGE, int LT_SG>
__device__ __forceinline__ void refresh_stage(const RefreshJob& j, int bx, int by) {
    if constexpr (STAGE == 0) prep_body(j, bx, by);
    else if constexpr (STAGE == 2) ltab_gemm_body<LT_SG>(j, bx, by);
    else if (j.v.mode == DUST_TABLE_LINEAR) kidx_body(j, bx, by);
    else inv_body(j, bx, by);
}

// One plan: the job by value, the stage's 2-D grid (the product in its
// split form).
template <int STAGE>
__global__ __launch_bounds__(256) void refresh_kernel(RefreshJob j) {
    if constexpr (STAGE == 2)
        ltab_gemm_split_body(j, blockIdx.x, blockIdx.y);
    else
        refresh_stage<STAGE, LT_SG_SINGLE>(j, blockIdx.x, blockIdx.y);
}

// Many plans in one launch: the flat block index is located among the plans'
// consecutive ranges (starts[p] = first block of plan p, ascending) and
// unfolded into that plan's 2-D grid of x extent gx.
template <int STAGE>
__global__ __launch_bounds__(256) void refresh_batched_kernel(const RefreshJob* __restrict__ jobs,
                                                              const int* __restrict__ starts,
                                                              int n_jobs) {
    const int b = blockIdx.x;
    int lo = 0, hi = n_jobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (starts[mid] <= b) lo = mid; else hi = mid - 1;
    }
    const RefreshJob& j = jobs[lo];
    const int local = b - starts[lo];
    const int gx = j.gx[STAGE];
    refresh_stage<STAGE, LT_SG_BATCHED>(j, local % gx, local / gx);
}

template <int STAGE>
hipError_t launch_stage(const RefreshJob& j, hipStream_t st) {
    // the single-plan product: one (16-point block, grain tile) per workgroup
    const int gx = (STAGE == 2) ? (j.v.N + 15) / 16 : j.gx[STAGE];
    const int gy = (STAGE == 2) ? (j.v.S + 15) / 16 : j.gy[STAGE];
    hipLaunchKernelGGL(refresh_kernel<STAGE>, dim3(gx, gy), dim3(256), 0, st, j);
    return hipGetLastError();
}

template <int STAGE>
hipError_t launch_batched_stage(const RefreshJob* d_jobs, const int* d_starts, int n_jobs,
                                int blocks, hipStream_t st) {
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(refresh_batched_kernel<STAGE>, dim3(blocks), dim3(256), 0, st, d_jobs,
                       d_starts, n_jobs);
    return hipGetLastError();
}

}  // namespace

void make_refresh_job(const dust_plan* p, RefreshJob* j) {
    const PlanView& v = p->view;
    *j = RefreshJob{};
    j->v = v;
    j->lam = p->d_lam; j->dlam = p->d_dlam; j->cabs = p->d_cabs; j->w = p->d_w;
    j->es = p->d_es; j->ge = p->ge;
    j->nu = p->d_nu; j->kf = p->d_kf; j->kb = p->d_kb; j->ku = p->d_ku; j->em = p->d_em;
    j->khi = p->d_khi; j->klo = p->d_klo; j->kdb = p->d_kdb; j->c2l = p->d_c2l;
    j->fwd = p->d_fwd; j->ylo = p->d_ylo; j->yhi = p->d_yhi;
    j->dyinv = p->d_dyinv; j->kidx = p->d_kidx; j->invd = p->d_invd;
    j->invf = reinterpret_cast<float2*>(p->d_invf);
    j->ylof = p->d_ylof; j->dyinvf = p->d_dyinvf;
    const bool tab = table_mode(v.mode);
    j->gx[0] = (v.NLp + 255) / 256;  j->gy[0] = v.Sp;
    j->gx[1] = 1;                    j->gy[1] = 0;
    j->gx[2] = (v.N + 63) / 64;
    j->gy[2] = tab ? (v.S + LT_SG_BATCHED * 16 - 1) / (LT_SG_BATCHED * 16) : 0;  // batched launches
    j->gx[3] = (v.M + 255) / 256;    j->gy[3] = tab ? v.S : 0;
}

hipError_t launch_prepare(const dust_plan* p, hipStream_t st) {
    RefreshJob j;
    make_refresh_job(p, &j);
    hipError_t e = launch_stage<0>(j, st);
    if (e != hipSuccess || !table_mode(j.v.mode)) return e;
    if ((e = launch_stage<2>(j, st)) != hipSuccess) return e;
    return launch_stage<3>(j, st);
}

hipError_t launch_prepare_batched(const RefreshJob* d_jobs, const int* const d_starts[4],
                                  int n_jobs, const int blocks[4], hipStream_t st) {
    hipError_t e;
    if ((e = launch_batched_stage<0>(d_jobs, d_starts[0], n_jobs, blocks[0], st)) != hipSuccess) return e;
    if ((e = launch_batched_stage<2>(d_jobs, d_starts[2], n_jobs, blocks[2], st)) != hipSuccess) return e;
    return launch_batched_stage<3>(d_jobs, d_starts[3], n_jobs, blocks[3], st);
}

}  // namespace dust
