// C-ABI entry points and the plan's host side.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <string>
#include <vector>

#include "device_common.h"

namespace dust {

static thread_local std::string g_last_error;

dust_status set_error(dust_status code, const std::string& msg) {
    g_last_error = msg;
    return code;
}

void clear_error() { g_last_error.clear(); }

dust_status hip_error(hipError_t e, const char* what) {
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    return set_error(e == hipErrorOutOfMemory ? DUST_ENOMEM : DUST_EDEVICE, m);
}

namespace {

constexpr int MAX_GRAINS = 1024;      // the LDS tile of the emission holds 16 x S floats
constexpr int MAX_LAMBDA = 1 << 20;
constexpr int MAX_TABLE = 65535;      // table indices are uint16

int round_up(int x, int m) { return (x + m - 1) / m * m; }

bool finite_nonneg(const double* a, int64_t n) {
    for (int64_t i = 0; i < n; ++i)
        if (!(a[i] >= 0.0) || !isfinite(a[i])) return false;
    return true;
}

}  // namespace

// Checks a grid descriptor (also used by the fluctuating-grain plan).
dust_status validate_grid(const dust_grid_desc* g) {
    if (!g) return set_error(DUST_EINVAL, "grid descriptor is NULL");
    if (g->n_lambda < 1 || g->n_lambda > MAX_LAMBDA)
        return set_error(DUST_EINVAL, "n_lambda must be in [1, 2^20]");
    if (g->n_grains < 1)
        return set_error(DUST_EINVAL, "n_grains must be >= 1");
    if (g->n_grains > MAX_GRAINS)
        return set_error(DUST_EUNSUPPORTED, "n_grains above 1024 is not supported");
    if (!g->lambda || !g->dlambda || !g->c_abs || !g->weight || !g->size)
        return set_error(DUST_EINVAL, "a grid table pointer is NULL");
    const int NL = g->n_lambda, S = g->n_grains;
    for (int l = 0; l < NL; ++l) {
        if (!(g->lambda[l] > 0.0) || !isfinite(g->lambda[l]))
            return set_error(DUST_EINVAL, "lambda must be finite and > 0");
        if (l > 0 && !(g->lambda[l] > g->lambda[l - 1]))
            return set_error(DUST_EINVAL, "lambda must be strictly increasing");
    }
    if (!finite_nonneg(g->dlambda, NL)) return set_error(DUST_EINVAL, "dlambda must be finite and >= 0");
    if (!finite_nonneg(g->c_abs, (int64_t)NL * S)) return set_error(DUST_EINVAL, "c_abs must be finite and >= 0");
    if (!finite_nonneg(g->weight, S)) return set_error(DUST_EINVAL, "weight must be finite and >= 0");
    for (int s = 0; s < S; ++s)
        if (!(g->size[s] > 0.0) || !isfinite(g->size[s]))
            return set_error(DUST_EINVAL, "size must be finite and > 0");
    return DUST_OK;
}

namespace {

dust_status resolve_options(const dust_options* in, dust_options* o) {
    dust_options d;
    memset(&d, 0, sizeof d);
    if (in) d = *in;
    if (d.mode != DUST_PLAIN_FP32 && d.mode != DUST_MIXED && d.mode != DUST_TABLE_LINEAR)
        return set_error(DUST_EINVAL, "mode must be DUST_PLAIN_FP32, DUST_MIXED or DUST_TABLE_LINEAR");
    const bool lin = d.mode == DUST_TABLE_LINEAR;
    if (d.maxit < 0) return set_error(DUST_EINVAL, "maxit must be >= 0");
    if (d.maxit == 0) d.maxit = 50;
    if (!(d.tol >= 0.0) || !isfinite(d.tol)) return set_error(DUST_EINVAL, "tol must be finite and >= 0");
    if (d.tol == 0.0) d.tol = 1e-5;
    if (d.ltab_n < 0 || (d.ltab_n > 0 && d.ltab_n < 16) || d.ltab_n > MAX_TABLE / 4)
        return set_error(DUST_EINVAL, "ltab_n must be 0 (default) or in [16, 16383]");
    if (d.ltab_n == 0) d.ltab_n = lin ? 2000 : 1024;
    if (d.fused_kernels < 0 || d.fused_kernels > 2)
        return set_error(DUST_EINVAL, "fused_kernels must be 0, 1 or 2");
    if (d.reserved != 0) return set_error(DUST_EINVAL, "dust_options.reserved must be 0");
    d.f32_lookup = d.f32_lookup != 0;
    d.newton_polish = d.newton_polish != 0;
    if (d.newton_polish && (d.mode != DUST_MIXED || d.f32_lookup))
        return set_error(DUST_EINVAL, "newton_polish needs DUST_MIXED with the FP64 lookup");
    if (d.ltab_tmin == 0.0) d.ltab_tmin = lin ? 3.0 : 2.7;
    if (d.ltab_tmax == 0.0) d.ltab_tmax = lin ? 1500.0 : 3000.0;
    if (!(d.ltab_tmin > 0.0) || !(d.ltab_tmax > d.ltab_tmin) || !isfinite(d.ltab_tmax) ||
        d.ltab_tmin < 1e-2 || d.ltab_tmax > 1e6)
        return set_error(DUST_EINVAL, "need 0.01 <= ltab_tmin < ltab_tmax <= 1e6");
    *o = d;
    return DUST_OK;
}

template <typename T>
hipError_t dev_alloc(T** p, size_t n) {
    *p = nullptr;
    return hipMalloc((void**)p, n * sizeof(T) > 0 ? n * sizeof(T) : 1);
}

void free_plan(dust_plan* p) {
    if (!p) return;
    void* ptrs[] = {p->d_lam, p->d_dlam, p->d_cabs, p->d_w,   p->d_size, p->d_es,   p->d_nu,
                    p->d_hscale, p->d_hinv, p->d_gs, p->d_kf,  p->d_kb,   p->d_em,   p->d_khi,
                    p->d_klo, p->d_kdb,  p->d_c2l,  p->d_fwd, p->d_ylo,  p->d_yhi,
                    p->d_dyinv, p->d_texp, p->d_lntab, p->d_kidx, p->d_invd, p->d_invf,
                    p->d_ylof, p->d_dyinvf, p->d_ku};
    for (void* q : ptrs)
        if (q) (void)hipFree(q);
    delete p;
}

}  // namespace
}  // namespace dust

using namespace dust;

extern "C" {

const char* dust_last_error(void) { return g_last_error.c_str(); }

const char* dust_version(void) { return "libdust 0.1 (gfx950)"; }

dust_status dust_plan_create(const dust_grid_desc* g, const dust_options* opt, dust_plan** out) {
    g_last_error.clear();
    if (!out) return set_error(DUST_EINVAL, "out is NULL");
    *out = nullptr;
    dust_status st = validate_grid(g);
    if (st != DUST_OK) return st;
    dust_options o;
    st = resolve_options(opt, &o);
    if (st != DUST_OK) return st;

    const int NL = g->n_lambda, S = g->n_grains;
    const int NLp = round_up(NL, PAD_L), Sp = round_up(S, PAD_S);

    // Host side: one exact power of two per grain puts max_l C dlam into
    // [0.5, 1); one for the whole emission table puts its maximum there.
    std::vector<int> es(Sp, 0);
    std::vector<float> hscale(Sp, 1.0f), hinv(Sp, 1.0f), gs(Sp, 0.0f);
    double emax = 0.0;
    for (int s = 0; s < S; ++s) {
        double kmax = 0.0, kbmax = 0.0;
        for (int l = 0; l < NL; ++l) {
            const double lm = g->lambda[l];
            const double K = g->c_abs[(int64_t)s * NL + l] * g->dlambda[l];
            kmax = fmax(kmax, K);
            // the solve's weights and its slope weights (times c2 log2(e) / lam)
            kbmax = fmax(kbmax, K * RAD_C1 / (lm * lm * lm * lm * lm) *
                                    fmax(1.0, RAD_C2 * LOG2E / lm));
            emax = fmax(emax, g->weight[s] * g->c_abs[(int64_t)s * NL + l] * RAD_C1 /
                                  (lm * lm * lm * lm * lm));
        }
        int e = 0;
        if (kmax > 0.0) (void)frexp(kmax, &e);
        es[s] = -e;
        if (kmax > 0.0 && !(ldexp(kbmax, -e) < 1e37))
            return set_error(DUST_EUNSUPPORTED,
                             "C dlam c1 lam^-5 (c2 / lam) spans more than FP32 holds for a grain");
        if (es[s] < -126 || es[s] > 126)
            return set_error(DUST_EUNSUPPORTED, "C dlam outside the FP32 exponent range");
        hscale[s] = ldexpf(1.0f, es[s]);
        hinv[s] = ldexpf(1.0f, -es[s]);
        const double la = log10(g->size[s]);
        gs[s] = (float)(log10(4.0 * M_PI) + es[s] * -log10(2.0) + -1.39 * la + 0.126 * la * la);
    }
    int ge = 0;
    if (emax > 0.0) (void)frexp(emax, &ge);
    if (ge < -100 || ge > 100)
        return set_error(DUST_EUNSUPPORTED, "emission weights outside the FP32 range");

    hipError_t e;
    int dev = 0;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return hip_error(e, "hipGetDevice");
    int max_lds = 65536;
    (void)hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    if (emit_lds_bytes(16, Sp) > (size_t)max_lds) {
        int lim = 16;
        while (emit_lds_bytes(16, lim + 16) <= (size_t)max_lds) lim += 16;
        return set_error(DUST_EUNSUPPORTED,
                         "n_grains too large for one emission tile in LDS on this device (limit " +
                             std::to_string(lim) + ")");
    }

    dust_plan* p = new dust_plan;
    memset(p, 0, sizeof *p);
    p->device = dev;
    p->opt = o;
    p->NL = NL; p->S = S; p->NLp = NLp; p->Sp = Sp;
    p->ge = ge;
    p->N = o.ltab_n;
    const bool lin = o.mode == DUST_TABLE_LINEAR;
    // nodes of the inverse table (mixed: a start for Newton only) or of the
    // search brackets (table-linear)
    p->M = lin ? 2048 : (o.ltab_n < 256 ? o.ltab_n : 256);
    p->lnTmin = log(o.ltab_tmin);
    p->hstep = (log(o.ltab_tmax) - log(o.ltab_tmin)) / (p->N - 1);
    const double tstep = (o.ltab_tmax - o.ltab_tmin) / (p->N - 1);
    const bool mixed = table_mode(o.mode);

#define ALLOC(ptr, n)                                              \
    if ((e = dev_alloc(&(ptr), (n))) != hipSuccess) {               \
        free_plan(p);                                              \
        return hip_error(e, "hipMalloc (" #ptr ")");               \
    }
    ALLOC(p->d_lam, NL);
    ALLOC(p->d_dlam, NL);
    ALLOC(p->d_cabs, (size_t)S * NL);
    ALLOC(p->d_w, S);
    ALLOC(p->d_size, S);
    ALLOC(p->d_es, Sp);
    ALLOC(p->d_nu, NLp);
    ALLOC(p->d_hscale, Sp);
    ALLOC(p->d_hinv, Sp);
    ALLOC(p->d_gs, Sp);
    ALLOC(p->d_kf, (size_t)Sp * NLp);
    ALLOC(p->d_kb, (size_t)Sp * NLp);
    ALLOC(p->d_ku, (size_t)Sp * NLp);
    ALLOC(p->d_em, (size_t)Sp * NLp);
    ALLOC(p->d_khi, (size_t)Sp * NLp);
    ALLOC(p->d_klo, (size_t)Sp * NLp);
    ALLOC(p->d_kdb, (size_t)S * NL);
    ALLOC(p->d_c2l, NL);
    if (mixed) {
        ALLOC(p->d_fwd, (size_t)S * p->N);
        if (lin) {
            ALLOC(p->d_kidx, (size_t)S * p->M);
        } else {
            ALLOC(p->d_invd, (size_t)S * p->M);
            ALLOC(p->d_invf, (size_t)S * (p->M - 1));
            ALLOC(p->d_ylof, S);
            ALLOC(p->d_dyinvf, S);
        }
        ALLOC(p->d_ylo, S);
        ALLOC(p->d_yhi, S);
        ALLOC(p->d_dyinv, S);
        ALLOC(p->d_texp, p->N);
        ALLOC(p->d_lntab, 256);
    }
#undef ALLOC

    struct Up { void* d; const void* h; size_t n; } ups[] = {
        {p->d_lam, g->lambda, sizeof(double) * NL},
        {p->d_dlam, g->dlambda, sizeof(double) * NL},
        {p->d_cabs, g->c_abs, sizeof(double) * S * (size_t)NL},
        {p->d_w, g->weight, sizeof(double) * S},
        {p->d_size, g->size, sizeof(double) * S},
        {p->d_es, es.data(), sizeof(int) * Sp},
        {p->d_hscale, hscale.data(), sizeof(float) * Sp},
        {p->d_hinv, hinv.data(), sizeof(float) * Sp},
        {p->d_gs, gs.data(), sizeof(float) * Sp},
    };
    // Static helper tables of the mixed lookup (they depend only on the
    // table range): T_k, and ln c_i, 1/c_i for the 256 mantissa intervals.
    std::vector<double> texp;
    std::vector<double2> lntab;
    if (mixed) {
        texp.resize(p->N);
        for (int k = 0; k < p->N; ++k)
            texp[k] = lin ? o.ltab_tmin + k * tstep : exp(p->lnTmin + k * p->hstep);
        lntab.resize(256);
        for (int i = 0; i < 256; ++i) {
            const double c = 1.0 + i / 256.0;
            lntab[i] = make_double2(log(c), 1.0 / c);
        }
        if ((e = hipMemcpy(p->d_texp, texp.data(), sizeof(double) * p->N, hipMemcpyHostToDevice)) != hipSuccess ||
            (e = hipMemcpy(p->d_lntab, lntab.data(), sizeof(double2) * 256, hipMemcpyHostToDevice)) != hipSuccess) {
            free_plan(p);
            return hip_error(e, "hipMemcpy (lookup tables)");
        }
    }
    for (const Up& u : ups) {
        if ((e = hipMemcpy(u.d, u.h, u.n, hipMemcpyHostToDevice)) != hipSuccess) {
            free_plan(p);
            return hip_error(e, "hipMemcpy (grid upload)");
        }
    }

    PlanView& v = p->view;
    v.NL = NL; v.S = S; v.NLp = NLp; v.Sp = Sp;
    v.mode = o.mode;
    v.maxit = o.maxit;
    v.tol = (float)o.tol;
    v.nu = p->d_nu;
    v.hscale = p->d_hscale;
    v.hinv = p->d_hinv;
    v.gs = p->d_gs;
    v.kf = p->d_kf;
    v.khi = p->d_khi;
    v.klo = p->d_klo;
    v.kb = p->d_kb;
    v.ku = p->d_ku;
    v.em = p->d_em;
    v.escale = ldexpf(1.0f, ge);
    v.kdb = p->d_kdb;
    v.c2l = p->d_c2l;
    v.fwd = p->d_fwd;
    v.ylo = p->d_ylo;
    v.yhi = p->d_yhi;
    v.dyinv = p->d_dyinv;
    v.N = p->N;
    v.M = p->M;
    v.lnTmin = p->lnTmin;
    v.hstep = p->hstep;
    v.texp = p->d_texp;
    v.lntab = p->d_lntab;
    v.kidx = p->d_kidx;
    v.invd = p->d_invd;
    v.invf = p->d_invf;
    v.ylof = p->d_ylof;
    v.dyinvf = p->d_dyinvf;
    v.f32_lookup = o.f32_lookup;
    v.polish = o.newton_polish;
    v.tstep = tstep;
    v.q = nullptr;
    v.ldq = 0;
    v.warm = 0;

    if ((e = launch_prepare(p, nullptr)) != hipSuccess) {
        free_plan(p);
        return hip_error(e, "plan kernels");
    }
    if ((e = hipDeviceSynchronize()) != hipSuccess) {
        free_plan(p);
        return hip_error(e, "plan kernels (synchronize)");
    }
    *out = p;
    return DUST_OK;
}

dust_status dust_plan_destroy(dust_plan* p) {
    g_last_error.clear();
    if (!p) return DUST_OK;
    hipError_t e = hipDeviceSynchronize();
    free_plan(p);
    return e == hipSuccess ? DUST_OK : hip_error(e, "hipDeviceSynchronize");
}

dust_status dust_plan_prepare(dust_plan* p, void* stream) {
    g_last_error.clear();
    if (!p) return set_error(DUST_EINVAL, "plan is NULL");
    hipError_t e = launch_prepare(p, (hipStream_t)stream);
    return e == hipSuccess ? DUST_OK : hip_error(e, "plan kernels");
}

dust_status dust_plan_info(const dust_plan* p, int32_t* nl, int32_t* ns, int32_t* mode) {
    g_last_error.clear();
    if (!p) return set_error(DUST_EINVAL, "plan is NULL");
    if (nl) *nl = p->NL;
    if (ns) *ns = p->S;
    if (mode) *mode = p->opt.mode;
    return DUST_OK;
}

static dust_status check_common(const dust_plan* p, int64_t n_cells) {
    if (!p) return set_error(DUST_EINVAL, "plan is NULL");
    if (n_cells < 0) return set_error(DUST_EINVAL, "n_cells must be >= 0");
    if (n_cells > ((int64_t)1 << 40)) return set_error(DUST_EINVAL, "n_cells too large");
    return DUST_OK;
}

static dust_status check_buf(const void* ptr, int64_t ld, int64_t width, int64_t n_cells,
                             const char* name) {
    if (n_cells == 0) return DUST_OK;
    if (!ptr) return set_error(DUST_EINVAL, std::string(name) + " is NULL");
    if (((uintptr_t)ptr & 3u) != 0) return set_error(DUST_EINVAL, std::string(name) + " is not 4-byte aligned");
    if (ld < width) return set_error(DUST_EINVAL, std::string("leading dimension of ") + name + " is smaller than its row");
    return DUST_OK;
}

dust_status dust_absorb(dust_plan* p, int64_t C, const float* J, int64_t ldj, float* H,
                        int64_t ldh, void* stream) {
    g_last_error.clear();
    dust_status st;
    if ((st = check_common(p, C)) != DUST_OK) return st;
    if ((st = check_buf(J, ldj, p->NL, C, "J")) != DUST_OK) return st;
    if ((st = check_buf(H, ldh, p->S, C, "H")) != DUST_OK) return st;
    hipError_t e = launch_absorb(p->view, C, J, ldj, H, ldh, (hipStream_t)stream);
    return e == hipSuccess ? DUST_OK : hip_error(e, "absorb launch");
}

// The per-call view: the plan's tables plus the optional solve inputs.
static dust_status apply_ext(const dust_plan* p, const dust_solve_ext* x, int64_t C,
                             PlanView* v) {
    *v = p->view;
    if (!x) return DUST_OK;
    if (x->reserved != 0) return set_error(DUST_EINVAL, "dust_solve_ext.reserved must be 0");
    if (x->Q) {
        dust_status st = check_buf(x->Q, x->ldq, p->S, C, "Q");
        if (st != DUST_OK) return st;
        v->q = x->Q;
        v->ldq = x->ldq;
    }
    v->warm = x->warm_start != 0;
    return DUST_OK;
}

dust_status dust_solve_T_ext(dust_plan* p, int64_t C, const float* H, int64_t ldh,
                             const dust_solve_ext* ext, float* T, int64_t ldt,
                             dust_counters* cnt, void* stream) {
    g_last_error.clear();
    dust_status st;
    if ((st = check_common(p, C)) != DUST_OK) return st;
    if ((st = check_buf(H, ldh, p->S, C, "H")) != DUST_OK) return st;
    if ((st = check_buf(T, ldt, p->S, C, "T")) != DUST_OK) return st;
    if (cnt && ((uintptr_t)cnt & 7u)) return set_error(DUST_EINVAL, "counters must be 8-byte aligned");
    PlanView v;
    if ((st = apply_ext(p, ext, C, &v)) != DUST_OK) return st;
    hipError_t e = launch_solve(v, C, H, ldh, T, ldt, cnt, (hipStream_t)stream);
    return e == hipSuccess ? DUST_OK : hip_error(e, "solve launch");
}

dust_status dust_solve_T(dust_plan* p, int64_t C, const float* H, int64_t ldh, float* T,
                         int64_t ldt, dust_counters* cnt, void* stream) {
    return dust_solve_T_ext(p, C, H, ldh, nullptr, T, ldt, cnt, stream);
}

dust_status dust_emit_sed(dust_plan* p, int64_t C, const float* T, int64_t ldt, const float* m,
                          float* L, int64_t ldl, void* stream) {
    g_last_error.clear();
    dust_status st;
    if ((st = check_common(p, C)) != DUST_OK) return st;
    if ((st = check_buf(T, ldt, p->S, C, "T")) != DUST_OK) return st;
    if ((st = check_buf(L, ldl, p->NL, C, "L")) != DUST_OK) return st;
    if (m && ((uintptr_t)m & 3u)) return set_error(DUST_EINVAL, "m_dust is not 4-byte aligned");
    hipError_t e = launch_emit(p->view, C, T, ldt, m, L, ldl, (hipStream_t)stream);
    return e == hipSuccess ? DUST_OK : hip_error(e, "emit launch");
}

dust_status dust_run_fused_ext(dust_plan* p, int64_t C, const float* J, int64_t ldj,
                               const float* m, const dust_solve_ext* ext, float* T, int64_t ldt,
                               float* L, int64_t ldl, dust_counters* cnt, void* stream) {
    g_last_error.clear();
    dust_status st;
    if ((st = check_common(p, C)) != DUST_OK) return st;
    if ((st = check_buf(J, ldj, p->NL, C, "J")) != DUST_OK) return st;
    if ((st = check_buf(T, ldt, p->S, C, "T")) != DUST_OK) return st;
    if ((st = check_buf(L, ldl, p->NL, C, "L")) != DUST_OK) return st;
    if (m && ((uintptr_t)m & 3u)) return set_error(DUST_EINVAL, "m_dust is not 4-byte aligned");
    if (cnt && ((uintptr_t)cnt & 7u)) return set_error(DUST_EINVAL, "counters must be 8-byte aligned");
    PlanView v;
    if ((st = apply_ext(p, ext, C, &v)) != DUST_OK) return st;
    const hipStream_t sm = (hipStream_t)stream;
    hipError_t e = (p->opt.fused_kernels == 2)
                       ? launch_absorb_solve(v, C, J, ldj, T, ldt, cnt, sm)
                       : launch_fused(v, C, J, ldj, m, T, ldt, L, ldl, cnt, sm);
    if (e == hipSuccess && p->opt.fused_kernels == 2)
        e = launch_emit(v, C, T, ldt, m, L, ldl, sm);
    return e == hipSuccess ? DUST_OK : hip_error(e, "fused launch");
}

dust_status dust_run_fused(dust_plan* p, int64_t C, const float* J, int64_t ldj, const float* m,
                           float* T, int64_t ldt, float* L, int64_t ldl, dust_counters* cnt,
                           void* stream) {
    return dust_run_fused_ext(p, C, J, ldj, m, nullptr, T, ldt, L, ldl, cnt, stream);
}

}  // extern "C"
