/*
 * dust.h -- C-ABI of libdust: dust-grain equilibrium temperatures and the
 * resulting emission SED on an AMD MI355X (gfx950) GPU.
 *
 * The calculation is the one of Jonsson & Primack, "Accelerating Dust
 * Temperature Calculations with Graphics Processing Units" (New Astronomy),
 * Section 4: for every grid cell c and grain s (a species and size),
 *
 *   absorb   H[c,s] = sum_l J[c,l] C[s,l] dlam[l]                     (Eq. 6)
 *   solve    T[c,s] such that sum_l C[s,l] dlam[l] B(lam_l, T) = H     (Eq. 7)
 *   emit     L[c,l] = m[c] sum_s w[s] C[s,l] B(lam_l, T[c,s])          (Eqs. 8-10)
 *
 * with B the Planck function (Eq. 1), J the mean intensity of the radiation
 * field, C the absorption cross-sections, w the number of grains per unit
 * dust mass (the paper's n_s) and m the dust mass of the cell (m_d;c).
 *
 * Units: SI at the boundary (lam, dlam in m; C in m^2; grain size in m;
 * J in W m^-2 m^-1 sr^-1).  H and L carry no factor 4 pi (both sides of
 * Eq. 7 drop the same factor, so T is unaffected).
 *
 * Conventions shared by every call:
 *  - Arrays are row-major.  C = cells, NL = wavelengths, S = grains.
 *  - Grid tables (dust_grid_desc) are HOST float64 pointers, read only during
 *    dust_plan_create; the caller keeps ownership.
 *  - J, H, T, L, m_dust are DEVICE pointers on the device that was current
 *    when the plan was created, 4-byte aligned; the caller owns them.
 *    Leading dimensions (ldj, ldh, ldt, ldl) count elements and must be at
 *    least the row width (NL for J and L, S for H and T).
 *  - `stream` is a hipStream_t (NULL = the null stream).  Calls only enqueue
 *    work: they neither allocate nor synchronise, except dust_plan_create,
 *    dust_plan_destroy, dust_batch_create, dust_batch_destroy and
 *    dust_batch_run (a stream-ordered allocation of its work list).
 *  - Every argument is checked before any HIP call; a bad argument returns
 *    DUST_EINVAL and the reason is available from dust_last_error().
 *  - Numerical conditions are not errors.  They are counted in an optional
 *    DEVICE dust_counters (zero it before the call; counts are added
 *    atomically):
 *      n_nonfinite     pairs whose H is NaN, infinite or negative -> T = NaN
 *      n_unconverged   pairs where the iteration cap was reached
 *                      (the last iterate is kept)
 *      n_out_of_table  pairs of the mixed solve whose T lies outside the
 *                      tabulated range (solved exactly instead)
 *    H == 0 gives T = 0, and a grain at T = 0 emits nothing.
 *  - Calls that share a plan may run concurrently on different streams,
 *    except those that rewrite its device tables (dust_plan_prepare, and
 *    the launch of a batch made with DUST_BATCH_REFRESH_PLANS): order
 *    them against the plan's other calls (one stream, or events).
 */
#ifndef DUST_H
#define DUST_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    DUST_OK = 0,
    DUST_EINVAL = -1,       /* invalid argument (nothing was enqueued) */
    DUST_EUNSUPPORTED = -2, /* valid but outside what this library handles */
    DUST_ENOMEM = -3,       /* device allocation failed */
    DUST_EDEVICE = -4       /* a HIP runtime call failed */
} dust_status;

typedef enum {
    /* FP32 throughout: FP32 MFMA heating, FP32 Newton on the exact sum of
       Eq. 7 from the Eq. 11 guess, FP32 emission. */
    DUST_PLAIN_FP32 = 0,
    /* Mixed precision: heating on BF16 MFMA with hi+lo split operands and
       FP32 accumulation; T from per-grain tables built in FP64 (ln P at
       log-spaced T, and from it the inverse ln T(ln H) at uniform steps):
       a cubic Hermite of the inverse evaluated in FP64 between FP64 nodes
       (interpolation error about 1e-9; relative T error about 5e-7,
       dominated by the heating); with `f32_lookup` the same Hermite in FP32
       from FP32 nodes (about 2e-6).  Pairs outside the tabulated range are
       solved exactly in FP64.  FP32 emission. */
    DUST_MIXED = 1,
    /* The production variant of the temperature step (Sections 2 and 5):
       per grain, the power of Eq. 7 tabulated in FP64 at ltab_n temperatures
       evenly spaced over [ltab_tmin, ltab_tmax] (defaults 2000, 3 K, 1500 K),
       and T(H) by linear interpolation between the two table points that
       bracket H.  An approximation: its error is that of the interpolation
       (about 1e-3 relative near 20 K with the defaults, larger at lower T,
       and T never above the exact root).  H outside the table gives the end
       temperature and is counted in n_out_of_table.  Heating and emission
       as in DUST_MIXED. */
    DUST_TABLE_LINEAR = 2
} dust_mode;

/* One grid: its wavelength grid and grain set (host float64). */
typedef struct {
    int32_t n_lambda;      /* NL >= 1 */
    int32_t n_grains;      /* S  >= 1 */
    const double* lambda;  /* [NL] wavelengths (m), > 0, strictly increasing */
    const double* dlambda; /* [NL] quadrature weights of the sums (m), >= 0 */
    const double* c_abs;   /* [S][NL] absorption cross-sections (m^2), >= 0 */
    const double* weight;  /* [S] grains per unit dust mass (n_s), >= 0 */
    const double* size;    /* [S] grain radius (m), > 0; only steers the
                              Eq. 11 initial guess of the FP32 Newton solve */
} dust_grid_desc;

/* Options; a zero field selects the default shown. */
typedef struct {
    int32_t mode;      /* dust_mode; default DUST_PLAIN_FP32 */
    int32_t maxit;     /* plain: Newton iteration cap, default 50 */
    double tol;        /* plain: stop when |P(T)/H - 1| <= tol, default 1e-5 */
    int32_t ltab_n;    /* table points per grain: mixed default 1024 (>= 16),
                          table-linear default 2000 (>= 16) */
    int32_t fused_kernels; /* dust_run_fused: 0 = library choice, 1 = one kernel
                              (absorb, solve and emit per cell tile), 2 = two
                              kernels (absorb + solve per tile, T written once;
                              then emit).  H never reaches device memory. */
    double ltab_tmin;  /* lowest tabulated T (K): mixed 2.7, table-linear 3 */
    double ltab_tmax;  /* highest tabulated T (K): mixed 3000, table-linear 1500 */
    int32_t f32_lookup; /* mixed: nonzero replaces the FP64 inverse-table
                           lookup by the FP32 one */
    int32_t newton_polish; /* mixed (FP64 lookup): nonzero follows the lookup
                           with an FP64 bracketed-Newton polish of Eq. 7 on the
                           grain's forward table of ln P at the ltab_n
                           temperatures (the cubic through the four table
                           values around the bracketing interval); T is then
                           the table's root to about 1e-11 before FP32
                           rounding.  Not for batched launches. */
    int32_t reserved;  /* must be 0 */
} dust_options;

/* Device-side event counters (see the conventions above). */
typedef struct {
    int64_t n_nonfinite;
    int64_t n_unconverged;
    int64_t n_out_of_table;
    int64_t n_newton_evals;  /* DUST_PLAIN_FP32: evaluations of Eq. 7's sum
                                (pairs x Newton iterations) */
} dust_counters;

/* Optional inputs of the temperature step (dust_solve_T_ext,
 * dust_run_fused_ext).  A zeroed struct, or NULL, means neither.
 *
 *  Q           DEVICE [n_cells][ldq] float: heating from sources other than
 *              the radiation field (Section 2 names collisions with energetic
 *              electrons), in the units of H.  The balance of Eq. 7 is solved
 *              for H + Q.  NULL: none.
 *  warm_start  nonzero: on entry T holds temperatures from a previous call
 *              (the passes of the global iteration Section 2 describes for
 *              dust that absorbs its own emission) and DUST_PLAIN_FP32 starts
 *              Newton there instead of at the Eq. 11 guess; entries that are
 *              not finite and > 0 fall back to the guess.  The root is the
 *              same; only the iteration count changes.  The table modes start
 *              from their own O(1) lookup and ignore it. */
typedef struct {
    const float* Q;
    int64_t ldq;
    int32_t warm_start;
    int32_t reserved;  /* must be 0 */
} dust_solve_ext;

/* Opaque, library-owned plan: the grid's derived device tables. */
typedef struct dust_plan dust_plan;

/* Build a plan on the current device: upload the grid, derive the kernel
 * tables (the paper's first kernel, Section 4.1: C dlam per grain and
 * wavelength, plus the emission weights and, for DUST_MIXED, the FP64
 * power tables) and wait for them.  Allocates device memory. */
dust_status dust_plan_create(const dust_grid_desc* grid, const dust_options* opt,
                             dust_plan** out);

/* Free a plan (waits for the device).  NULL is accepted. */
dust_status dust_plan_destroy(dust_plan* plan);

/* Re-derive the plan's tables on `stream` from its stored float64 grid
 * (the same work dust_plan_create does, without allocating). */
dust_status dust_plan_prepare(dust_plan* plan, void* stream);

/* Query plan sizes: any pointer may be NULL. */
dust_status dust_plan_info(const dust_plan* plan, int32_t* n_lambda,
                           int32_t* n_grains, int32_t* mode);

/* Eq. 6 (Section 4.2): H[c*ldh + s] for c < n_cells, s < S, FP32 output.
 * Any 4-byte aligned J is accepted; J 16-byte aligned with ldj a multiple of
 * 4 (every row 16-byte aligned) takes the fastest form, which loads J
 * straight into on-chip memory. */
dust_status dust_absorb(dust_plan* plan, int64_t n_cells,
                        const float* J, int64_t ldj,
                        float* H, int64_t ldh, void* stream);

/* Eq. 7 (Section 4.3): T[c*ldt + s] from H[c*ldh + s].  `counters` may be
 * NULL. */
dust_status dust_solve_T(dust_plan* plan, int64_t n_cells,
                         const float* H, int64_t ldh,
                         float* T, int64_t ldt,
                         dust_counters* counters, void* stream);

/* dust_solve_T with the optional inputs of dust_solve_ext (ext may be NULL).
 * With warm_start, T is read before it is written (in place). */
dust_status dust_solve_T_ext(dust_plan* plan, int64_t n_cells,
                             const float* H, int64_t ldh,
                             const dust_solve_ext* ext,
                             float* T, int64_t ldt,
                             dust_counters* counters, void* stream);

/* Eqs. 9-10 (Section 4.4): L[c*ldl + l] from T[c*ldt + s].  m_dust may be
 * NULL (every cell has unit dust mass). */
dust_status dust_emit_sed(dust_plan* plan, int64_t n_cells,
                          const float* T, int64_t ldt, const float* m_dust,
                          float* L, int64_t ldl, void* stream);

/* Eqs. 6, 7, 9-10 in one launch per cell tile: H stays on chip and never
 * reaches device memory.  Same results as absorb -> solve -> emit. */
dust_status dust_run_fused(dust_plan* plan, int64_t n_cells,
                           const float* J, int64_t ldj, const float* m_dust,
                           float* T, int64_t ldt, float* L, int64_t ldl,
                           dust_counters* counters, void* stream);

/* dust_run_fused with the optional inputs of dust_solve_ext (ext may be
 * NULL): Q is added to the on-chip heating; with warm_start, T is read
 * before it is written (in place). */
dust_status dust_run_fused_ext(dust_plan* plan, int64_t n_cells,
                               const float* J, int64_t ldj, const float* m_dust,
                               const dust_solve_ext* ext,
                               float* T, int64_t ldt, float* L, int64_t ldl,
                               dust_counters* counters, void* stream);

/* Many independent grids in one launch (the batching of Section 4's
 * per-cell-block decomposition over several grids; each grid is its own
 * plan).  A batch binds plans and buffers once (host arrays of length
 * n_grids; m_dust[g] may be NULL), builds the work list of (grid, cell tile)
 * items ordered by cost and records one HIP graph.  Flags:
 *   DUST_BATCH_AUTOTUNE       pick the launch form (one workgroup per item,
 *                             or a work queue with 2, 4 or 6 resident
 *                             workgroups per CU), the cells per tile (16 or
 *                             32) and the grain tiles per wave by timing
 *                             candidate launches on the bound buffers, which
 *                             it overwrites;
 *   DUST_BATCH_REFRESH_PLANS  the graph first re-derives every plan's tables
 *                             (dust_plan_prepare), so one replay is the whole
 *                             path for every grid.
 * Every launch form gives the same results, bit for bit, as dust_run_fused
 * on each grid.  All plans must be DUST_MIXED plans (FP64 lookup) of the
 * current device.  Allocates device memory and synchronises (it runs the
 * autotuner's candidates). */
typedef struct dust_batch dust_batch;

enum { DUST_BATCH_AUTOTUNE = 1, DUST_BATCH_REFRESH_PLANS = 2 };

dust_status dust_batch_create(dust_plan* const* plans, int32_t n_grids,
                              const int64_t* n_cells,
                              const float* const* J, const int64_t* ldj,
                              const float* const* m_dust,
                              float* const* T, const int64_t* ldt,
                              float* const* L, const int64_t* ldl,
                              dust_counters* counters, int32_t flags,
                              dust_batch** out);

/* Replay the batch's graph on `stream` (allocates nothing). */
dust_status dust_batch_launch(dust_batch* batch, void* stream);

/* Tile configuration the batch uses (cells per tile), for reporting. */
dust_status dust_batch_info(const dust_batch* batch, int32_t* cells_per_tile,
                            int64_t* n_items);

/* The batch's launch form: cells per tile, grain tiles per wave in one
 * heating pass, and resident workgroups per CU of the work-queue form (0: one
 * workgroup per item).  Any pointer may be NULL. */
dust_status dust_batch_form(const dust_batch* batch, int32_t* cells_per_tile,
                            int32_t* tiles_per_wave, int32_t* per_cu);

dust_status dust_batch_destroy(dust_batch* batch);

/* One-shot batched launch on `stream`: the same arguments and checks as
 * dust_batch_create, the same results, but nothing is kept.  The work list
 * (the grids' launch arguments and the (grid, tile) items) is built on the
 * host, copied into a stream-ordered device allocation (hipMallocAsync,
 * released with hipFreeAsync after the kernel on the same stream) and the
 * batched kernel runs once, one workgroup per 16-cell item (the batch's
 * default form; no autotuning, no plan refresh).  The host copy is from
 * pageable memory, so the call may wait for `stream`'s earlier work before
 * it returns; it cannot be recorded into a HIP graph (use dust_batch_create,
 * whose graph does the same work). */
dust_status dust_batch_run(dust_plan* const* plans, int32_t n_grids,
                           const int64_t* n_cells,
                           const float* const* J, const int64_t* ldj,
                           const float* const* m_dust,
                           float* const* T, const int64_t* ldt,
                           float* const* L, const int64_t* ldl,
                           dust_counters* counters, void* stream);

/* dust_batch_run for callers that cannot allocate device memory (serving
 * loops and harnesses that forbid hipMalloc): the same arguments, checks,
 * kernel and results, but the work list goes into a fixed array of 4 MiB
 * that the library reserves on every device it runs on when it is loaded
 * (a static device array, held until the process ends), instead of a
 * stream-ordered allocation.  It calls no allocating routine.  Limits,
 * checked before any HIP call (DUST_EINVAL, nothing enqueued): at most 256
 * grids, and at most about 5.1e5 16-cell tiles over all grids (the exact
 * figure is in the error text).  The array holds only what each call writes
 * before its kernel reads it (no counter or partial result carries over), so
 * nothing needs clearing between calls.  All calls on one device share the
 * array: calls ordered on one stream are safe, calls that may overlap (other
 * streams, other host threads) race on it.  Not capturable into a HIP graph
 * (the work list is copied from pageable host memory). */
dust_status dust_batch_run_noalloc(dust_plan* const* plans, int32_t n_grids,
                                   const int64_t* n_cells,
                                   const float* const* J, const int64_t* ldj,
                                   const float* const* m_dust,
                                   float* const* T, const int64_t* ldt,
                                   float* const* L, const int64_t* ldl,
                                   dust_counters* counters, void* stream);

/* --- Thermally fluctuating grains ----------------------------------------
 * Grains too small to hold the equilibrium temperature of Eq. 7 are heated
 * in spikes by single photons and cool in between (Section 2; Section 6
 * names the calculation and the transition-matrix method it takes).  For
 * each cell and grain the library computes the steady-state probability of
 * each of the grain's enthalpy levels, and the emission averaged over it:
 *
 *   levels    E_0 = 0 < E_1 < ... < E_{M-1} (J) at temperatures
 *             T_0 = 0 < T_1 < ... (K), per grain (they follow from the grain's
 *             heat capacity, which the caller supplies this way);
 *   heating   photons of wavelength bin l (energy h c / lam_l, rate
 *             J_l C_l dlam_l / (h c / lam_l)) lift the grain from level i to
 *             E_i + h c / lam_l, shared between the two levels around it so
 *             that the mean energy gained is the photon's (above the top
 *             level: to the top level);
 *   cooling   from level j > 0 to j - 1 at the rate P(T_j) / (E_j - E_{j-1}),
 *             P(T) the grain power of Eq. 7;
 *   P[c,s,j]  the steady state of those transitions, normalised to sum 1
 *             (the flux balance across each level boundary, solved level by
 *             level upwards in FP64);
 *   L[c,l]    m[c] sum_s w_s C[s,l] sum_j P[c,s,j] B(lam_l, T_sj) (Eq. 10
 *             averaged over the distribution).
 * The common factor 4 pi of heating and cooling is dropped, as in Eq. 7. */
typedef struct {
    int32_t n_levels;     /* M, in [2, 256] */
    const double* T;      /* [S][M] level temperatures (K): T[s][0] = 0, then
                             strictly increasing, finite */
    const double* E;      /* [S][M] level enthalpies (J): E[s][0] = 0, then
                             strictly increasing, finite */
} dust_levels;

/* Opaque, library-owned plan of a grid's fluctuating grains. */
typedef struct dust_fluct_plan dust_fluct_plan;

/* Build the plan on the current device: upload the grid and the levels
 * (host float64, read during the call only) and derive, on the device, the
 * photon-rate weights, the cooling rates, the photon-count table of every
 * level pair and the emission table; wait for them.  Allocates device
 * memory.  DUST_EINVAL for a bad grid or levels, or when a level above the
 * ground level radiates no power in FP64 (its temperature is too low for the
 * wavelength grid). */
dust_status dust_fluct_plan_create(const dust_grid_desc* grid, const dust_levels* levels,
                                   dust_fluct_plan** out);

/* Free a plan (waits for the device).  NULL is accepted. */
dust_status dust_fluct_plan_destroy(dust_fluct_plan* plan);

/* The level distributions: P[c*ldp + s*M + j] (float32, ldp >= S*M) from
 * J[c*ldj + l].  A cell whose J holds a negative or non-finite value gets
 * NaN for every level of every grain (counted in n_nonfinite per pair); a
 * cell without radiation stays in the ground level.  Pairs that put more
 * than 1e-6 of their probability on the top level (the levels end too low
 * for the field) are counted in n_out_of_table.  counters may be NULL. */
dust_status dust_fluct_solve_P(dust_fluct_plan* plan, int64_t n_cells,
                               const float* J, int64_t ldj, float* P, int64_t ldp,
                               dust_counters* counters, void* stream);

/* The emission averaged over the distributions, L[c*ldl + l] (float32);
 * m_dust may be NULL (unit mass).  accumulate nonzero adds to L instead of
 * overwriting it (e.g. onto the equilibrium grains' SED of dust_run_fused). */
dust_status dust_fluct_emit_sed(dust_fluct_plan* plan, int64_t n_cells,
                                const float* P, int64_t ldp, const float* m_dust,
                                float* L, int64_t ldl, int32_t accumulate, void* stream);

/* Text of the last error on the calling thread ("" if none). */
const char* dust_last_error(void);

/* Library version string. */
const char* dust_version(void);

#ifdef __cplusplus
}
#endif
#endif
