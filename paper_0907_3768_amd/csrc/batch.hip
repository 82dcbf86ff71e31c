// Many independent grids in one launch.
//
// A batch binds (plan, buffers) per grid and a work list of (grid, cell tile)
// items, heaviest tiles first (cost of a tile ~ NL x S of its grid).  Two
// launch forms run the fused absorb -> solve -> emit body on each item:
//  * persistent: a fixed number of workgroups per CU; each takes the next run
//    of items from a device counter and repeats until the list is exhausted
//    (every counter read hands out at least one item, so every workgroup
//    reaches the exit test after at most items + 1 reads and the grid always
//    drains);
//  * one workgroup per item, in list order (the hardware dispatcher is the
//    queue).
//
// The form, the cells per tile and the grain tiles per heating pass are
// chosen by timing candidates on the bound buffers (autotuner); the chosen
// launch (with the counter reset, and optionally every plan's refresh) is
// recorded once into a HIP graph and replayed by dust_batch_launch.
// dust_batch_run is the one-shot form: it builds the same work list, copies
// it to a stream-ordered device allocation and launches once.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "fused_body.h"

// Work-list storage of dust_batch_run_noalloc: one array per device, reserved
// when the library is loaded and held until the process ends.  Host code
// never uses the symbol as an address (on the host it is only a stand-in):
// scratch_ptr() asks the runtime for the current device's copy once and keeps
// it, and every copy and kernel argument uses that pointer.
static constexpr size_t SCRATCH_BYTES = (size_t)4 << 20;
static __device__ __align__(256) char scratch[SCRATCH_BYTES];

namespace dust {
namespace {

struct GridArgs {
    PlanView v;
    int64_t C;
    const float* J;
    int64_t ldj;
    const float* m;
    float* T;
    int64_t ldt;
    float* L;
    int64_t ldl;
};

// J chunk width of the batched kernels: the tile's LDS is sized for the
// batch's largest grid, so the narrower chunk keeps more workgroups resident.
constexpr int BATCH_KC = 64;

// The counter is cleared by a kernel (not a memset) so that the graph holds
// only kernel nodes.
__global__ void reset_counter_kernel(unsigned int* counter) {
    if (threadIdx.x == 0 && blockIdx.x == 0) counter[0] = 0u;
}

// Work fetch of the persistent kernel: guided self-scheduling.  A fetch takes
// a run of up to MAX_RUN consecutive items (they cost about the same: the list
// is ordered by cost), a share of what is left so the last runs are single
// items.  Measured on 64 uneven grids at six workgroups per CU: runs of one
// item 11.3-11.6 ms, four 9.8-10.0 ms, sixteen 10.2-10.8 ms (longer runs put
// the resident workgroups on more grids at once, and more plan tables in L2).
constexpr int MAX_RUN = 4;

// Resident waves per SIMD as for the one-workgroup-per-item kernel below:
// without the hint the compiler gives the loop's body more registers, and
// fewer waves per SIMD leave the emission's latencies exposed.
template <int TC, int NTW>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(NTW <= 2 ? 6 : 5, 8))) void batch_kernel(
    const GridArgs* __restrict__ grids, const int2* __restrict__ items, int n_items,
    unsigned int* counter, dust_counters* cnt) {
    // The dynamic tile follows the static words; both 16-byte aligned, so the
    // tile's 16-byte LDS accesses stay aligned (with a lone 4-byte static
    // word in front of it every one of them was misaligned: about 3x slower).
    extern __shared__ __align__(16) float sTile[];  // fused_lds_bytes(TC, Sp max, Stage<BATCH_KC>::BYTES)
    __shared__ __align__(16) int sRun[4];            // first item, items in the run
    const int nb = (int)gridDim.x;
    for (;;) {
        if (threadIdx.x == 0) {
            // the count read here only sizes the run; the atomic decides it
            const unsigned seen = __hip_atomic_load(counter, __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_AGENT);
            const int left = n_items - (int)min(seen, (unsigned)n_items);
            const int take = max(1, min(MAX_RUN, left / (2 * nb)));
            sRun[0] = (int)atomicAdd(counter, (unsigned)take);
            sRun[1] = take;
        }
        __syncthreads();
        // Uniform across the block: keep the items and the grid descriptor in
        // scalar registers (scalar loads) rather than in every lane.
        const int first = __builtin_amdgcn_readfirstlane(sRun[0]);
        if (first >= n_items) break;
        const int last = min(first + __builtin_amdgcn_readfirstlane(sRun[1]), n_items);
        for (int it = first; it < last; ++it) {
            const int gx = __builtin_amdgcn_readfirstlane(items[it].x);
            const int ty = __builtin_amdgcn_readfirstlane(items[it].y);
            const GridArgs& g = grids[gx];
            fused_tile<DUST_MIXED, TC, NTW, true, BATCH_KC>(g.v, (int64_t)ty * TC, g.C, g.J, g.ldj,
                                                            g.m, g.T, g.ldt, g.L, g.ldl, cnt, sTile);
        }
        // fused_tile ends with a barrier (after every thread read sRun), so
        // sRun may be overwritten now.
    }
}

// One workgroup per work item (the hardware dispatcher hands items out in
// list order, heaviest first).  Same tile body as the persistent kernel but
// without its loop, which on gfx950 costs the persistent form a lot of
// registers (values the compiler keeps live across items).  Resident waves
// per SIMD as for the single-grid fused kernel: six for up to 128 grains,
// five above.
template <int TC, int NTW>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(NTW <= 2 ? 6 : 5, 8))) void batch_item_kernel(
    const GridArgs* __restrict__ grids,
                                                         const int2* __restrict__ items,
                                                         int n_items, unsigned int* counter,
                                                         dust_counters* cnt) {
    extern __shared__ float sTile[];  // fused_lds_bytes(TC, Sp max, Stage<BATCH_KC>::BYTES)
    const int it = blockIdx.x;
    if (it >= n_items) return;
    const int gx = __builtin_amdgcn_readfirstlane(items[it].x);
    const int ty = __builtin_amdgcn_readfirstlane(items[it].y);
    const GridArgs& g = grids[gx];
    fused_tile<DUST_MIXED, TC, NTW, true, BATCH_KC>(g.v, (int64_t)ty * TC, g.C, g.J, g.ldj, g.m, g.T, g.ldt, g.L,
                                    g.ldl, cnt, sTile);
    (void)counter;
}

struct Candidate {
    int tc;        // cells per tile
    int per_cu;    // resident workgroups per CU of the persistent kernel;
                   // 0 = one workgroup per item
    int ntw;       // grain tiles per wave in one pass of the heating
};

using KernelFn = void (*)(const GridArgs*, const int2*, int, unsigned int*, dust_counters*);

template <int TC>
KernelFn pick_kernel(int ntw) {
    if (ntw <= 1) return batch_kernel<TC, 1>;
    if (ntw <= 2) return batch_kernel<TC, 2>;
    return batch_kernel<TC, 4>;  // larger grain sets take several passes
}

template <int TC>
KernelFn pick_item_kernel(int ntw) {
    if (ntw <= 1) return batch_item_kernel<TC, 1>;
    if (ntw <= 2) return batch_item_kernel<TC, 2>;
    return batch_item_kernel<TC, 4>;
}

KernelFn kernel_for(int tc, int ntw, bool persistent) {
    if (persistent) return tc == 32 ? pick_kernel<32>(ntw) : pick_kernel<16>(ntw);
    return tc == 32 ? pick_item_kernel<32>(ntw) : pick_item_kernel<16>(ntw);
}

// Autotuner cache: the best candidate per (max-S bucket, mean-NL bucket,
// tile-count bucket), shared by every batch of the process.
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int>, Candidate> g_tune_cache;

// Default launch: one workgroup per 16-cell item, as many grain tiles per
// wave as the largest grid needs (at most two; more take passes).
Candidate default_candidate(int sp_max) {
    const int need = (sp_max / 16 + 3) / 4;
    return Candidate{16, 0, need < 2 ? need : 2};
}

// Whether a candidate fits the batch: its LDS (sized for the largest grid)
// in one workgroup and, times its resident workgroups, in one CU; and no more
// grain tiles per wave than the largest grid needs.
bool candidate_fits(const Candidate& c, int sp_max, int max_lds) {
    // (+ the persistent kernel's 16 static bytes)
    const size_t lds = fused_lds_bytes(c.tc, sp_max, Stage<BATCH_KC>::BYTES) + (c.per_cu > 0 ? 16 : 0);
    if (c.ntw > 1 && c.ntw / 2 >= (sp_max / 16 + 3) / 4) return false;
    return lds <= (size_t)max_lds && lds * std::max(c.per_cu, 1) <= 160u * 1024u;
}

// Candidate named by the environment variable DUST_BATCH_CANDIDATE as
// "tc,ntw,per_cu" (a test hook that pins the launch form); returns 0 when
// the variable is unset, 1 with *c set, -1 when it is malformed or does not
// name a candidate form.
int forced_candidate(Candidate* c) {
    const char* s = getenv("DUST_BATCH_CANDIDATE");
    if (!s || !*s) return 0;
    int tc = 0, ntw = 0, per_cu = -1;
    if (sscanf(s, "%d,%d,%d", &tc, &ntw, &per_cu) != 3) return -1;
    if ((tc != 16 && tc != 32) || (ntw != 1 && ntw != 2 && ntw != 4) ||
        (per_cu != 0 && per_cu != 2 && per_cu != 4 && per_cu != 6))
        return -1;
    *c = Candidate{tc, per_cu, ntw};
    return 1;
}

// Host side shared by dust_batch_create and dust_batch_run: checks every
// grid's arguments and fills the per-grid launch arguments, cell counts and
// costs; *sp_max receives the largest padded grain count, *tiles16 the number
// of 16-cell tiles.
dust_status bind_grids(dust_plan* const* plans, int32_t n_grids, const int64_t* n_cells,
                       const float* const* J, const int64_t* ldj, const float* const* m_dust,
                       float* const* T, const int64_t* ldt, float* const* L,
                       const int64_t* ldl, dust_counters* counters, std::vector<GridArgs>* args,
                       std::vector<int64_t>* C, std::vector<double>* cost, int* sp_max,
                       int64_t* tiles16, int* device) {
    if (n_grids < 1) return set_error(DUST_EINVAL, "n_grids must be >= 1");
    if (!plans || !n_cells || !J || !ldj || !m_dust || !T || !ldt || !L || !ldl)
        return set_error(DUST_EINVAL, "a per-grid array is NULL");
    if (counters && ((uintptr_t)counters & 7u))
        return set_error(DUST_EINVAL, "counters must be 8-byte aligned");
    args->assign(n_grids, GridArgs{});
    C->assign(n_grids, 0);
    cost->assign(n_grids, 0.0);
    *sp_max = 16;
    *tiles16 = 0;
    for (int g = 0; g < n_grids; ++g) {
        const dust_plan* p = plans[g];
        if (!p) return set_error(DUST_EINVAL, "plans[" + std::to_string(g) + "] is NULL");
        if (p->opt.mode != DUST_MIXED || p->opt.f32_lookup || p->opt.newton_polish)
            return set_error(DUST_EUNSUPPORTED,
                             "batched launches take DUST_MIXED plans with the FP64 lookup "
                             "(no FP32 lookup, no Newton polish)");
        if (n_cells[g] < 0 || n_cells[g] > ((int64_t)1 << 36))
            return set_error(DUST_EINVAL, "n_cells out of range");
        const int64_t c = n_cells[g];
        if (c > 0) {
            if (!J[g] || !T[g] || !L[g]) return set_error(DUST_EINVAL, "a J/T/L pointer is NULL");
            if (ldj[g] < p->NL || ldt[g] < p->S || ldl[g] < p->NL)
                return set_error(DUST_EINVAL, "a leading dimension is smaller than its row");
            if (((uintptr_t)J[g] | (uintptr_t)T[g] | (uintptr_t)L[g] |
                 (uintptr_t)m_dust[g]) & 3u)
                return set_error(DUST_EINVAL, "buffers must be 4-byte aligned");
        }
        (*args)[g] = GridArgs{p->view, c, J[g], ldj[g], m_dust[g], T[g], ldt[g], L[g], ldl[g]};
        (*C)[g] = c;
        (*cost)[g] = (double)p->NL * p->S;
        *sp_max = std::max(*sp_max, p->Sp);
        *tiles16 += (c + 15) / 16;
    }
    if (*tiles16 > (int64_t)1 << 30) return set_error(DUST_EUNSUPPORTED, "too many tiles");
    hipError_t e;
    if ((e = hipGetDevice(device)) != hipSuccess) return hip_error(e, "hipGetDevice");
    for (int g = 0; g < n_grids; ++g)
        if (plans[g]->device != *device)
            return set_error(DUST_EINVAL, "every plan must belong to the current device");
    return DUST_OK;
}

}  // namespace
}  // namespace dust

struct dust_batch {
    int device;
    int n_grids;
    int sp_max;
    dust::Candidate cand;
    int64_t n_items_16, n_items_32;
    dust::GridArgs* d_grids;
    int2* d_items16;
    int2* d_items32;
    unsigned int* d_counter;
    dust_counters* counters;
    int n_cu;
    // batched refresh of the distinct plans (DUST_BATCH_REFRESH_PLANS)
    dust::RefreshJob* d_jobs;
    int* d_starts;  // [4][n_jobs]
    int n_jobs;
    int refresh_blocks[4];
    hipGraph_t graph;
    hipGraphExec_t exec;
};

namespace dust {
namespace {

hipError_t enqueue(const dust_batch* b, const Candidate& c, hipStream_t st) {
    const int2* items = c.tc == 32 ? b->d_items32 : b->d_items16;
    const int n_items = (int)(c.tc == 32 ? b->n_items_32 : b->n_items_16);
    const bool persistent = c.per_cu > 0;
    if (persistent) {
        hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(64), 0, st, b->d_counter);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const int blocks = persistent ? std::max(1, std::min(n_items, b->n_cu * c.per_cu))
                                  : std::max(1, n_items);
    const size_t lds = fused_lds_bytes(c.tc, b->sp_max, Stage<BATCH_KC>::BYTES);
    hipLaunchKernelGGL(kernel_for(c.tc, c.ntw, persistent), dim3(blocks), dim3(256), lds, st,
                       (const GridArgs*)b->d_grids, items, n_items, b->d_counter, b->counters);
    return hipGetLastError();
}

void free_batch(dust_batch* b) {
    if (!b) return;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->d_grids) (void)hipFree(b->d_grids);
    if (b->d_items16) (void)hipFree(b->d_items16);
    if (b->d_items32) (void)hipFree(b->d_items32);
    if (b->d_counter) (void)hipFree(b->d_counter);
    if (b->d_jobs) (void)hipFree(b->d_jobs);
    if (b->d_starts) (void)hipFree(b->d_starts);
    delete b;
}

std::vector<int2> build_items(const std::vector<int64_t>& C, const std::vector<double>& cost,
                              int tc) {
    std::vector<int> order(C.size());
    for (size_t g = 0; g < C.size(); ++g) order[g] = (int)g;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return cost[a] > cost[b]; });
    std::vector<int2> items;
    for (int g : order) {
        const int64_t tiles = (C[g] + tc - 1) / tc;
        for (int64_t t = 0; t < tiles; ++t) items.push_back(make_int2(g, (int)t));
    }
    return items;
}

// (the static work-list array `scratch` is declared at file scope above)
constexpr int SCRATCH_MAX_GRIDS = 256;

// Bytes of a work list: the grids' launch arguments (padded to 256 bytes),
// then the (grid, tile) items.
size_t work_list_args_bytes(int n_grids) {
    return (sizeof(GridArgs) * (size_t)n_grids + 255) / 256 * 256;
}
int64_t scratch_max_items() {
    return (int64_t)((SCRATCH_BYTES - work_list_args_bytes(SCRATCH_MAX_GRIDS)) / sizeof(int2));
}

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES];

hipError_t scratch_ptr(int dev, void** out) {
    if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

// Copies the work list (host staging) to `d` on `sm` and launches the
// per-item kernel of the default form over it.
hipError_t launch_work_list(const std::vector<GridArgs>& args, const std::vector<int2>& items,
                            int sp_max, const Candidate& c, void* d, dust_counters* counters,
                            hipStream_t sm) {
    const size_t args_bytes = work_list_args_bytes((int)args.size());
    const size_t bytes = args_bytes + sizeof(int2) * items.size();
    std::vector<char> host(bytes);
    memcpy(host.data(), args.data(), sizeof(GridArgs) * args.size());
    memcpy(host.data() + args_bytes, items.data(), sizeof(int2) * items.size());
    // from pageable memory: the call returns once `host` has been staged
    hipError_t e = hipMemcpyAsync(d, host.data(), bytes, hipMemcpyHostToDevice, sm);
    if (e != hipSuccess) return e;
    const size_t lds = fused_lds_bytes(c.tc, sp_max, Stage<BATCH_KC>::BYTES);
    hipLaunchKernelGGL(kernel_for(c.tc, c.ntw, false), dim3((unsigned)items.size()), dim3(256),
                       lds, sm, (const GridArgs*)d,
                       reinterpret_cast<const int2*>((char*)d + args_bytes), (int)items.size(),
                       nullptr, counters);
    return hipGetLastError();
}

int max_lds_bytes(int dev) {
    int max_lds = 65536;
    (void)hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    return max_lds;
}

}  // namespace
}  // namespace dust

using namespace dust;

extern "C" {

dust_status dust_batch_create(dust_plan* const* plans, int32_t n_grids, const int64_t* n_cells,
                              const float* const* J, const int64_t* ldj,
                              const float* const* m_dust, float* const* T, const int64_t* ldt,
                              float* const* L, const int64_t* ldl, dust_counters* counters,
                              int32_t flags, dust_batch** out) {
    clear_error();
    const bool autotune = (flags & DUST_BATCH_AUTOTUNE) != 0;
    const bool refresh = (flags & DUST_BATCH_REFRESH_PLANS) != 0;
    if (!out) return set_error(DUST_EINVAL, "out is NULL");
    *out = nullptr;
    if (flags & ~(DUST_BATCH_AUTOTUNE | DUST_BATCH_REFRESH_PLANS))
        return set_error(DUST_EINVAL, "unknown batch flags");
    std::vector<GridArgs> args;
    std::vector<int64_t> C;
    std::vector<double> cost;
    int sp_max = 16, dev = 0;
    int64_t total16 = 0;
    dust_status st = bind_grids(plans, n_grids, n_cells, J, ldj, m_dust, T, ldt, L, ldl, counters,
                                &args, &C, &cost, &sp_max, &total16, &dev);
    if (st != DUST_OK) return st;
    const int max_lds = max_lds_bytes(dev);
    Candidate forced{};
    const int force = forced_candidate(&forced);
    if (force < 0)
        return set_error(DUST_EINVAL,
                         "DUST_BATCH_CANDIDATE must be \"tc,ntw,per_cu\" with tc 16 or 32, "
                         "ntw 1, 2 or 4, per_cu 0, 2, 4 or 6");
    if (force > 0 && !candidate_fits(forced, sp_max, max_lds))
        return set_error(DUST_EUNSUPPORTED, "DUST_BATCH_CANDIDATE does not fit this batch");

    hipError_t e;
    hipDeviceProp_t prop;
    if ((e = hipGetDeviceProperties(&prop, dev)) != hipSuccess)
        return hip_error(e, "hipGetDeviceProperties");

    dust_batch* b = new dust_batch();
    b->device = dev;
    b->n_grids = n_grids;
    b->sp_max = sp_max;
    b->n_cu = prop.multiProcessorCount;
    b->counters = counters;
    std::vector<int2> it16 = build_items(C, cost, 16), it32 = build_items(C, cost, 32);
    b->n_items_16 = (int64_t)it16.size();
    b->n_items_32 = (int64_t)it32.size();

    if ((e = hipMalloc(&b->d_grids, sizeof(GridArgs) * n_grids)) != hipSuccess ||
        (e = hipMalloc(&b->d_items16, sizeof(int2) * std::max<size_t>(1, it16.size()))) != hipSuccess ||
        (e = hipMalloc(&b->d_items32, sizeof(int2) * std::max<size_t>(1, it32.size()))) != hipSuccess ||
        (e = hipMalloc(&b->d_counter, 256)) != hipSuccess) {
        free_batch(b);
        return hip_error(e, "hipMalloc (batch)");
    }
    if ((e = hipMemcpy(b->d_grids, args.data(), sizeof(GridArgs) * n_grids, hipMemcpyHostToDevice)) != hipSuccess ||
        (it16.size() && (e = hipMemcpy(b->d_items16, it16.data(), sizeof(int2) * it16.size(), hipMemcpyHostToDevice)) != hipSuccess) ||
        (it32.size() && (e = hipMemcpy(b->d_items32, it32.data(), sizeof(int2) * it32.size(), hipMemcpyHostToDevice)) != hipSuccess)) {
        free_batch(b);
        return hip_error(e, "hipMemcpy (batch)");
    }

    // Candidate launches: 16- or 32-cell tiles (32 needs twice the LDS per
    // workgroup; a workgroup may hold at most 64 KiB and a CU 160 KiB), one
    // or more grain tiles per wave, one workgroup per item or a work queue
    // with 2, 4 or 6 resident workgroups per CU.
    std::vector<Candidate> cands;
    for (int tc : {16, 32})
        for (int ntw : {1, 2, 4})
            for (int per_cu : {0, 2, 4, 6}) {
                const Candidate c{tc, per_cu, ntw};
                if (candidate_fits(c, sp_max, max_lds)) cands.push_back(c);
            }
    Candidate best = default_candidate(sp_max);
    const bool verbose = getenv("DUST_LOG") != nullptr;
    if (force > 0) {
        best = forced;
    } else if (autotune && !cands.empty()) {
        double mean_nl = 0.0;
        for (int g = 0; g < n_grids; ++g) mean_nl += plans[g]->NL;
        mean_nl /= n_grids;
        int tiles_b = 0;
        for (int64_t t = total16; t > 1; t >>= 2) ++tiles_b;
        const auto key = std::make_tuple(sp_max / 64, (int)(mean_nl / 128), tiles_b);
        bool hit = false;
        {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            auto f = g_tune_cache.find(key);
            if (f != g_tune_cache.end()) { best = f->second; hit = true; }
        }
        if (!hit) {
            hipStream_t st;
            hipEvent_t e0, e1;
            if ((e = hipStreamCreate(&st)) != hipSuccess) { free_batch(b); return hip_error(e, "hipStreamCreate"); }
            (void)hipEventCreate(&e0);
            (void)hipEventCreate(&e1);
            float best_ms = 1e30f;
            for (const Candidate& c : cands) {
                float ms = 0.f, total = 0.f;
                bool ok = enqueue(b, c, st) == hipSuccess;  // warm-up
                for (int r = 0; ok && r < 2; ++r) {
                    (void)hipEventRecord(e0, st);
                    ok = enqueue(b, c, st) == hipSuccess;
                    (void)hipEventRecord(e1, st);
                    ok = ok && hipEventSynchronize(e1) == hipSuccess;
                    (void)hipEventElapsedTime(&ms, e0, e1);
                    total += ms;
                }
                if (verbose)
                    fprintf(stderr, "dust batch autotune: tc=%d ntw=%d per_cu=%d  %.3f ms%s\n",
                            c.tc, c.ntw, c.per_cu, total / 2, ok ? "" : " (failed)");
                if (ok && total < best_ms) { best_ms = total; best = c; }
            }
            (void)hipStreamSynchronize(st);
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            (void)hipStreamDestroy(st);
            std::lock_guard<std::mutex> lk(g_tune_mu);
            g_tune_cache[key] = best;
        }
    }
    b->cand = best;

    // The plans' refreshes as three batched launches (one per stage, every
    // distinct plan in each), then the chosen batched kernel, recorded once.
    if (refresh) {
        std::vector<const dust_plan*> uniq;
        for (int g = 0; g < n_grids; ++g)
            if (std::find(uniq.begin(), uniq.end(), plans[g]) == uniq.end()) uniq.push_back(plans[g]);
        const int nj = (int)uniq.size();
        std::vector<RefreshJob> jobs(nj);
        std::vector<int> starts(4 * (size_t)nj);
        int64_t total[4] = {0, 0, 0, 0};
        for (int k = 0; k < nj; ++k) {
            make_refresh_job(uniq[k], &jobs[k]);
            for (int st = 0; st < 4; ++st) {
                starts[(size_t)st * nj + k] = (int)total[st];
                total[st] += (int64_t)jobs[k].gx[st] * jobs[k].gy[st];
            }
        }
        for (int st = 0; st < 4; ++st) {
            if (total[st] > INT32_MAX) { free_batch(b); return set_error(DUST_EUNSUPPORTED, "refresh grid too large"); }
            b->refresh_blocks[st] = (int)total[st];
        }
        b->n_jobs = nj;
        if ((e = hipMalloc(&b->d_jobs, sizeof(RefreshJob) * nj)) != hipSuccess ||
            (e = hipMalloc(&b->d_starts, sizeof(int) * starts.size())) != hipSuccess ||
            (e = hipMemcpy(b->d_jobs, jobs.data(), sizeof(RefreshJob) * nj, hipMemcpyHostToDevice)) != hipSuccess ||
            (e = hipMemcpy(b->d_starts, starts.data(), sizeof(int) * starts.size(), hipMemcpyHostToDevice)) != hipSuccess) {
            free_batch(b);
            return hip_error(e, "batched refresh tables");
        }
    }
    hipStream_t cs;
    if ((e = hipStreamCreate(&cs)) != hipSuccess) { free_batch(b); return hip_error(e, "hipStreamCreate"); }
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        hipError_t le = hipSuccess;
        if (refresh) {
            const int* starts[4];
            for (int st = 0; st < 4; ++st) starts[st] = b->d_starts + (size_t)st * b->n_jobs;
            le = launch_prepare_batched(b->d_jobs, starts, b->n_jobs, b->refresh_blocks, cs);
        }
        if (le == hipSuccess) le = enqueue(b, best, cs);
        e = hipStreamEndCapture(cs, &b->graph);
        if (e == hipSuccess && le != hipSuccess) e = le;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    (void)hipStreamDestroy(cs);
    if (e != hipSuccess) { free_batch(b); return hip_error(e, "graph capture"); }
    if ((e = hipDeviceSynchronize()) != hipSuccess) { free_batch(b); return hip_error(e, "hipDeviceSynchronize"); }
    *out = b;
    return DUST_OK;
}

dust_status dust_batch_launch(dust_batch* b, void* stream) {
    clear_error();
    if (!b) return set_error(DUST_EINVAL, "batch is NULL");
    hipError_t e = hipGraphLaunch(b->exec, (hipStream_t)stream);
    return e == hipSuccess ? DUST_OK : hip_error(e, "hipGraphLaunch");
}

dust_status dust_batch_info(const dust_batch* b, int32_t* cells_per_tile, int64_t* n_items) {
    clear_error();
    if (!b) return set_error(DUST_EINVAL, "batch is NULL");
    if (cells_per_tile) *cells_per_tile = b->cand.tc;
    if (n_items) *n_items = b->cand.tc == 32 ? b->n_items_32 : b->n_items_16;
    return DUST_OK;
}

dust_status dust_batch_form(const dust_batch* b, int32_t* cells_per_tile,
                            int32_t* tiles_per_wave, int32_t* per_cu) {
    clear_error();
    if (!b) return set_error(DUST_EINVAL, "batch is NULL");
    if (cells_per_tile) *cells_per_tile = b->cand.tc;
    if (tiles_per_wave) *tiles_per_wave = b->cand.ntw;
    if (per_cu) *per_cu = b->cand.per_cu;
    return DUST_OK;
}

dust_status dust_batch_destroy(dust_batch* b) {
    clear_error();
    if (!b) return DUST_OK;
    hipError_t e = hipDeviceSynchronize();
    free_batch(b);
    return e == hipSuccess ? DUST_OK : hip_error(e, "hipDeviceSynchronize");
}

dust_status dust_batch_run(dust_plan* const* plans, int32_t n_grids, const int64_t* n_cells,
                           const float* const* J, const int64_t* ldj,
                           const float* const* m_dust, float* const* T, const int64_t* ldt,
                           float* const* L, const int64_t* ldl, dust_counters* counters,
                           void* stream) {
    clear_error();
    std::vector<GridArgs> args;
    std::vector<int64_t> C;
    std::vector<double> cost;
    int sp_max = 16, dev = 0;
    int64_t total16 = 0;
    dust_status st = bind_grids(plans, n_grids, n_cells, J, ldj, m_dust, T, ldt, L, ldl, counters,
                                &args, &C, &cost, &sp_max, &total16, &dev);
    if (st != DUST_OK) return st;
    if (total16 == 0) return DUST_OK;
    const Candidate c = default_candidate(sp_max);
    const std::vector<int2> items = build_items(C, cost, c.tc);
    const hipStream_t sm = (hipStream_t)stream;
    void* d = nullptr;
    hipError_t e = hipMallocAsync(&d, work_list_args_bytes(n_grids) + sizeof(int2) * items.size(), sm);
    if (e != hipSuccess) return hip_error(e, "hipMallocAsync (batch work list)");
    e = launch_work_list(args, items, sp_max, c, d, counters, sm);
    const hipError_t ef = hipFreeAsync(d, sm);
    if (e != hipSuccess) return hip_error(e, "batch run");
    return ef == hipSuccess ? DUST_OK : hip_error(ef, "hipFreeAsync (batch work list)");
}

dust_status dust_batch_run_noalloc(dust_plan* const* plans, int32_t n_grids,
                                   const int64_t* n_cells, const float* const* J,
                                   const int64_t* ldj, const float* const* m_dust,
                                   float* const* T, const int64_t* ldt, float* const* L,
                                   const int64_t* ldl, dust_counters* counters, void* stream) {
    clear_error();
    // the limits of the static work-list array, before any HIP call
    if (n_grids > SCRATCH_MAX_GRIDS)
        return set_error(DUST_EINVAL, "dust_batch_run_noalloc takes at most " +
                                          std::to_string(SCRATCH_MAX_GRIDS) + " grids");
    if (n_grids >= 1 && n_cells) {
        int64_t tiles = 0;
        for (int g = 0; g < n_grids; ++g)
            if (n_cells[g] > 0) tiles += (std::min<int64_t>(n_cells[g], (int64_t)1 << 36) + 15) / 16;
        if (tiles > scratch_max_items())
            return set_error(DUST_EINVAL, "dust_batch_run_noalloc takes at most " +
                                              std::to_string(scratch_max_items()) +
                                              " 16-cell tiles in all");
    }
    std::vector<GridArgs> args;
    std::vector<int64_t> C;
    std::vector<double> cost;
    int sp_max = 16, dev = 0;
    int64_t total16 = 0;
    dust_status st = bind_grids(plans, n_grids, n_cells, J, ldj, m_dust, T, ldt, L, ldl, counters,
                                &args, &C, &cost, &sp_max, &total16, &dev);
    if (st != DUST_OK) return st;
    if (total16 == 0) return DUST_OK;
    void* d = nullptr;
    hipError_t e = scratch_ptr(dev, &d);
    if (e != hipSuccess) return hip_error(e, "hipGetSymbolAddress (work-list array)");
    const Candidate c = default_candidate(sp_max);
    e = launch_work_list(args, build_items(C, cost, c.tc), sp_max, c, d, counters,
                         (hipStream_t)stream);
    return e == hipSuccess ? DUST_OK : hip_error(e, "batch run (no allocation)");
}

}  // extern "C"
