// Heating, Eq. 6 (Section 4.2): H[c,s] = sum_l J[c,l] K[s,l], a dense
// contraction over wavelength on the MFMA units.
//
//   DUST_PLAIN_FP32: a workgroup computes the heating of 16 cells for every
//                    grain with the LDS-staged MFMA routine of the fused
//                    kernel (fused_absorb) on v_mfma_f32_16x16x4_f32 (exact
//                    FP32 products), then writes the 16 x S block of H with
//                    coalesced stores, undoing the per-grain power of two.
//   DUST_MIXED, DUST_TABLE_LINEAR:
//                    v_mfma_f32_16x16x32_bf16 on hi+lo splits,
//                    J_hi K_hi + J_hi K_lo + J_lo K_hi, FP32 accumulation:
//                    a blocked product of 256 cells x up to 256 grains per
//                    workgroup with J and the weight fragments staged in LDS
//                    (absorb_dl_kernel: loaded straight into LDS, for J rows
//                    aligned to 16 bytes; absorb_gemm_kernel: through
//                    registers), or, on a device that cannot give one
//                    workgroup its 144 KB of LDS, 64 cells per workgroup
//                    with the fragments read from L2 (absorb_mb_kernel).
#include "fused_body.h"

namespace dust {
namespace {

template <int MODE, int NTW>
__global__ __launch_bounds__(256) void absorb_kernel(PlanView v, int64_t C,
                                                     const float* __restrict__ J, int64_t ldj,
                                                     float* __restrict__ H, int64_t ldh) {
    extern __shared__ float lds[];  // sH [16][Sp], then the J staging buffers
    float* sH = lds;
    char* sStage = reinterpret_cast<char*>(lds + 16 * v.Sp);
    const int64_t c0 = (int64_t)blockIdx.x * 16;
    fused_absorb<MODE, NTW>(v, c0, C, J, ldj, sH, sStage);
    __syncthreads();
    for (int i = threadIdx.x; i < 16 * v.Sp; i += 256) {
        const int cc = i / v.Sp, s = i - cc * v.Sp;
        if (s < v.S && c0 + cc < C) H[(c0 + cc) * ldh + s] = sH[i] * v.hinv[s];
    }
}

// ---------------------------------------------------------------------------
// bf16 hi+lo heating of 16 MB cells per workgroup of NW waves (MB 16-cell
// MFMA row blocks): each wave loads the weight fragments of its grain tiles
// (tiles wave, wave + NW, ...) once per k-step and applies them to all MB row
// blocks, 1 / MB of the fragment traffic of one block per workgroup.  Eight
// waves for more than four grain tiles: fewer tiles, and registers, per wave.  J goes through LDS in chunks of 16 MB
// cells x 64 wavelengths as bf16 hi and lo planes (rows KC + 8 long, 4 banks
// apart), double-buffered, one barrier per chunk; the accumulators go
// straight to H.  Each product runs over every accumulator before the next
// (consecutive MFMAs are independent), and the k-steps and the three products
// of any one accumulator run in the order of the fused kernel's heating, so
// H is the same bit for bit.
// ---------------------------------------------------------------------------
constexpr int A_KC = 64;
constexpr int A_ROW = A_KC + 8;

// Eight-wave workgroups with up to two grain tiles per wave ask for four
// resident waves per SIMD (two workgroups per CU; a few spilled registers):
// 8.9 ms against 13.1 ms at two waves on 4194304 cells x 1000 x 240.
template <int NTW, int MB, int NW>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(NW == 8 && NTW <= 2 ? 4 : 1, 8))) void absorb_mb_kernel(PlanView v, int64_t C,
                                                            const float* __restrict__ J,
                                                            int64_t ldj, float* __restrict__ H,
                                                            int64_t ldh) {
    constexpr int CELLS = 16 * MB;
    constexpr int NT = 64 * NW;              // threads
    constexpr int NX = CELLS * A_KC / NT;    // J values per thread and chunk
    constexpr int PASSES = NX / 4;           // loader rows per thread
    constexpr int RSTEP = NT / 16;           // rows between a thread's loader rows
    static_assert(NX % 4 == 0 && PASSES * RSTEP == CELLS, "loader covers the chunk");
    __shared__ __bf16 sJ[2][2][CELLS][A_ROW];  // [buffer][hi, lo][cell][wavelength]
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int row = lane & 15, kq = lane >> 4;
    const int tiles = v.Sp / 16;
    const int nsteps = v.NLp / 32;
    const int nchunks = (nsteps + 1) / 2;  // two k-steps per chunk
    const int64_t c0 = (int64_t)blockIdx.x * CELLS;
    // loader: thread t takes rows (t >> 4) + RSTEP p and column pairs 2 (t mod 16) + 32 i
    const int lrow = tid >> 4, lcol = (tid & 15) * 2;
    auto load_j = [&](int k0, float (&x)[NX]) {
#pragma unroll
        for (int p = 0; p < PASSES; ++p) {
            const int64_t c = c0 + lrow + RSTEP * p;
            const bool ok = c < C;
            const float* jl = J + (ok ? c : 0) * ldj;
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const int k = k0 + lcol + 32 * i;
                x[4 * p + 2 * i] = (ok && k < v.NL) ? jl[k] : 0.0f;
                x[4 * p + 2 * i + 1] = (ok && k + 1 < v.NL) ? jl[k + 1] : 0.0f;
            }
        }
    };
    auto store_j = [&](int buf, const float (&x)[NX]) {
        typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
#pragma unroll
        for (int p = 0; p < PASSES; ++p) {
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const float x0 = x[4 * p + 2 * i], x1 = x[4 * p + 2 * i + 1];
                const __bf16 h0 = (__bf16)x0, h1 = (__bf16)x1;
                const bf16x2 hi = {h0, h1};
                const bf16x2 lo = {(__bf16)(x0 - (float)h0), (__bf16)(x1 - (float)h1)};
                *reinterpret_cast<bf16x2*>(&sJ[buf][0][lrow + RSTEP * p][lcol + 32 * i]) = hi;
                *reinterpret_cast<bf16x2*>(&sJ[buf][1][lrow + RSTEP * p][lcol + 32 * i]) = lo;
            }
        }
    };
    for (int tg = 0; tg < tiles; tg += NW * NTW) {
        f32x4 acc[NTW][MB];
#pragma unroll
        for (int t = 0; t < NTW; ++t)
#pragma unroll
            for (int mb = 0; mb < MB; ++mb) acc[t][mb] = f32x4{0.f, 0.f, 0.f, 0.f};
        float x[NX];
        load_j(0, x);
        store_j(0, x);
        __syncthreads();
        for (int ch = 0; ch < nchunks; ++ch) {
            const int buf = ch & 1;
            if (ch + 1 < nchunks) load_j((ch + 1) * A_KC, x);  // next chunk in flight
#pragma unroll 1
            for (int ks = 0; ks < 2; ++ks) {
                const int step = ch * 2 + ks;
                if (step >= nsteps) break;  // uniform
                bf16x8 khi[NTW], klo[NTW];
#pragma unroll
                for (int t = 0; t < NTW; ++t) {
                    const int tile = tg + wave + NW * t;
                    if (tile < tiles) {
                        const int64_t o = (((int64_t)tile * nsteps + step) * 64 + lane) * 8;
                        khi[t] = *reinterpret_cast<const bf16x8*>(v.khi + o);
                        klo[t] = *reinterpret_cast<const bf16x8*>(v.klo + o);
                    }
                }
                bf16x8 ahi[MB], alo[MB];
#pragma unroll
                for (int mb = 0; mb < MB; ++mb) {
                    ahi[mb] = *reinterpret_cast<const bf16x8*>(&sJ[buf][0][16 * mb + row][ks * 32 + kq * 8]);
                    alo[mb] = *reinterpret_cast<const bf16x8*>(&sJ[buf][1][16 * mb + row][ks * 32 + kq * 8]);
                }
#pragma unroll
                for (int pr = 0; pr < 3; ++pr)
#pragma unroll
                    for (int t = 0; t < NTW; ++t) {
                        if (tg + wave + NW * t < tiles) {
#pragma unroll
                            for (int mb = 0; mb < MB; ++mb)
                                acc[t][mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                                    pr == 2 ? alo[mb] : ahi[mb], pr == 1 ? klo[t] : khi[t],
                                    acc[t][mb], 0, 0, 0);
                        }
                    }
            }
            if (ch + 1 < nchunks) store_j(buf ^ 1, x);
            __syncthreads();
        }
        // accumulator element r of lane (row, kq): cell 16 mb + 4 kq + r, grain 16 tile + row
#pragma unroll
        for (int t = 0; t < NTW; ++t) {
            const int tile = tg + wave + NW * t;
            const int s = tile * 16 + row;
            if (tile < tiles && s < v.S) {
                const float hinv = v.hinv[s];
#pragma unroll
                for (int mb = 0; mb < MB; ++mb)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int64_t c = c0 + 16 * mb + 4 * kq + r;
                        if (c < C) H[c * ldh + s] = acc[t][mb][r] * hinv;
                    }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// bf16 hi+lo heating as a blocked matrix product for the large shapes: a
// workgroup of sixteen waves computes 256 cells x up to 16 grain tiles (256
// grains; more grains take further passes, blockIdx.y), the weight
// fragments of all its grain tiles and the J block of its cells staged in
// LDS for one 32-wavelength k-step at a time, double-buffered:
//   A (J): [buffer][hi, lo][cell][32 wavelengths + 8 pad] bf16 (80-byte rows:
//          the 16 rows one MFMA operand read touches fall on distinct banks);
//   B (K): [buffer][tile][hi, lo][lane] 16-byte fragments, copied from the
//          plan's fragment order as they are.
// Sixteen waves, four per SIMD: with eight or more tiles they split into eight
// cell groups of 32 x two grain groups, each holding 2 row blocks x NT/2
// tiles of accumulators (64 registers at 16 tiles, 120 in all), so each
// fragment read from LDS feeds 6 MFMAs; fewer tiles: sixteen cell groups of
// 16.  (Eight waves of 64 cells x 8 tiles, 12 MFMAs per fragment read but two
// waves per SIMD, measured 12-18 % slower: the four waves per SIMD cover the
// LDS and barrier latencies.)  A fragment read from L2 once per workgroup
// serves 256 cells (64 in absorb_mb_kernel).  The next k-step's J
// values and fragments are loaded into registers during the MFMAs of the
// current one and written to the other buffer after them; one barrier per
// k-step; each tile's fragments are read from LDS one tile ahead of its
// MFMAs.  The products of each accumulator run in the fused kernel's order
// (k-steps ascending; hi.hi, hi.lo, lo.hi), so H is the same bit for bit.
// ---------------------------------------------------------------------------
constexpr int G_CELLS = 256;
constexpr int G_NT = 16;             // most grain tiles per pass
constexpr int G_ROW = 40;            // bf16 per LDS row of a cell (32 + 8 pad)
constexpr int GW = 16;               // waves per workgroup (four per SIMD)

// NT: grain tiles of the instantiation (the pass's own count nt <= NT; the
// MFMAs run over all NT without branches, the surplus ones on stale LDS, and
// their accumulators are dropped).
// VW: J load width in floats (4 or 2: rows and J aligned to it; 1 otherwise).
template <int NT, int VW>
__global__ __launch_bounds__(64 * GW) __attribute__((amdgpu_waves_per_eu(GW / 4, GW / 4))) void absorb_gemm_kernel(
    PlanView v, int64_t C, const float* __restrict__ J, int64_t ldj, float* __restrict__ H,
    int64_t ldh) {
    __shared__ __align__(16) __bf16 sA[2][2][G_CELLS][G_ROW];  // 80 KB
    __shared__ __align__(16) bf16x8 sB[2][NT][2][64];           // up to 64 KB
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int row = lane & 15, kq = lane >> 4;
    const int t0 = (int)blockIdx.y * NT;
    const int nt = __builtin_amdgcn_readfirstlane(min(NT, v.Sp / 16 - t0));
    const int nsteps = v.NLp / 32;
    const int64_t c0 = (int64_t)blockIdx.x * G_CELLS;
    // J loader: thread t takes cell t / TPR, wavelengths PER (t mod TPR) .. + PER of a k-step
    constexpr int NTH = 64 * GW;
    constexpr int PER = G_CELLS * 32 / NTH;   // J values per thread and step
    constexpr int TPR = 32 / PER;             // threads per cell row
    const int lc = tid / TPR, lk = (tid % TPR) * PER;
    const int64_t lcell = c0 + lc;
    const float* jrow = J + (lcell < C ? lcell : 0) * ldj;
    auto load_j = [&](int step, float (&x)[PER]) {
        const int k0 = step * 32 + lk;
        if (lcell >= C) {
#pragma unroll
            for (int e = 0; e < PER; ++e) x[e] = 0.0f;
        } else if (VW == 4 && k0 + PER <= v.NL) {
#pragma unroll
            for (int q = 0; q < PER / 4; ++q) {
                const float4 f = *reinterpret_cast<const float4*>(jrow + k0 + 4 * q);
                x[4 * q] = f.x;
                x[4 * q + 1] = f.y;
                x[4 * q + 2] = f.z;
                x[4 * q + 3] = f.w;
            }
        } else if (VW == 2 && k0 + PER <= v.NL) {
#pragma unroll
            for (int q = 0; q < PER / 2; ++q) {
                const float2 f = *reinterpret_cast<const float2*>(jrow + k0 + 2 * q);
                x[2 * q] = f.x;
                x[2 * q + 1] = f.y;
            }
        } else {
#pragma unroll
            for (int e = 0; e < PER; ++e) x[e] = k0 + e < v.NL ? jrow[k0 + e] : 0.0f;
        }
    };
    auto store_j = [&](int buf, const float (&x)[PER]) {
        bf16x8 hi[PER / 8], lo[PER / 8];
#pragma unroll
        for (int e = 0; e < PER; ++e) {
            const __bf16 h = (__bf16)x[e];
            hi[e >> 3][e & 7] = h;
            lo[e >> 3][e & 7] = (__bf16)(x[e] - (float)h);
        }
#pragma unroll
        for (int q = 0; q < PER / 8; ++q) {
            *reinterpret_cast<bf16x8*>(&sA[buf][0][lc][lk + 8 * q]) = hi[q];
            *reinterpret_cast<bf16x8*>(&sA[buf][1][lc][lk + 8 * q]) = lo[q];
        }
    };
    // fragment loader: entry e = tid + NTH q: tile e / 128, plane (e / 64) mod 2, lane e mod 64
    constexpr int KQ = (NT * 128 + NTH - 1) / NTH;  // fragment entries per thread
    auto load_k = [&](int step, bf16x8 (&y)[KQ]) {
#pragma unroll
        for (int q = 0; q < KQ; ++q) {
            const int e = tid + NTH * q;
            const int t = e >> 7, pl = (e >> 6) & 1, ln = e & 63;
            if (t < nt) {
                const int64_t o = (((int64_t)(t0 + t) * nsteps + step) * 64 + ln) * 8;
                y[q] = *reinterpret_cast<const bf16x8*>((pl ? v.klo : v.khi) + o);
            }
        }
    };
    auto store_k = [&](int buf, const bf16x8 (&y)[KQ]) {
#pragma unroll
        for (int q = 0; q < KQ; ++q) {
            const int e = tid + NTH * q;
            const int t = e >> 7, pl = (e >> 6) & 1, ln = e & 63;
            if (t < nt) sB[buf][t][pl][ln] = y[q];
        }
    };
    // wave layout: WC cell groups x WGR grain groups; a wave takes MBW row
    // blocks (16 MBW cells) x TW grain tiles, so each fragment read from LDS
    // feeds 3 MBW MFMAs
    constexpr int WGR = NT >= 8 ? 2 : 1;
    constexpr int WC = GW / WGR;
    constexpr int MBW = 16 / WC;
    constexpr int TW = NT / WGR;
    static_assert(TW * WGR == NT, "tiles split evenly over grain groups");
    const int cg = wave % WC, gg = wave / WC;
    f32x4 acc[MBW][TW];
#pragma unroll
    for (int mb = 0; mb < MBW; ++mb)
#pragma unroll
        for (int t = 0; t < TW; ++t) acc[mb][t] = f32x4{0.f, 0.f, 0.f, 0.f};
    float x[PER];
    bf16x8 y[KQ];
    load_j(0, x);
    load_k(0, y);
    store_j(0, x);
    store_k(0, y);
    __syncthreads();
    for (int step = 0; step < nsteps; ++step) {
        const int buf = step & 1;
        const bool more = step + 1 < nsteps;
        if (more) {  // next k-step in flight
            load_j(step + 1, x);
            load_k(step + 1, y);
        }
        bf16x8 ahi[MBW], alo[MBW];
#pragma unroll
        for (int mb = 0; mb < MBW; ++mb) {
            const int cell = 16 * (MBW * cg + mb) + row;
            ahi[mb] = *reinterpret_cast<const bf16x8*>(&sA[buf][0][cell][kq * 8]);
            alo[mb] = *reinterpret_cast<const bf16x8*>(&sA[buf][1][cell][kq * 8]);
        }
        // fragments one tile ahead of their MFMAs
        bf16x8 bhi[2], blo[2];
        bhi[0] = sB[buf][TW * gg][0][lane];
        blo[0] = sB[buf][TW * gg][1][lane];
#pragma unroll
        for (int t = 0; t < TW; ++t) {
            if (t + 1 < TW) {
                bhi[(t + 1) & 1] = sB[buf][TW * gg + t + 1][0][lane];
                blo[(t + 1) & 1] = sB[buf][TW * gg + t + 1][1][lane];
            }
#pragma unroll
            for (int pr = 0; pr < 3; ++pr)
#pragma unroll
                for (int mb = 0; mb < MBW; ++mb)
                    acc[mb][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                        pr == 2 ? alo[mb] : ahi[mb], pr == 1 ? blo[t & 1] : bhi[t & 1],
                        acc[mb][t], 0, 0, 0);
        }
        if (more) {
            store_j(buf ^ 1, x);
            store_k(buf ^ 1, y);
        }
        __syncthreads();
    }
    // accumulator element r of lane (row, kq): cell 16 (MBW cg + mb) + 4 kq + r,
    // grain 16 (t0 + TW gg + t) + row
#pragma unroll
    for (int t = 0; t < TW; ++t) {
        const int s = 16 * (t0 + TW * gg + t) + row;
        if (TW * gg + t < nt && s < v.S) {
            const float hinv = v.hinv[s];
#pragma unroll
            for (int mb = 0; mb < MBW; ++mb)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int64_t c = c0 + 16 * (MBW * cg + mb) + 4 * kq + r;
                    if (c < C) H[c * ldh + s] = acc[mb][t][r] * hinv;
                }
        }
    }
}

// ---------------------------------------------------------------------------
// The same blocked product with J and the weight fragments moved from memory
// straight into LDS (global_load_lds_dwordx4: no staging registers), J three
// k-steps deep, so that two k-steps of J (64 KB per CU) are in flight while
// the MFMAs of a third run; the register-staged form above keeps one (32 KB).
// J lands in LDS as FP32; the wave that loaded a row block splits it in
// place into bf16 hi and lo before the k-step's barrier, once per value for
// all the waves that read it (the same round-to-nearest-even split as above,
// so H is the same bit for bit).  LDS: 3 x 32 KB of J + the double-buffered
// fragments (160 KB at 16 tiles).  Needs J rows 16-byte aligned; a ragged
// last k-step (NL not a multiple of 32) is read from global memory into
// registers with zeros past NL; rows past C read row C - 1 and are not stored.
// Stage layout [row block][chunk of 4 wavelengths][row] of float4: a wave's
// direct load fills one row block's 4 chunks x 16 rows (1 KB, lane l at
// chunk l / 16, row l mod 16), and a fragment read (lanes 0-15: rows 0-15 of
// one chunk) touches 256 consecutive bytes.
// Synchronisation is by hand: every full k-step issues the same loads in the
// same order (fragments of step + 1, then J of step + 2), so "all but this
// wave's last two loads landed" (vmcnt(2)) before the barrier means the
// k-step about to be read is in LDS; the LDS reads are asm statements that
// wait for themselves, since the compiler would make each read wait for every
// direct load in flight.
// ---------------------------------------------------------------------------
constexpr int D_STAGES = 3;
typedef __attribute__((address_space(3))) void* lds_ptr;
typedef float4 JStage[G_CELLS / 16][8][16];  // 32 KB

// vmcnt(n) with lgkmcnt(0): this wave's LDS writes done and all but its last
// n global loads (the direct loads of the next k-step) landed.
#define DUST_WAIT_VM2_LGKM0 0x0072
#define DUST_WAIT_VM0_LGKM0 0x0070

// Two 16-byte LDS reads (at addr + OFF and addr + OFF + GAP) and their wait,
// as one statement: the compiler would otherwise make every LDS read wait for
// all the direct loads in flight (it cannot tell the stages apart), which
// would undo the pipeline.  The offsets are immediates, so a wave needs one
// address register per array.
template <int OFF, int GAP, typename T>
__device__ __forceinline__ void lds_read2(uint32_t addr, T& a, T& b) {
    static_assert(OFF >= 0 && OFF + GAP < 65536, "16-bit LDS offset");
    asm volatile(
        "ds_read_b128 %0, %2 offset:%3\n\t"
        "ds_read_b128 %1, %2 offset:%4\n\t"
        "s_waitcnt lgkmcnt(0)"
        : "=&v"(a), "=&v"(b)
        : "v"(addr), "i"(OFF), "i"(OFF + GAP));
}
// Two 16-byte LDS writes (at addr + OFF and addr + OFF + GAP) and their wait.
template <int OFF, int GAP, typename T>
__device__ __forceinline__ void lds_write2(uint32_t addr, const T& a, const T& b) {
    static_assert(OFF >= 0 && OFF + GAP < 65536, "16-bit LDS offset");
    asm volatile(
        "ds_write_b128 %0, %1 offset:%3\n\t"
        "ds_write_b128 %0, %2 offset:%4\n\t"
        "s_waitcnt lgkmcnt(0)"
        :
        : "v"(addr), "v"(a), "v"(b), "i"(OFF), "i"(OFF + GAP)
        : "memory");
}
template <typename T>
__device__ __forceinline__ uint32_t lds_addr(T* p) {
    return (uint32_t)(uintptr_t)(__attribute__((address_space(3))) T*)p;
}
// f(integral_constant<int, I>) for I = B .. E - 1, unrolled at compile time
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

template <int NT>
__global__ __launch_bounds__(64 * GW) __attribute__((amdgpu_waves_per_eu(GW / 4, GW / 4))) void absorb_dl_kernel(
    PlanView v, int64_t C, const float* __restrict__ J, int64_t ldj, float* __restrict__ H,
    int64_t ldh) {
    __shared__ __align__(16) JStage sJ0, sJ1, sJ2;        // 96 KB
    __shared__ __align__(16) bf16x8 sB[2][NT][2][64];     // up to 64 KB
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int row = lane & 15, kq = lane >> 4;
    const int t0 = (int)blockIdx.y * NT;
    const int nt = __builtin_amdgcn_readfirstlane(min(NT, v.Sp / 16 - t0));
    const int nsteps = v.NLp / 32;
    const int nfull = v.NL / 32;  // k-steps with every wavelength inside NL
    const int64_t c0 = (int64_t)blockIdx.x * G_CELLS;
    // J mover: wave w fills row block w (GW = 16 row blocks of 16 cells); a
    // k-step past the last full one re-reads that one into a stage nobody
    // reads again, so that every k-step issues the same two loads last
    const int64_t dcell = c0 + 16 * wave + row;
    const float* drow = J + (dcell < C ? dcell : C - 1) * ldj + 4 * kq;
    auto next_j = [&](int step, JStage& dst) {
        const int sj = step < nfull ? step : nfull - 1;
#pragma unroll
        for (int i = 0; i < 2; ++i)
            __builtin_amdgcn_global_load_lds(drow + sj * 32 + 16 * i,
                                             (lds_ptr)&dst[wave][4 * i][0], 16, 0, 0);
    };
    // fragment mover: the plan's fragment (tile t, plane pl) of a k-step is
    // 64 x 16 bytes in lane order, one direct load into sB[buf][t][pl];
    // fragment p = wave + 16 j of the 2 NT goes to tile p / 2, plane p mod 2
    constexpr int PW = (2 * NT + GW - 1) / GW;
    auto next_k = [&](int step, int buf) {
#pragma unroll
        for (int j = 0; j < PW; ++j) {
            const int p = wave + GW * j;
            const int t = p >> 1, pl = p & 1;
            if (p < 2 * NT && t < nt) {
                const int64_t o = (((int64_t)(t0 + t) * nsteps + step) * 64 + lane) * 8;
                __builtin_amdgcn_global_load_lds((pl ? v.klo : v.khi) + o,
                                                 (lds_ptr)&sB[buf][t][pl][0], 16, 0, 0);
            }
        }
    };
    // wave layout: WC cell groups x WGR grain groups, each wave MBW row blocks
    // x TW tiles (16 tiles: 32 cells x 128 grains; 64 x 64, a fifth fewer LDS
    // bytes per MFMA, measured the same)
    constexpr int WGR = NT >= 6 ? 2 : 1;
    constexpr int WC = GW / WGR;
    constexpr int MBW = 16 / WC;
    constexpr int TW = NT / WGR;
    static_assert(TW * WGR == NT, "tiles split evenly over grain groups");
    const int cg = wave % WC, gg = wave / WC;
    f32x4 acc[MBW][TW];
#pragma unroll
    for (int mb = 0; mb < MBW; ++mb)
#pragma unroll
        for (int t = 0; t < TW; ++t) acc[mb][t] = f32x4{0.f, 0.f, 0.f, 0.f};
    // bf16 hi and lo of the wave's J values (row `row`, wavelengths 8 kq ..
    // 8 kq + 7 of a k-step) of row block mb
    // (two values per v_cvt_pk_bf16_f32, the hi parts back to FP32 by shift
    // and mask: the same round-to-nearest-even split as element by element,
    // in three instructions per value instead of four)
    auto split = [&](const float (&x)[8], bf16x8& hi, bf16x8& lo) {
        typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
        typedef float f32x2 __attribute__((ext_vector_type(2)));
        typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
        u32x4 h, l;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const float a = x[2 * e], b = x[2 * e + 1];
            const uint32_t hp =
                __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2{a, b}, bf16x2));
            const f32x2 r = {a - __uint_as_float(hp << 16), b - __uint_as_float(hp & 0xffff0000u)};
            h[e] = hp;
            l[e] = __builtin_bit_cast(uint32_t, __builtin_convertvector(r, bf16x2));
        }
        hi = __builtin_bit_cast(bf16x8, h);
        lo = __builtin_bit_cast(bf16x8, l);
    };
    // the MFMAs of one k-step from the split J and fragment buffer buf; the
    // wave's fragments of tile t sit at b0 + 2 KB t (hi) and + 1 KB (lo)
    const uint32_t b0 = lds_addr(&sB[0][TW * gg][0][lane]);
    constexpr uint32_t BUF_BYTES = sizeof(bf16x8) * NT * 2 * 64;
    auto mfmas = [&](const bf16x8 (&ahi)[MBW], const bf16x8 (&alo)[MBW], int buf) {
        const uint32_t bb = b0 + (buf ? BUF_BYTES : 0u);
        bf16x8 bhi[2], blo[2];
        lds_read2<0, 1024>(bb, bhi[0], blo[0]);
        static_for<0, TW>([&](auto tc) {
            constexpr int t = decltype(tc)::value;
#pragma unroll
            for (int pr = 0; pr < 3; ++pr)
#pragma unroll
                for (int mb = 0; mb < MBW; ++mb)
                    acc[mb][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                        pr == 2 ? alo[mb] : ahi[mb], pr == 1 ? blo[t & 1] : bhi[t & 1],
                        acc[mb][t], 0, 0, 0);
            if constexpr (t + 1 < TW)  // the next tile's fragments while these MFMAs run
                lds_read2<2048 * (t + 1), 1024>(bb, bhi[(t + 1) & 1], blo[(t + 1) & 1]);
        });
    };
    // a bare barrier (a fenced one would also wait for the loads in flight);
    // the empty asm statements keep the compiler's memory accesses on their side
    auto barrier = [&]() {
        asm volatile("" ::: "memory");
        __builtin_amdgcn_s_barrier();
        asm volatile("" ::: "memory");
    };
    // one full k-step: J of `step` in cur; fragments of step + 1 and J of
    // step + 2 are issued (in that order) before its MFMAs
    auto substep = [&](int step, JStage& cur, JStage& nxt2) {
        __builtin_amdgcn_s_waitcnt(DUST_WAIT_VM2_LGKM0);  // all but step + 1's J loads
        {
            // split the row block this wave loaded, in place, once for all the
            // waves that read it: the 8 values of (row, chunks 2 kq and
            // 2 kq + 1) become their bf16 hi (in chunk 2 kq) and lo (in chunk
            // 2 kq + 1), where the operand reads below find them
            const uint32_t own = lds_addr(&cur[wave][2 * kq][row]);
            f32x4 p, q;
            lds_read2<0, 256>(own, p, q);
            const float x[8] = {p[0], p[1], p[2], p[3], q[0], q[1], q[2], q[3]};
            bf16x8 hi, lo;
            split(x, hi, lo);
            lds_write2<0, 256>(own, hi, lo);
        }
        barrier();
        if (step + 1 < nsteps) next_k(step + 1, (step + 1) & 1);
        next_j(step + 2, nxt2);  // the stage every wave finished reading before the barrier
        // the wave's split J of row block MBW cg + mb: hi at a0 + 2 KB mb, lo + 256 B
        const uint32_t a0 = lds_addr(&cur[MBW * cg][2 * kq][row]);
        bf16x8 ahi[MBW], alo[MBW];
        static_for<0, MBW>([&](auto mc) {
            constexpr int mb = decltype(mc)::value;
            lds_read2<2048 * mb, 256>(a0, ahi[mb], alo[mb]);
        });
        mfmas(ahi, alo, step & 1);
    };
    next_k(0, 0);
    if (nfull > 0) {
        next_j(0, sJ0);
        next_j(1, sJ1);
        int step = 0;
        for (; step + 3 <= nfull; step += 3) {
            substep(step, sJ0, sJ2);
            substep(step + 1, sJ1, sJ0);
            substep(step + 2, sJ2, sJ1);
        }
        if (step < nfull) substep(step, sJ0, sJ2);
        if (step + 1 < nfull) substep(step + 1, sJ1, sJ0);
    }
    __builtin_amdgcn_s_waitcnt(DUST_WAIT_VM0_LGKM0);  // no load into LDS outlives this point
    if (nfull < nsteps) {  // the ragged last k-step: J straight from global, zeros past NL
        barrier();
        bf16x8 ahi[MBW], alo[MBW];
#pragma unroll
        for (int mb = 0; mb < MBW; ++mb) {
            const int64_t c = c0 + 16 * (MBW * cg + mb) + row;
            const int k = nfull * 32 + 8 * kq;
            const float* src = J + (c < C ? c : 0) * ldj + k;
            float x[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) x[e] = (c < C && k + e < v.NL) ? src[e] : 0.0f;
            split(x, ahi[mb], alo[mb]);
        }
        mfmas(ahi, alo, nfull & 1);
    }
#pragma unroll
    for (int t = 0; t < TW; ++t) {
        const int s = 16 * (t0 + TW * gg + t) + row;
        if (TW * gg + t < nt && s < v.S) {
            const float hinv = v.hinv[s];
#pragma unroll
            for (int mb = 0; mb < MBW; ++mb)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int64_t c = c0 + 16 * (MBW * cg + mb) + 4 * kq + r;
                    if (c < C) H[c * ldh + s] = acc[mb][t][r] * hinv;
                }
        }
    }
}

// LDS the current device gives one workgroup (asked once per device; 0 if
// unknown).
int lds_per_block() {
    static int cached[64];  // 0 unknown, else bytes + 1
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
    if (!cached[dev]) {
        int lds = 0;
        (void)hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
        cached[dev] = lds + 1;
    }
    return cached[dev] - 1;
}

// Whether one workgroup can hold the register-staged blocked kernel's 144 KB,
// or the direct-load kernel's 160 KB (at 16 tiles).
bool gemm_fits() {
    return (size_t)lds_per_block() >=
           sizeof(__bf16) * 2 * 2 * G_CELLS * G_ROW + sizeof(bf16x8) * 2 * G_NT * 2 * 64;
}
bool dl_fits() {
    return (size_t)lds_per_block() >=
           sizeof(float4) * D_STAGES * G_CELLS * 8 + sizeof(bf16x8) * 2 * G_NT * 2 * 64;
}

template <int NT>
hipError_t launch_gemm(const PlanView& v, int64_t C, const float* J, int64_t ldj, float* H,
                       int64_t ldh, hipStream_t st) {
    const dim3 grid((unsigned)((C + G_CELLS - 1) / G_CELLS), (unsigned)((v.Sp / 16 + NT - 1) / NT));
    const uintptr_t a = (uintptr_t)J;
    if ((a & 15u) == 0 && (ldj & 3) == 0 && dl_fits())
        hipLaunchKernelGGL((absorb_dl_kernel<NT>), grid, dim3(64 * GW), 0, st, v, C, J, ldj, H,
                           ldh);
    else if ((a & 15u) == 0 && (ldj & 3) == 0)
        hipLaunchKernelGGL((absorb_gemm_kernel<NT, 4>), grid, dim3(64 * GW), 0, st, v, C, J, ldj, H,
                           ldh);
    else if ((a & 7u) == 0 && (ldj & 1) == 0)
        hipLaunchKernelGGL((absorb_gemm_kernel<NT, 2>), grid, dim3(64 * GW), 0, st, v, C, J, ldj, H,
                           ldh);
    else
        hipLaunchKernelGGL((absorb_gemm_kernel<NT, 1>), grid, dim3(64 * GW), 0, st, v, C, J, ldj, H,
                           ldh);
    return hipGetLastError();
}

template <int NTW>
hipError_t launch_ntw(const PlanView& v, int64_t C, const float* J, int64_t ldj, float* H,
                      int64_t ldh, hipStream_t st) {
    if (table_mode(v.mode) && gemm_fits()) {  // blocked bf16 hi+lo heating
        const int tiles = v.Sp / 16;
        if (tiles <= 2) return launch_gemm<2>(v, C, J, ldj, H, ldh, st);
        if (tiles <= 4) return launch_gemm<4>(v, C, J, ldj, H, ldh, st);
        if (tiles <= 6) return launch_gemm<6>(v, C, J, ldj, H, ldh, st);
        if (tiles <= 8) return launch_gemm<8>(v, C, J, ldj, H, ldh, st);
        if (tiles <= 12) return launch_gemm<12>(v, C, J, ldj, H, ldh, st);
        return launch_gemm<16>(v, C, J, ldj, H, ldh, st);  // passes of 16 tiles
    }
    if (table_mode(v.mode)) {  // bf16 hi+lo heating, 64 cells per workgroup
        constexpr int MB = 4;
        const dim3 grid((unsigned)((C + 16 * MB - 1) / (16 * MB)));
        const int tiles = v.Sp / 16;
        if (tiles <= 4)  // four waves, one grain tile each
            hipLaunchKernelGGL((absorb_mb_kernel<1, MB, 4>), grid, dim3(256), 0, st, v, C, J, ldj,
                               H, ldh);
        else if (tiles <= 8)
            hipLaunchKernelGGL((absorb_mb_kernel<1, MB, 8>), grid, dim3(512), 0, st, v, C, J, ldj,
                               H, ldh);
        else if (tiles <= 16)
            hipLaunchKernelGGL((absorb_mb_kernel<2, MB, 8>), grid, dim3(512), 0, st, v, C, J, ldj,
                               H, ldh);
        else  // four tiles per wave and pass; more passes above 32 tiles
            hipLaunchKernelGGL((absorb_mb_kernel<4, MB, 8>), grid, dim3(512), 0, st, v, C, J, ldj,
                               H, ldh);
        return hipGetLastError();
    }
    const dim3 grid((unsigned)((C + 15) / 16));
    const size_t lds = sizeof(float) * 16 * v.Sp + STAGE_BYTES;
    hipLaunchKernelGGL((absorb_kernel<DUST_PLAIN_FP32, NTW>), grid, dim3(256), lds, st, v, C, J,
                       ldj, H, ldh);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_absorb(const PlanView& v, int64_t C, const float* J, int64_t ldj, float* H,
                         int64_t ldh, hipStream_t st) {
    if (C == 0) return hipSuccess;
    const int ntw = (v.Sp / 16 + 3) / 4;  // grain tiles per wave in one pass
    if (ntw <= 1) return launch_ntw<1>(v, C, J, ldj, H, ldh, st);
    if (ntw <= 2) return launch_ntw<2>(v, C, J, ldj, H, ldh, st);
    if (ntw <= 3) return launch_ntw<3>(v, C, J, ldj, H, ldh, st);
    if (ntw <= 4) return launch_ntw<4>(v, C, J, ldj, H, ldh, st);
    return launch_ntw<4>(v, C, J, ldj, H, ldh, st);  // several passes
}

}  // namespace dust
