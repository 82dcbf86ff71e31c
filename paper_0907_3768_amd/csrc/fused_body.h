// The per-tile body of the fused absorb -> solve -> emit kernel, shared by
// the single-grid fused launch and the batched persistent launch.
#pragma once

#include "device_common.h"

namespace dust {

constexpr int FUSED_TC = 16;  // default cells per tile (one MFMA M-block)

// LDS staging of J in chunks of 16 cells x KC wavelengths, double-buffered.
// Mixed mode keeps a chunk as bf16 hi and lo planes (rows padded to KC + 8
// values), plain mode as FP32 (rows padded to KC + 4).  The padding makes a
// row 4 banks apart from the next, so the 16 lanes of each 128-bit read
// phase touch every bank exactly twice.  A chunk of 64 wavelengths halves
// the staging's LDS (one more barrier per 64 wavelengths); that pays where
// LDS, not registers, limits the resident workgroups (many grains).  The
// chunk width only changes when J is staged, not the order of the MFMA
// k-steps, so the heating is the same bit for bit.
template <int KC>
struct Stage {
    static_assert(KC % 32 == 0 && (KC / 16) % 2 == 0, "chunk of whole k-steps");
    static constexpr int KSTEPS = KC / 32;     // MFMA k-steps per chunk
    static constexpr int ROW_BF16 = KC + 8;
    static constexpr int ROW_F32 = KC + 4;
    static constexpr int BUF_BYTES = 2 * 16 * ROW_BF16 * 2;  // >= 16 * ROW_F32 * 4
    static_assert(BUF_BYTES >= 16 * ROW_F32 * 4, "FP32 staging must fit");
    static constexpr int BYTES = 2 * BUF_BYTES;
};
constexpr int ABS_KC = 128;  // default chunk width
constexpr int STAGE_BYTES = Stage<ABS_KC>::BYTES;

// Phase 1: heating of a 16-cell block into sH[16][Sp] (rows of the tile's
// LDS array) in the plan's scaled units H' = H 2^es, on the MFMA units.
//
// J streams through LDS in chunks of KC wavelengths: every thread loads
// KC/16 values of the next chunk (thread t: row t/16, column pairs
// 2 (t mod 16) + 32 i) while the current chunk is multiplied, then splits
// them (mixed: bf16 hi + lo) into the other buffer; one barrier per chunk.
// Each wave multiplies with its grain tiles w, w+4, ... (NTW of them per
// pass; grids with more than 4 NTW tiles take several passes).  (Loading the
// weight fragments one k-step ahead measured no faster and costs VGPRs.)
//
// K-order: lane (row = lane mod 16, q = lane / 16) supplies wavelengths
// k0 + 8q .. k0 + 8q + 7 to both operands -- one 16x16x32 bf16 MFMA, or eight
// 16x16x4 FP32 MFMAs in which MFMA i takes k0 + 8q + i.  Any assignment of
// wavelengths to MFMA k-slots gives the same sum as long as both operands
// use it.
template <int MODE, int NTW, int KC = ABS_KC>
__device__ __forceinline__ void fused_absorb(const PlanView& v, int64_t c0, int64_t C,
                                             const float* __restrict__ J, int64_t ldj,
                                             float* sH, char* sStage) {
    constexpr bool BF = table_mode(MODE);
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int row = lane & 15, kq = lane >> 4;
    const int tiles = v.Sp / 16;
    // loader role: 256 threads x KC/16 values = one 16 x KC chunk
    using St = Stage<KC>;
    constexpr int NX = KC / 16;  // values per thread
    const int lrow = tid >> 4, lcol = (tid & 15) * 2;
    const bool lrow_ok = c0 + lrow < C;
    const float* jl = J + (lrow_ok ? c0 + lrow : 0) * ldj;

    auto load_j = [&](int k0, float (&x)[NX]) {
#pragma unroll
        for (int i = 0; i < NX / 2; ++i) {
            const int k = k0 + lcol + 32 * i;
            x[2 * i] = (lrow_ok && k < v.NL) ? jl[k] : 0.0f;
            x[2 * i + 1] = (lrow_ok && k + 1 < v.NL) ? jl[k + 1] : 0.0f;
        }
    };
    // this thread's first slot in a staging buffer; the other slots are
    // constant offsets from it (lcol is even)
    const int slot0 = BF ? (lrow * St::ROW_BF16 + lcol) / 2 : (lrow * St::ROW_F32 + lcol) / 2;
    auto store_j = [&](int buf, const float (&x)[NX]) {
        char* base = sStage + buf * St::BUF_BYTES;
#pragma unroll
        for (int i = 0; i < NX / 2; ++i) {
            const float x0 = x[2 * i], x1 = x[2 * i + 1];
            if constexpr (BF) {
                // [hi|lo][16 rows][ROW_BF16] bf16; a pair of columns per 32-bit store
                typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
                const __bf16 h0 = (__bf16)x0, h1 = (__bf16)x1;
                const bf16x2 hi = {h0, h1};
                const bf16x2 lo = {(__bf16)(x0 - (float)h0), (__bf16)(x1 - (float)h1)};
                bf16x2* b = reinterpret_cast<bf16x2*>(base) + slot0;
                b[16 * i] = hi;
                b[8 * St::ROW_BF16 + 16 * i] = lo;
            } else {
                float2* b = reinterpret_cast<float2*>(base) + slot0;
                b[16 * i] = make_float2(x0, x1);
            }
        }
    };

    const int nsteps = v.NLp / 32;  // k-steps (NLp is a multiple of 32)
    // Weight fragments of one k-step for the wave's tiles (bf16 hi/lo, or
    // 8 FP32 values).
    struct KFrag {
        bf16x8 hi[NTW], lo[NTW];
        float4 f0[NTW], f1[NTW];
    };
    auto load_k = [&](int tg, int k0, KFrag& f) {
#pragma unroll
        for (int t = 0; t < NTW; ++t) {
            const int tile = tg + wave + 4 * t;
            if (tile < tiles) {
                // fragment order: this lane's 8 values of (tile, k-step) (see kfrag_bf16)
                const int64_t fr = (int64_t)tile * nsteps + (k0 >> 5);
                if constexpr (BF) {
                    const int64_t o = (fr * 64 + lane) * 8;
                    f.hi[t] = *reinterpret_cast<const bf16x8*>(v.khi + o);
                    f.lo[t] = *reinterpret_cast<const bf16x8*>(v.klo + o);
                } else {
                    const int64_t o = (fr * 128 + lane) * 4;
                    f.f0[t] = *reinterpret_cast<const float4*>(v.kf + o);
                    f.f1[t] = *reinterpret_cast<const float4*>(v.kf + o + 256);
                }
            }
        }
    };

    const int nchunks = (nsteps + St::KSTEPS - 1) / St::KSTEPS;
    // Grain tiles in groups of 4 NTW (one pass over J each).
    for (int tg = 0; tg < tiles; tg += 4 * NTW) {
        f32x4 acc[NTW];
#pragma unroll
        for (int t = 0; t < NTW; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
        float x[NX];
        load_j(0, x);
        store_j(0, x);
        __syncthreads();
        for (int ch = 0; ch < nchunks; ++ch) {
            const int buf = ch & 1;
            if (ch + 1 < nchunks) load_j((ch + 1) * KC, x);  // next chunk in flight
#pragma unroll 1
            for (int ks = 0; ks < St::KSTEPS; ++ks) {
                const int step = ch * St::KSTEPS + ks;
                if (step >= nsteps) break;  // uniform
                KFrag kc;
                load_k(tg, step * 32, kc);
                if constexpr (BF) {
                    const __bf16* b = reinterpret_cast<const __bf16*>(sStage + buf * St::BUF_BYTES);
                    const bf16x8 ahi = *reinterpret_cast<const bf16x8*>(
                        b + row * St::ROW_BF16 + ks * 32 + kq * 8);
                    const bf16x8 alo = *reinterpret_cast<const bf16x8*>(
                        b + 16 * St::ROW_BF16 + row * St::ROW_BF16 + ks * 32 + kq * 8);
#pragma unroll
                    for (int t = 0; t < NTW; ++t) {
                        if (tg + wave + 4 * t < tiles) {
                            acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi, kc.hi[t], acc[t], 0, 0, 0);
                            acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi, kc.lo[t], acc[t], 0, 0, 0);
                            acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo, kc.hi[t], acc[t], 0, 0, 0);
                        }
                    }
                } else {
                    const float* b = reinterpret_cast<const float*>(sStage + buf * St::BUF_BYTES);
                    const float4 a0 = *reinterpret_cast<const float4*>(
                        b + row * St::ROW_F32 + ks * 32 + kq * 8);
                    const float4 a1 = *reinterpret_cast<const float4*>(
                        b + row * St::ROW_F32 + ks * 32 + kq * 8 + 4);
                    const float a[8] = {a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w};
#pragma unroll
                    for (int t = 0; t < NTW; ++t) {
                        if (tg + wave + 4 * t < tiles) {
                            const float bb[8] = {kc.f0[t].x, kc.f0[t].y, kc.f0[t].z, kc.f0[t].w,
                                                 kc.f1[t].x, kc.f1[t].y, kc.f1[t].z, kc.f1[t].w};
#pragma unroll
                            for (int i = 0; i < 8; ++i)
                                acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], bb[i], acc[t], 0, 0, 0);
                        }
                    }
                }
            }
            if (ch + 1 < nchunks) store_j(buf ^ 1, x);
            __syncthreads();
        }
#pragma unroll
        for (int t = 0; t < NTW; ++t) {
            const int tile = tg + wave + 4 * t;
            if (tile < tiles) {
                const int s = tile * 16 + row;
#pragma unroll
                for (int r = 0; r < 4; ++r) sH[(kq * 4 + r) * v.Sp + s] = acc[t][r];
            }
        }
    }  // tile groups
}

// Phases 2 and 3 on a tile whose scaled heating sits in sH: solve every pair
// (T to device memory, 1/T back into sH), then emit the tile's SEDs.  The
// group minima of 1/T follow sH in LDS (see emit_accumulate).
// LDS used by the solve phase for its list of pending pairs.
constexpr int SOLVE_LDS_BYTES = (PENDING_CAP + 4) * (int)sizeof(int);

// Phase 2: solve every pair of the tile from sH (scaled heating, to which
// the optional extra heating Q is added), write T and leave 1/T in sH.
// Mixed: pairs outside the table are marked by a negative sH (-H'), listed
// in LDS and solved exactly by the block's waves in turn; the list is
// rebuilt until no mark is left.  Plain: Newton from the Eq. 11 guess or,
// with a warm start, from the T already in the output.  Table-linear:
// interpolation in the grain's table.
template <int MODE, int TC>
__device__ __forceinline__ void fused_solve(const PlanView& v, int64_t c0, int64_t C,
                                            float* __restrict__ T, int64_t ldt,
                                            dust_counters* cnt, float* sH, int* sSolve) {
    const int n = TC * v.Sp;
    int* sCount = sSolve;
    int* sList = sSolve + 4;
    if constexpr (mixed_mode(MODE)) {
        if (threadIdx.x == 0) *sCount = 0;
        __syncthreads();
    }
    int evals = 0;
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        // Plain: cells fastest, so a wave spans 64/TC grains and the Newton
        // sums read few distinct weight rows.  Otherwise grains fastest.
        int cc, s;
        if constexpr (MODE == DUST_PLAIN_FP32) {
            s = j / TC;
            cc = j - s * TC;
        } else {
            cc = j / v.Sp;
            s = j - cc * v.Sp;
        }
        const int i = cc * v.Sp + s;
        const int64_t c = c0 + cc;
        const bool pair = s < v.S && c < C;
        float inv = __builtin_inff();
        if (pair) {
            float h = sH[i];
            if (v.q) h += v.q[c * v.ldq + s] * v.hscale[s];
            float t;
            if constexpr (mixed_mode(MODE)) {
                if (mixed_lookup<MODE>(v, s, h, &t, cnt) != 0) {
                    const int k = atomicAdd(sCount, 1);
                    if (k < PENDING_CAP) sList[k] = i;
                    sH[i] = -h;  // pending: solved below
                    continue;
                }
            } else if constexpr (MODE == DUST_TABLE_LINEAR) {
                t = table_linear_T(v, s, h, cnt);
            } else {
                const float t0 = v.warm ? T[c * ldt + s] : 0.0f;
                int ev;
                t = solve_newton_f32(v.kb + (int64_t)s * v.NLp, v.nu, v.NL, h, v.gs[s], v.tol,
                                     v.maxit, t0, &ev, cnt);
                evals += ev;
            }
            T[c * ldt + s] = t;
            inv = inv_temperature(t);
        }
        sH[i] = inv;
    }
    if constexpr (MODE == DUST_PLAIN_FP32) {
        if (cnt) wave_count_add(&cnt->n_newton_evals, evals);
    }
    if constexpr (mixed_mode(MODE)) {
        __syncthreads();
        for (;;) {
            const int total = *sCount;
            if (total == 0) break;  // uniform: read after a barrier
            const int listed = total < PENDING_CAP ? total : PENDING_CAP;
            for (int e = threadIdx.x >> 6; e < listed; e += blockDim.x >> 6) {
                const int i = sList[e];
                const int cc = i / v.Sp, s = i - cc * v.Sp;
                const float t = wave_solve_pending(v, s, -(double)sH[i], cnt);
                if ((threadIdx.x & 63) == 0) {
                    T[(c0 + cc) * ldt + s] = t;
                    sH[i] = inv_temperature(t);
                }
            }
            __syncthreads();
            if (total <= PENDING_CAP) break;
            // the list overflowed: collect the pairs still marked
            if (threadIdx.x == 0) *sCount = 0;
            __syncthreads();
            for (int i = threadIdx.x; i < n; i += blockDim.x) {
                if (sH[i] < 0.0f) {
                    const int k = atomicAdd(sCount, 1);
                    if (k < PENDING_CAP) sList[k] = i;
                }
            }
            __syncthreads();
        }
    }
}

template <int MODE, int TC, bool TAIL>
__device__ __forceinline__ void fused_solve_emit(const PlanView& v, int64_t c0, int64_t C,
                                                 const float* __restrict__ m,
                                                 float* __restrict__ T, int64_t ldt,
                                                 float* __restrict__ L, int64_t ldl,
                                                 dust_counters* cnt, float* sH) {
    const int n = TC * v.Sp;
    fused_solve<MODE, TC>(v, c0, C, T, ldt, cnt, sH,
                          reinterpret_cast<int*>(reinterpret_cast<char*>(sH) +
                                                 emit_lds_bytes(TC, v.Sp)));
    __syncthreads();
    uint32_t* sChunk = reinterpret_cast<uint32_t*>(sH + n);
    fill_chunk_min<TC>(sH, sChunk, v.Sp);
    __syncthreads();
    // Wave w takes the wavelength blocks w, w + 4, ...; grids with fewer
    // than four blocks would leave waves idle, so there the waves split the
    // tile's cells as well.
    constexpr int LW = 64 / EMIT_ROWS;
    const int NB = (v.NL + LW - 1) / LW;
    if (NB >= 4) {
        const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
        emit_tile<EMIT_ROWS, TC, TAIL>(v, c0, C, m, L, ldl, sH, sChunk, w, 4, NB);
    } else if (v.NL > 64) {
        emit_cell_part<TC / 2, TC>(v, c0, C, m, L, ldl, sH, sChunk, 2);
    } else {
        emit_cell_part<TC / 4, TC>(v, c0, C, m, L, ldl, sH, sChunk, 1);
    }
}

// LDS bytes of a fused tile of TC cells.  The first TC x Sp floats hold H'
// and then 1/T throughout.  Behind them the J staging buffers of the heating
// share the space with what only the later phases use: the emission's group
// minima (sChunk, sPair) and the solve's pending list, which follows them.
// The heating's last read of the staging precedes a barrier, so the sharing
// needs no extra synchronisation; it lowers the LDS a workgroup holds, and
// with it the limit on resident workgroups, by the smaller of the two.
__host__ __device__ constexpr size_t fused_lds_bytes(int TC, int Sp, int stage_bytes) {
    return (size_t)TC * Sp * sizeof(float) + stage_bytes >
                   emit_lds_bytes(TC, Sp) + SOLVE_LDS_BYTES
               ? (size_t)TC * Sp * sizeof(float) + stage_bytes
               : emit_lds_bytes(TC, Sp) + SOLVE_LDS_BYTES;
}

// Chunk width of the single-grid fused kernel: with three or four grain
// tiles per wave (more than 128 grains) the tile's LDS, not its registers,
// limits the resident workgroups, and the narrower chunk lifts that limit.
__host__ __device__ constexpr int fused_kc(int ntw) { return ntw >= 3 ? 64 : 128; }

// One tile of TC cells (TC a multiple of 16) starting at cell c0, J staged in
// chunks of KC wavelengths; lds holds fused_lds_bytes(TC, Sp,
// Stage<KC>::BYTES) bytes.  Ends with every thread past its last read of the
// tile's LDS.
template <int MODE, int TC, int NTW, bool TAIL, int KC>
__device__ __forceinline__ void fused_tile(const PlanView& v, int64_t c0, int64_t C,
                                           const float* __restrict__ J, int64_t ldj,
                                           const float* __restrict__ m, float* __restrict__ T,
                                           int64_t ldt, float* __restrict__ L, int64_t ldl,
                                           dust_counters* cnt, float* lds) {
    float* sH = lds;
    char* sStage = reinterpret_cast<char*>(lds + TC * v.Sp);  // shared, see fused_lds_bytes
#pragma unroll
    for (int mb = 0; mb < TC / 16; ++mb)
        fused_absorb<MODE, NTW, KC>(v, c0 + 16 * mb, C, J, ldj, sH + 16 * mb * v.Sp, sStage);
    __syncthreads();
    fused_solve_emit<MODE, TC, TAIL>(v, c0, C, m, T, ldt, L, ldl, cnt, sH);
    __syncthreads();
}

}  // namespace dust
