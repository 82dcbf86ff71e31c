/*
 * alu_probe.h -- measurement-only library (libdust_probe.so), loaded by the
 * benchmark and by nothing else; not part of libdust's C-ABI.
 *
 * Throughput probes of the vector ALU forms the emission and the solve are
 * built from, for checking on the device at hand the ALU peak that roofline
 * figures divide by.  `blocks` workgroups of 256 threads each run `iters`
 * iterations of 8 independent dependency chains of the chosen form:
 *   ALU_PROBE_EXP2      v_exp_f32
 *   ALU_PROBE_RCP       v_rcp_f32
 *   ALU_PROBE_FMA       v_fma_f32
 *   ALU_PROBE_EXP2_FMA  v_exp_f32 plus an independent v_fma_f32 per step
 *                       (shows whether other VALU work issues alongside the
 *                       transcendental unit)
 *   ALU_PROBE_TERM      the emission's exact Planck term (mul, exp, sub, rcp,
 *                       fma)
 *   ALU_PROBE_FMA64     v_fma_f64 (the FP64 work of the fluctuating-grain
 *                       level recursion)
 * and writes one float per thread to the device buffer `out` (caller-owned,
 * at least 256 * blocks floats).  Returns 0 once launched on `stream` (a
 * hipStream_t; time it with events there), -1 for blocks or iters outside
 * [1, 2^20], a NULL `out` or an unknown kind, -4 when the launch fails.
 */
#ifndef ALU_PROBE_H
#define ALU_PROBE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    ALU_PROBE_EXP2 = 0,
    ALU_PROBE_RCP = 1,
    ALU_PROBE_FMA = 2,
    ALU_PROBE_EXP2_FMA = 3,
    ALU_PROBE_TERM = 4,
    ALU_PROBE_FMA64 = 5
};

int alu_probe_run(int32_t kind, int32_t blocks, int32_t iters, float* out, void* stream);

#ifdef __cplusplus
}
#endif
#endif
