/* Throughput probes of the FP32 vector ALU (measurement utility).
 *
 * The sweeps of the renderer are bound by the vector ALU: fused multiply-adds
 * plus the transcendental instructions of the phase factors and reciprocals
 * (paper Sec. 4, Eq. 7-10).  To price a pair against the device, the
 * benchmark measures how many of each instruction kind the device retires
 * per second.  This library is not part of the renderer's interface.
 */
#ifndef DM_PROBE_H
#define DM_PROBE_H

#ifdef __cplusplus
extern "C" {
#endif

/* Instruction kinds of dmp_alu_time. */
enum {
  DMP_FMA = 0, /* v_fma_f32, all operands in VGPRs */
  DMP_SIN = 1, /* hardware sine (argument in revolutions) */
  DMP_COS = 2, /* hardware cosine */
  DMP_RCP = 3, /* hardware reciprocal */
  DMP_MIX = 4, /* per step 8 FMA chains and 2 sine chains, all independent */
  DMP_FMA_SGPR = 5 /* v_fma_f32 reading its multiplier from an SGPR */
};

/* Runs `blocks` workgroups of 256 lanes on `device`; every lane executes
 * `iters` steps of 8 independent dependency chains of the given kind (DMP_MIX:
 * 8 FMA and 2 sine chains per step).  Lane-instruction count per launch:
 * blocks * 256 * iters * 8 (DMP_MIX: plus blocks * 256 * iters * 2 sines).
 * Times `reps` launches after one warm-up with HIP events and writes the
 * average launch time in milliseconds to *ms_out (host pointer).  Allocates
 * and frees a device buffer of blocks * 256 floats.
 * Returns 0 on success, -1 for invalid arguments (op outside 0..5, blocks,
 * iters or reps < 1, ms_out NULL), -5 for a HIP error.  On gfx950 the
 * two FMA forms retire at different rates: an SGPR operand limits the
 * instruction to the base issue rate. */
int dmp_alu_time(int device, int op, int blocks, int iters, int reps, double* ms_out);

#ifdef __cplusplus
}
#endif

#endif
