/*
 * hs_probe -- instruction issue-rate probes used to pin the integer VALU
 * roofline of the sweep kernel on the device it runs on.  Measurement only:
 * no part of the parallel-tempering path calls it.
 */
#ifndef HS_PROBE_H
#define HS_PROBE_H

#ifdef __cplusplus
extern "C" {
#endif

/* Lane-operations per second of one instruction class, measured with 8
 * independent chains per thread on 8 workgroups of 256 threads per compute
 * unit (enough waves to saturate issue).
 *   which: 0 v_add_u32, 1 v_bitop3_b32, 2 v_mad_u64_u32, 3 v_mul_hi_u32,
 *          4 v_mul_lo_u32, 5 v_dot4_i32_i8, 6 v_mad_i32_i24
 *   iters: loop trip count (each trip issues 16 x 8 instructions per thread)
 *   scratch: device pointer to >= 4 writable bytes (never written in practice)
 * Synchronises the default stream.  Returns 0, -1 on bad arguments, -4 on a
 * HIP error. */
int hs_probe_rate(int which, int iters, double *ops_per_s, void *scratch);

#ifdef __cplusplus
}
#endif

#endif /* HS_PROBE_H */
