/*
 * psclbm_probe.h -- bandwidth ceilings of the device, for the roofline of the
 * lattice step (part of libpsclbm.so, not of the method).
 *
 * The step kernel moves 2 Q s bytes per cell and step (Q distributions of s
 * bytes read and written once).  Its fraction of the HBM peak is compared with
 * what plain data movement of the same volume attains on the same device:
 *   - psclbm_stream_copy: a copy, each thread moving 16 bytes with
 *     non-temporal loads and stores;
 *   - psclbm_stream_swap: the memory traffic of an even lattice step alone, q
 *     structure-of-arrays FP32 arrays of n elements read at each cell and
 *     written back in place with the arrays of each opposite pair exchanged
 *     (array 0 stays; arrays 2k-1 and 2k swap), two cells per thread.
 * Both enqueue one kernel on the given HIP stream (a hipStream_t, NULL for
 * the null stream) and return without waiting; time them with events.  All
 * pointers are device pointers owned by the caller; nothing is allocated.
 */
#ifndef PSCLBM_PROBE_H
#define PSCLBM_PROBE_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Copy bytes from d_src to d_dst (not overlapping).  bytes must be a positive
 * multiple of 16 and both pointers 16-byte aligned (PSCLBM_EINVAL otherwise);
 * PSCLBM_EHIP if the launch fails. */
int psclbm_stream_copy(const void* d_src, void* d_dst, size_t bytes, void* hip_stream);

/* In-place exchange over q arrays of n floats each, array k at d_a + k n
 * (q 9 or 19; n even and positive; d_a 8-byte aligned; PSCLBM_EINVAL
 * otherwise); moves 8 q n bytes.  PSCLBM_EHIP if the launch fails. */
int psclbm_stream_swap(float* d_a, long long n, int q, void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* PSCLBM_PROBE_H */
