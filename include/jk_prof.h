/*
 * jk_prof.h -- kernel timing hook of the gfx950 J/K library, for benchmarks.
 *
 * When enabled, every kernel launch of the library is bracketed by a pair of
 * HIP events recorded on the launch stream (the stream passed to jk_build /
 * jk_vjp / jk_build_batched).  The events come from a pool created by
 * jk_prof_enable, so timing creates nothing inside the timed region.  Events
 * beyond the pool capacity are not recorded (jk_prof_dropped counts them).
 * Not thread-safe: enable, run, read from one host thread.
 */
#ifndef JK_GFX950_PROF_H
#define JK_GFX950_PROF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* capacity > 0: create a pool of capacity event pairs (on the current
 * device) and start recording; capacity == 0: stop recording.  Returns 0 on
 * success, -1 if the events could not be created. */
int jk_prof_enable(int32_t capacity);

/* Forget recorded launches (keeps the pool and the enabled state). */
void jk_prof_reset(void);

/* Synchronise the recorded events and aggregate them per kernel name.
 * Returns the number of distinct kernel names (or -1 on a HIP error). */
int32_t jk_prof_collect(void);

/* After jk_prof_collect: name, total milliseconds and launch count of entry i
 * (0 <= i < the collected count).  Returns 0, or -1 if i is out of range. */
int jk_prof_entry(int32_t i, const char **name, double *total_ms, int64_t *launches);

/* Launches not recorded because the pool was full. */
int64_t jk_prof_dropped(void);

/* Matrix-core peak microbenchmark on the current device (allocates a small
 * buffer, launches on the default stream and synchronises; not for use in a
 * timed region).  kind 0: V_MFMA_I32_32X32X32_I8 in the slice engine's
 * pattern (13 digit-pair products per two output tiles), in int8 ops/s;
 * kind 1: V_MFMA_F64_16X16X4_F64, in flop/s.  random != 0: operands drawn per
 * lane (uniform bytes, like the digits), else constants; the sustained INT8
 * rate depends on the data.  Returns -1 on an error. */
double jk_peak_mfma(int32_t kind, int32_t random);

#ifdef __cplusplus
}
#endif
#endif /* JK_GFX950_PROF_H */
