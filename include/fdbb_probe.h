/*
 * fdbb_probe.h -- streaming probes that measure what HBM delivers on the
 * device at hand (read-only, write-only, copy), and give the plain copy
 * kernel against which hardware byte counters are calibrated.  They are not
 * building blocks of the method; they bound them: every building block is a
 * pure streaming pass, so these rates are its practical ceiling.
 *
 * Pointers are device pointers, 16-byte aligned; `bytes` is a multiple of
 * 16.  Calls enqueue one kernel on `stream` (hipStream_t as void*, NULL for
 * the default stream) and return at once.  Return values are fdbb_status
 * codes (fdbb.h): FDBB_EINVAL for NULL, misaligned or negative arguments,
 * FDBB_EHIP for a launch error.
 */
#ifndef FDBB_PROBE_H
#define FDBB_PROBE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* dst[0 .. bytes) = src[0 .. bytes): reads and writes `bytes` each. */
int fdbb_probe_copy(const void *src, void *dst, int64_t bytes, int grid, void *stream);

/* Fill dst[0 .. bytes) with a 64-bit pattern; writes `bytes`. */
int fdbb_probe_write(void *dst, int64_t bytes, uint64_t pattern, int grid, void *stream);

/* Read src[0 .. bytes) and store one 64-bit xor per workgroup to sink[] (the
 * caller provides at least `grid` elements); reads `bytes`. */
int fdbb_probe_read(const void *src, int64_t bytes, uint64_t *sink, int grid, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* FDBB_PROBE_H */
