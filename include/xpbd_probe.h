/* Measurement support: the LDS bandwidth the step kernel's roofline is set
 * against.  Not part of the method; the benchmark calls it to state the LDS
 * peak it divides by.
 *
 * The step kernel reads a particle's position and inverse mass with one
 * 16-byte LDS read and writes a position with one 12-byte LDS write per
 * particle of every projection (Alg. 1's constraint loops).  The probe runs
 * those two access forms alone, conflict-free, on 256-thread workgroups of
 * 64 KB LDS each (two per CU), and reports what it moved and how long it
 * took. */
#ifndef XPBD_PROBE_H
#define XPBD_PROBE_H

#include <stdint.h>

#include "xpbd.h"

#ifdef __cplusplus
extern "C" {
#endif

#define XPBD_PROBE_LDS_READ_B128 0   /* 16-byte reads (ds_read_b128) */
#define XPBD_PROBE_LDS_WRITE_B96 1   /* 12-byte writes at a 16-byte stride (ds_write_b96) */

/* Run the probe `kind` on `workgroups` workgroups, each thread making 8
 * accesses per repetition for `reps` repetitions, on hip_stream (NULL: the
 * null stream), once untimed and once timed with HIP events.  Synchronises.
 * out (host, [4]): [0] the timed launch in ms, [1] bytes moved by it,
 * [2] mean shader-clock cycles per workgroup between the barriers around the
 * loop (s_memtime), [3] mean 100 MHz real-time ticks over the same span
 * (s_memrealtime).  Allocates and frees a small device buffer per call.
 * Errors: XPBD_E_ARG for an unknown kind, workgroups outside [1, 65536] or
 * reps outside [1, 2^24]; XPBD_E_HIP for a HIP failure. */
xpbd_status xpbd_lds_probe(int32_t kind, int32_t workgroups, int32_t reps, void *hip_stream,
                           double *out);

#ifdef __cplusplus
}
#endif

#endif /* XPBD_PROBE_H */
