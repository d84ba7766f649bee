/*
 * prngd_probe.h -- measurement probes of libprngd: the ceilings that bound a
 * PRNGD fill on the current GPU.  They compute nothing a user needs; they
 * price the parts of the fill (stores to HBM, the Philox4x32-10 integer
 * work of Section 2's base generator) for the roofline report.
 *
 * All calls enqueue one kernel on `stream` (a hipStream_t as void*, NULL =
 * null stream) and return 0 on success, 1 for invalid arguments (nothing
 * enqueued), 4 if the launch failed.  Buffers are caller-owned device
 * memory.
 */
#ifndef PRNGD_PROBE_H
#define PRNGD_PROBE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Write n doubles (n even; out 16-byte aligned), one 16-byte store per
 * thread over a one-shot grid: the HBM write ceiling of a fill of n
 * outputs. */
int prngd_probe_write(double *out, uint64_t n, void *stream);

/* Copy n doubles from src to dst (n even; both 16-byte aligned; the two
 * ranges must not overlap): 8n bytes read and 8n written, the known
 * traffic against which HBM byte counters are scaled. */
int prngd_probe_copy(double *dst, const double *src, uint64_t n, void *stream);

/* Compute `blocks` Philox4x32-10 blocks (a fill of n outputs of the single
 * Philox generator needs n / 2) and fold them into one word per thread of
 * `sink` (sink_words >= grid * 256; the grid shrinks to fit). */
int prngd_probe_philox(uint32_t *sink, uint64_t sink_words, uint64_t blocks, void *stream);

/* Philox blocks -> two pairs -> the Eq. (5) map -> 16-byte stores, every
 * pair kept (n even; out 16-byte aligned): the fill without acceptance,
 * compaction or the cross-block scan. */
int prngd_probe_philox_store(double *out, uint64_t n, void *stream);

/* For tests of the stall path of the ordered look-back: the polls a
 * look-back wait makes before it reports a stall, for launches planned
 * after the call (0 restores the default, 2^20).  A small value makes
 * waits that a correct launch would finish end early: that launch drains
 * (every wait is bounded, its outputs are not defined) and the next call
 * on the device returns PRNGD_ERR_DEVICE.  Host only; returns 0. */
int prngd_probe_set_spin_limit(uint32_t polls);

#ifdef __cplusplus
}
#endif
#endif
