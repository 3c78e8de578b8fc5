/*
 * rowbench.h -- measurement kernels beside libpg (librowbench.so): the
 * achievable HBM read bandwidth of the device, and the sorted-row
 * intersection |N(u) & N(v)| over many row pairs with several
 * intersection variants, each timed on its own.
 *
 * The intersection is the set operation Peregrine's matching engine is
 * built from (Sec. 4.1: candidates of a pattern vertex are the
 * intersection of its matched neighbours' adjacency lists; Sec. 5.1:
 * sorted adjacency lists, ranges restricted by binary search).  These
 * kernels measure that operation alone, on rows of a resident CSR, so the
 * variants can be compared per row length; they are not used by the
 * matching path.
 *
 * Conventions: every pointer argument marked "device" is device memory
 * owned by the caller; "host" pointers are caller-owned host memory.  Each
 * call enqueues on hip_stream (NULL = null stream), waits for completion,
 * and returns 0, or a negative value on a bad argument (-1) or a HIP error
 * (-3); rb_last_error() then describes it.  Nothing here allocates device
 * memory.
 */
#ifndef ROWBENCH_H
#define ROWBENCH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Read n_words 32-bit words of buf (device, 16-byte aligned, n_words a
 * multiple of 4) reps times with 16-byte loads from every lane of a full
 * grid, and report the mean time of one pass (ms, host) and the wrapping
 * sum of all words read (checksum, host; it keeps the loads live).  acc:
 * one device uint64 the kernel accumulates into.  The achievable read
 * bandwidth is 4 n_words / ms_per_pass. */
int rb_stream_read(const void *buf, int64_t n_words, int32_t reps, uint64_t *acc, double *ms_per_pass,
                   uint64_t *checksum, void *hip_stream);

/* Overwrite buf (device, n_words 32-bit words) with a value: run between
 * timed launches so rows are read from HBM, not from L2 or the
 * last-level cache. */
int rb_flush(void *buf, int64_t n_words, void *hip_stream);

/* Intersection variants (all give the same counts):
 *   RB_BINARY     64 pairs per wavefront; every lane takes elements of the
 *                 shorter row (across the batch's pairs, laid end to end)
 *                 and binary-searches the longer row in global memory
 *   RB_GALLOP     as RB_BINARY, but a lane searches forward from where its
 *                 previous element of the same pair landed (exponential
 *                 then binary search)
 *   RB_MERGEPATH  one wavefront per pair: the merge of the two rows is cut
 *                 into 64 equal diagonals, each lane merges its part
 *   RB_LDS        64 pairs per wavefront; the longer rows are first copied
 *                 into LDS with coalesced loads (when the batch's fit in
 *                 16 KB), then searched there; batches that do not fit
 *                 take RB_BINARY */
#define RB_BINARY 0
#define RB_GALLOP 1
#define RB_MERGEPATH 2
#define RB_LDS 3

/* out[i] = |row(pu[i]) & row(pv[i])| for i < n_pairs, with rows of the CSR
 * (row_ptr int64[n+1], col int32[row_ptr[n]], every row ascending; all
 * device).  pu, pv: device int32[n_pairs] vertex ids in [0, n); out: device
 * uint32[n_pairs].  grid: wavefronts (0 = 2048).  ms: host, receives the
 * kernel's duration from HIP events. */
int rb_intersect(int32_t variant, const int64_t *row_ptr, const int32_t *col, const int32_t *pu,
                 const int32_t *pv, int64_t n_pairs, uint32_t *out, int32_t grid, double *ms, void *hip_stream);

/* Message for the last error on this thread. */
const char *rb_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* ROWBENCH_H */
