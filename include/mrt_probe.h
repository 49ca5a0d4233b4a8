/*
 * mrt_probe.h -- data-movement probes that measure the practical HBM
 * ceiling of the lattice step on the GPU (no lattice Boltzmann arithmetic).
 *
 * One lattice update moves 19 population values in and 19 out (Eq. (5):
 * pull streaming between two arrays), so the step is bound by HBM bandwidth.
 * These kernels move the same bytes with nothing else to do, in three
 * patterns, and give the rates against which the step kernels are judged:
 *   - a flat copy of one contiguous buffer;
 *   - 19 direction planes streamed element by element (the step's reads and
 *     writes without shifts, seams, halo or arithmetic);
 *   - the same 19 planes marched by tiles through z in the order the step
 *     kernels use (one block per tile column, plane after plane).
 *
 * Conventions: device pointers owned by the caller, 256-byte aligned, source
 * and destination distinct and not overlapping; launches are asynchronous on
 * hip_stream (NULL = default stream).  streaming_stores != 0 stores with the
 * non-temporal policy.  Returns LBM_OK, or LBM_ERR_INVALID_ARG (message in
 * lbm_probe_last_error) before any launch.
 */
#ifndef MRT_PROBE_H
#define MRT_PROBE_H

#include <stddef.h>
#include <stdint.h>

#include "mrt_lbm.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Copy `bytes` (a multiple of 16) from dev_src to dev_dst with 16-byte
 * accesses, `blocks` workgroups of 256 threads (0: 8192). */
lbm_status lbm_probe_copy(const void *dev_src, void *dev_dst, size_t bytes, int32_t streaming_stores,
                          int32_t blocks, void *hip_stream);

/* 19 planes of plane_bytes each (a multiple of group_bytes), back to back:
 * every group of group_bytes (8 or 16) of every plane is read from dev_src
 * and written to the same place in dev_dst; one thread moves the same group
 * of all 19 planes (19 loads, then 19 stores).  blocks as above. */
lbm_status lbm_probe_stream19(const void *dev_src, void *dev_dst, size_t plane_bytes, int32_t group_bytes,
                              int32_t streaming_stores, int32_t blocks, void *hip_stream);

/* The same 19 planes seen as lattices of nx_groups x ny x nz groups of
 * group_bytes (8 or 16), x fastest: one 256-thread block per tile column of
 * tx groups x ty rows x cz planes, marching its planes in z order (each
 * thread moves groups of its column, 19 loads then 19 stores per plane);
 * tiles numbered x-fastest and dealt to the eight XCDs in contiguous ranges,
 * as the step kernels deal theirs.  tx * ty <= 1024. */
lbm_status lbm_probe_march19(const void *dev_src, void *dev_dst, int32_t nx_groups, int32_t ny, int32_t nz,
                             int32_t group_bytes, int32_t tx, int32_t ty, int32_t cz, int32_t streaming_stores,
                             void *hip_stream);

const char *lbm_probe_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MRT_PROBE_H */
