/*
 * amped_diag.h -- diagnostic entry point of the load-balance build of the
 * sparse MTTKRP library (built as libamped_qstats.so with AMPED_QUEUE_STATS=1;
 * the production libamped.so does not export it).
 *
 * The paper reports how evenly its load-balancing scheme spreads the compute
 * over its GPUs (Sec. 5.5, Workload Distribution among GPUs).  On one GPU the
 * same question is how evenly the work queue (the dynamic partition-to-SM
 * mapping of Sec. 4.2) spreads the chunks over the compute units.  In this
 * build every wave of the MTTKRP-shaped kernels records its share.
 */
#ifndef AMPED_DIAG_H
#define AMPED_DIAG_H

#include <stdint.h>

#include "amped.h"

#ifdef __cplusplus
extern "C" {
#endif

/*
 * Records of the last amped_mttkrp / amped_mttkrp_bf16 / amped_cp_grad /
 * amped_cp_loss kernel launch in this process (synchronises the device first).
 * One record per wave of the persistent grid, in the order
 * (block, wave within block), each 4 uint64 words:
 *   [0] chunks the wave took from the work queue
 *   [1] nonzeros in those chunks
 *   [2] wall-clock time of its first pop (0 if it took none)
 *   [3] wall-clock time at which it exited
 *   records          host, 4 * max_records words, nullable (then only the
 *                    counts are returned)
 *   n_records        host, receives the number of records of that launch
 *   waves_per_block  host, receives the waves per block of that launch
 *   clock_hz         host, receives the wall-clock rate of the time stamps
 * Errors: INVALID for a NULL count output; HIP if the copy fails.
 */
amped_status amped_queue_stats(uint64_t *records, int64_t max_records, int64_t *n_records,
                               int32_t *waves_per_block, double *clock_hz);

#ifdef __cplusplus
}
#endif

#endif /* AMPED_DIAG_H */
