/*
 * sslic_profile.h -- per-kernel timing of libsslic.so with HIP events.
 * While enabled on a context, every launch of a kernel class of sslic_run
 * ("seed", "bins", "sweep", "assign_persist", "update", "finalize",
 * "connectivity") and of sslic_run_batch enqueued directly, not from a
 * graph ("sweep_batch", "finalize_batch": one launch per group of images of
 * one kind) is bracketed by a pair of hipEvents recorded on the launch
 * stream.  Same conventions as sslic.h (SSLIC_OK or a negative code,
 * sslic_last_error()).
 */
#ifndef SSLIC_PROFILE_H
#define SSLIC_PROFILE_H

#include "sslic.h"

#ifdef __cplusplus
extern "C" {
#endif

/* enable != 0 starts recording (dropping anything recorded before);
 * enable == 0 stops.  Events are created by the library and reused. */
int sslic_profile_enable(sslic_ctx* ctx, int enable);

/* Total device time (ms) and number of launches of `kernel` recorded since
 * the last enable or read; waits for the recorded events, then forgets them.
 * total_ms, launches: host pointers (either may be NULL). */
int sslic_profile_read(sslic_ctx* ctx, const char* kernel, double* total_ms, int64_t* launches);

#ifdef __cplusplus
}
#endif
#endif /* SSLIC_PROFILE_H */
