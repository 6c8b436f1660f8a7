// Host-side helpers of the runtime shared with the serving core.
#pragma once
#include "mpnl.h"

#include <cstddef>

namespace mpnl {

// MPNL_OK, or the error code mpnl_detect() would return for this job's shape.
int validate_job_shape(const mpnl_job &j);

// Device bytes the job holds inside mpnl_detect_batch() (slot state, rotated
// vectors, partial results and its job-table entry).
size_t job_device_bytes(const mpnl_job &j);

// Device ordinal of a context.
int context_device(const mpnl_ctx *ctx);

}  // namespace mpnl
