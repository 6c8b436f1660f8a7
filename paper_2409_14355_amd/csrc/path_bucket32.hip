// Soft-output path-search kernels for 25..32 users.
#define MPNL_NMAX 32
#include "path_bucket.inc"
