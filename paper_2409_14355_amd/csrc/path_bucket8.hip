// Soft-output path-search kernels for 1..8 users.
#define MPNL_NMAX 8
#include "path_bucket.inc"
