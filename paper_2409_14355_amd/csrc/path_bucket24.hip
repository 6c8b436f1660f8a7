// Soft-output path-search kernels for 17..24 users.
#define MPNL_NMAX 24
#include "path_bucket.inc"
