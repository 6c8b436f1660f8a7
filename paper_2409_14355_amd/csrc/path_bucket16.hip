// Soft-output path-search kernels for 9..16 users.
#define MPNL_NMAX 16
#include "path_bucket.inc"
