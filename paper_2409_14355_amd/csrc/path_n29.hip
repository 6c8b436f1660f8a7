// Path-search kernels for 29 users.
#define MPNL_N 29
#include "path_exact.inc"
