// Path-search kernels for 23 users.
#define MPNL_N 23
#include "path_exact.inc"
