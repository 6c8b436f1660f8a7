// Path-search kernels for 28 users.
#define MPNL_N 28
#include "path_exact.inc"
