// Path-search kernels for 1 users.
#define MPNL_N 1
#include "path_exact.inc"
