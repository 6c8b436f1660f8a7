// Path-search kernels for 3 users.
#define MPNL_N 3
#include "path_exact.inc"
