// Path-search kernels for 2 users.
#define MPNL_N 2
#include "path_exact.inc"
