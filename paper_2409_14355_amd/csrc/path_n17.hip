// Path-search kernels for 17 users.
#define MPNL_N 17
#include "path_exact.inc"
