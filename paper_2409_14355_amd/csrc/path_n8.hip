// Path-search kernels for 8 users.
#define MPNL_N 8
#include "path_exact.inc"
