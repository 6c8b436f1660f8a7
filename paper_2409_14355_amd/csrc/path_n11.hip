// Path-search kernels for 11 users.
#define MPNL_N 11
#include "path_exact.inc"
