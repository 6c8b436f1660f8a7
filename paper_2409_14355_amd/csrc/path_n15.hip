// Path-search kernels for 15 users.
#define MPNL_N 15
#include "path_exact.inc"
