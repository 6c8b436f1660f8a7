// Path-search kernels for 6 users.
#define MPNL_N 6
#include "path_exact.inc"
