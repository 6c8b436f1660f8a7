// Path-search kernels for 18 users.
#define MPNL_N 18
#include "path_exact.inc"
