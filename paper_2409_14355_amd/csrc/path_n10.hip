// Path-search kernels for 10 users.
#define MPNL_N 10
#include "path_exact.inc"
