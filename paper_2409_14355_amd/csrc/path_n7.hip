// Path-search kernels for 7 users.
#define MPNL_N 7
#include "path_exact.inc"
