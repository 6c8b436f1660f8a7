// Path-search kernels for 13 users.
#define MPNL_N 13
#include "path_exact.inc"
