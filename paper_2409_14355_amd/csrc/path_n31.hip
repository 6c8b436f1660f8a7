// Path-search kernels for 31 users.
#define MPNL_N 31
#include "path_exact.inc"
