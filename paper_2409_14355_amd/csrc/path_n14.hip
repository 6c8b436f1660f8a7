// Path-search kernels for 14 users.
#define MPNL_N 14
#include "path_exact.inc"
