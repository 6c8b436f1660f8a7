// Path-search kernels for 12 users.
#define MPNL_N 12
#include "path_exact.inc"
