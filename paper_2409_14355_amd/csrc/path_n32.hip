// Path-search kernels for 32 users.
#define MPNL_N 32
#include "path_exact.inc"
