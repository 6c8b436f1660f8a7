// Path-search kernels for 4 users.
#define MPNL_N 4
#include "path_exact.inc"
