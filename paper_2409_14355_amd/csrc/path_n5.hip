// Path-search kernels for 5 users.
#define MPNL_N 5
#include "path_exact.inc"
