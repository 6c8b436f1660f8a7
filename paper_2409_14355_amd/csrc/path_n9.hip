// Path-search kernels for 9 users.
#define MPNL_N 9
#include "path_exact.inc"
