// Path-search kernels for 19 users.
#define MPNL_N 19
#include "path_exact.inc"
