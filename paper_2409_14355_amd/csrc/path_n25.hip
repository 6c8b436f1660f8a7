// Path-search kernels for 25 users.
#define MPNL_N 25
#include "path_exact.inc"
