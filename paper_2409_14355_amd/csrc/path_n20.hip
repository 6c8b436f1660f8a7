// Path-search kernels for 20 users.
#define MPNL_N 20
#include "path_exact.inc"
