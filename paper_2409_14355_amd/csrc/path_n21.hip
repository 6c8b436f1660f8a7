// Path-search kernels for 21 users.
#define MPNL_N 21
#include "path_exact.inc"
