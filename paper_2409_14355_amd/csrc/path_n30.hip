// Path-search kernels for 30 users.
#define MPNL_N 30
#include "path_exact.inc"
