// Path-search kernels for 16 users.
#define MPNL_N 16
#include "path_exact.inc"
