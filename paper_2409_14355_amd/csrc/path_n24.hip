// Path-search kernels for 24 users.
#define MPNL_N 24
#include "path_exact.inc"
