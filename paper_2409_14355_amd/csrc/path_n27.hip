// Path-search kernels for 27 users.
#define MPNL_N 27
#include "path_exact.inc"
