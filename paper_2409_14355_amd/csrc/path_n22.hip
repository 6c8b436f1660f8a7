// Path-search kernels for 22 users.
#define MPNL_N 22
#include "path_exact.inc"
