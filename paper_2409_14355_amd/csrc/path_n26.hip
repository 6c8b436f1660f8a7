// Path-search kernels for 26 users.
#define MPNL_N 26
#include "path_exact.inc"
