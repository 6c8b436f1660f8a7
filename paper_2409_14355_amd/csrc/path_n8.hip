// Path-search kernels for up to 8 users.
#define MPNL_NMAX 8
#include "path_inst.inc"
