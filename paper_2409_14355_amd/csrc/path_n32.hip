// Path-search kernels for up to 32 users.
#define MPNL_NMAX 32
#include "path_inst.inc"
