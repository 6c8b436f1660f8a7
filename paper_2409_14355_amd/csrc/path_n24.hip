// Path-search kernels for up to 24 users.
#define MPNL_NMAX 24
#include "path_inst.inc"
