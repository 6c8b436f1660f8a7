// Path-search kernels for up to 16 users.
#define MPNL_NMAX 16
#include "path_inst.inc"
