// Kernels for transform length 32 (row length nx = 32 and/or column length ny = 32).
#include "pd_kern_impl.hpp"
PD_INSTANTIATE(32)
