// Kernels for transform length 64 (row length nx = 64 and/or column length ny = 64).
#include "pd_kern_impl.hpp"
PD_INSTANTIATE(64)
