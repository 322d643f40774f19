// Kernels for transform length 8 (row length nx = 8 and/or column length ny = 8).
#include "pd_kern_impl.hpp"
PD_INSTANTIATE(8)
