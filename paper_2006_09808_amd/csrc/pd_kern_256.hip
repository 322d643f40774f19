// Kernels for transform length 256 (row length nx = 256 and/or column length ny = 256).
#include "pd_kern_impl.hpp"
PD_INSTANTIATE(256)
