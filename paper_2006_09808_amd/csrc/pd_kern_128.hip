// Kernels for transform length 128 (row length nx = 128 and/or column length ny = 128).
#include "pd_kern_impl.hpp"
PD_INSTANTIATE(128)
