// Kernels for transform length 512 (row length nx = 512 and/or column length ny = 512).
#include "pd_kern_impl.hpp"
PD_INSTANTIATE(512)
