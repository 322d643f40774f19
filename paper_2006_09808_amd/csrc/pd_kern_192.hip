// Kernels for transform length 192 (row length nx = 192 and/or column length ny = 192).
#include "pd_kern_impl.hpp"
PD_INSTANTIATE(192)
