// Kernels for transform length 16 (row length nx = 16 and/or column length ny = 16).
#include "pd_kern_impl.hpp"
PD_INSTANTIATE(16)
