// Kernels for transform length 96 (row length nx = 96 and/or column length ny = 96).
#include "pd_kern_impl.hpp"
PD_INSTANTIATE(96)
