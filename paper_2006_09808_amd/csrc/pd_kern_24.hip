// Kernels for transform length 24 (row length nx = 24 and/or column length ny = 24).
#include "pd_kern_impl.hpp"
PD_INSTANTIATE(24)
