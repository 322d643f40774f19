// Kernels for transform length 48 (row length nx = 48 and/or column length ny = 48).
#include "pd_kern_impl.hpp"
PD_INSTANTIATE(48)
