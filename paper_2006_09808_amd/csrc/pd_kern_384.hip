// Kernels for transform length 384 (row length nx = 384 and/or column length ny = 384).
#include "pd_kern_impl.hpp"
PD_INSTANTIATE(384)
