// Kernels for transform length 64 (row length nx = 64 and/or column length ny = 64),
// and the resident kernel of 64x64 slices (2 workgroups of 256 threads per pair).
#include "pd_resident.hpp"
PD_INSTANTIATE(64)
PD_INSTANTIATE_RESIDENT(64, 2, 256)
