// Kernels for transform length 256 (row length nx = 256 and/or column length ny = 256),
// and the resident kernel of 256x256 slices (8 workgroups of 512 threads per pair).
#include "pd_resident.hpp"
PD_INSTANTIATE(256)
PD_INSTANTIATE_RESIDENT(256, 8, 512)
