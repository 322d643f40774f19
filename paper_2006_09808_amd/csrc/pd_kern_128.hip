// Kernels for transform length 128 (row length nx = 128 and/or column length ny = 128),
// and the resident kernel of 128x128 slices (4 workgroups of 256 threads per pair).
#include "pd_resident.hpp"
PD_INSTANTIATE(128)
PD_INSTANTIATE_RESIDENT(128, 4, 256)
