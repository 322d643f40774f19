// Kernels for transform length 192 (row length nx = 192 and/or column length ny = 192),
// and the resident kernel of 192x192 slices (12 workgroups of 256 threads per pair).
#include "pd_resident.hpp"
PD_INSTANTIATE(192)
PD_INSTANTIATE_RESIDENT(192, 12, 256)
