// Kernels for transform length 192 (row length nx = 192 and/or column length ny = 192),
// and the resident kernel variants of 192x192 slices (workgroups per pair x block size:
// 12 x 256 threads, 24 x 128 threads).
#include "pd_resident.hpp"
PD_INSTANTIATE(192)
PD_INSTANTIATE_RESIDENT(192, 0, 12, 256, 0)
PD_INSTANTIATE_RESIDENT(192, 1, 24, 128, 0)
