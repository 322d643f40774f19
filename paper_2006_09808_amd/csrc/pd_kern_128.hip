// Kernels for transform length 128 (row length nx = 128 and/or column length ny = 128),
// and the resident kernel variants of 128x128 slices (workgroups per pair x block size:
// 4 x 256 threads, 8 x 128 threads, 16 x 128 threads).
#include "pd_resident.hpp"
PD_INSTANTIATE(128)
PD_INSTANTIATE_RESIDENT(128, 0, 4, 256)
PD_INSTANTIATE_RESIDENT(128, 1, 8, 128)
PD_INSTANTIATE_RESIDENT(128, 2, 16, 128)
