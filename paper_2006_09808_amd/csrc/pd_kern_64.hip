// Kernels for transform length 64 (row length nx = 64 and/or column length ny = 64),
// and the resident kernel variants of 64x64 slices (workgroups per pair x block size:
// 2 x 256 threads, 4 x 128 threads, 8 x 64 threads).
#include "pd_resident.hpp"
PD_INSTANTIATE(64)
PD_INSTANTIATE_RESIDENT(64, 0, 2, 256, 0)
PD_INSTANTIATE_RESIDENT(64, 1, 4, 128, 0)
PD_INSTANTIATE_RESIDENT(64, 2, 8, 64, 0)
