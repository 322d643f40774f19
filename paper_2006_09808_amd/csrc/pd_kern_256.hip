// Kernels for transform length 256 (row length nx = 256 and/or column length ny = 256),
// and the resident kernel variants of 256x256 slices (workgroups per pair x block size:
// 8 x 512 threads, 16 x 256 threads, 32 x 128 threads).
#include "pd_resident.hpp"
PD_INSTANTIATE(256)
PD_INSTANTIATE_RESIDENT(256, 0, 8, 512)
PD_INSTANTIATE_RESIDENT(256, 1, 16, 256)
PD_INSTANTIATE_RESIDENT(256, 2, 32, 128)
