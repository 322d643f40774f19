// Kernels for transform length 256 (row length nx = 256 and/or column length ny = 256),
// and the resident kernel variants of 256x256 slices (workgroups per pair x block size,
// FFT pass plan: 8 x 512, 16 x 256 and 32 x 128 on 16 x 16; 16 x 256 on 8 x 8 x 4).
#include "pd_resident.hpp"
PD_INSTANTIATE(256)
PD_INSTANTIATE_RESIDENT(256, 0, 8, 512, 0)
PD_INSTANTIATE_RESIDENT(256, 1, 16, 256, 0)
PD_INSTANTIATE_RESIDENT(256, 2, 32, 128, 0)
PD_INSTANTIATE_RESIDENT(256, 3, 16, 256, 1)
