// Kernels for transform length 128 (row length nx = 128 and/or column length ny = 128),
// and the resident kernel variants of 128x128 slices (workgroups per pair x block size,
// FFT pass plan: 4 x 256, 8 x 128 and 16 x 128 on 16 x 8; 16 x 128 and 8 x 256 on 8 x 4 x 4).
#include "pd_resident.hpp"
PD_INSTANTIATE(128)
PD_INSTANTIATE_RESIDENT(128, 0, 4, 256, 0)
PD_INSTANTIATE_RESIDENT(128, 1, 8, 128, 0)
PD_INSTANTIATE_RESIDENT(128, 2, 16, 128, 0)
PD_INSTANTIATE_RESIDENT(128, 3, 16, 128, 2)
PD_INSTANTIATE_RESIDENT(128, 4, 8, 256, 2)
