// Kernels for transform length 192 (row length nx = 192 and/or column length ny = 192),
// and the resident kernel variants of 192x192 slices (workgroups per pair x block size:
// 12 x 256 threads, 24 x 128 threads), each at one wave per SIMD (its state in
// registers) and at two (part of it spilled, twice the co-resident pairs).
#include "pd_resident.hpp"
PD_INSTANTIATE(192)
PD_INSTANTIATE_RESIDENT(192, 0, 12, 256, 0)
PD_INSTANTIATE_RESIDENT(192, 1, 24, 128, 0)
PD_INSTANTIATE_RESIDENT_MW(192, 2, 12, 256, 0, 2)
PD_INSTANTIATE_RESIDENT_MW(192, 3, 24, 128, 0, 2)
