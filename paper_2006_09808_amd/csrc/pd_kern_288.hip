// Kernels for transform length 288 = 12 x 24 (rows or columns of 288, and the
// Bluestein transforms of lengths 129..144, whose convolutions need at least
// 2n - 1 <= 287 points).
#include "pd_kern_impl.hpp"
PD_INSTANTIATE(288)
