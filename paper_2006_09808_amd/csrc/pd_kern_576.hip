// Kernels for transform length 576 = 24 x 24 (rows or columns of 576, and the
// Bluestein transforms of lengths 257..288, whose convolutions need at least
// 2n - 1 <= 575 points).
#include "pd_kern_impl.hpp"
PD_INSTANTIATE(576)
