// Kernels for transform length 768 (rows or columns of 768, and the Bluestein
// transforms of lengths 289..384).
#include "pd_kern_impl.hpp"
PD_INSTANTIATE(768)
