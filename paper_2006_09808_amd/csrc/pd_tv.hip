// pd_tv.hip - admission set-up of a weighted-TV volume (Eq. (1)): pack the
// caller's planar W, M and delta into the pair layout the row kernels read,
// and test the PD step condition (Sec. II-A, pseudocode step 1)
//
//     tau sigma ||K||^2 < 1,   ||K||^2 <= max|W|^2 max|D|^2 + max|M|^2 (4/dx^2 + 4/dy^2),
//
// (+ 4/dz^2 for the model in three dimensions, with D the 3-D kernel), which
// needs the maxima of W and M, known only on the device.
#include "pd_internal.hpp"
#include "pd_fft.hpp"

namespace pdk {

namespace {

template <typename T>
__global__ __launch_bounds__(kThreads) void k_tv_pack(const Vol* __restrict__ vols, Ctl* __restrict__ ctl, int slot) {
  const Vol& V = vols[slot];
  const size_t plane = (size_t)V.nx * V.ny;
  const size_t total = (size_t)V.P * plane;
  const int nz = V.nz;
  const T* __restrict__ uw = (const T*)V.user_w;
  const T* __restrict__ um = (const T*)V.user_m;
  const T* __restrict__ ud = (const T*)V.user_in;
  cpx<T>* __restrict__ wg = (cpx<T>*)V.wgt;
  cpx<T>* __restrict__ mk_ = (cpx<T>*)V.msk;
  cpx<T>* __restrict__ dp = (cpx<T>*)V.dpk;
  double wmax = 0.0, mmax = 0.0;
  int bad = 0;
  for (size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x; i < total; i += (size_t)gridDim.x * kThreads) {
    const size_t p = i / plane, o = i - p * plane;
    const size_t za = (2 * p) * plane + o;
    const bool has_b = (int)(2 * p + 1) < nz;
    const T wa = uw[za], ma = um[za], da = ud[za];
    const T wb = has_b ? uw[za + plane] : (T)0;
    const T mb = has_b ? um[za + plane] : (T)0;
    const T db = has_b ? ud[za + plane] : (T)0;
    bad |= !(isfinite((double)wa) && isfinite((double)wb) && isfinite((double)ma) && isfinite((double)mb) &&
             isfinite((double)da) && isfinite((double)db));
    wmax = fmax(wmax, fmax(fabs((double)wa), fabs((double)wb)));
    mmax = fmax(mmax, fmax(fabs((double)ma), fabs((double)mb)));
    wg[i] = mk(wa, wb);
    mk_[i] = mk(ma, mb);
    dp[i] = mk(da, db);
  }
  // wave maxima, then one atomic per wave (order-independent: max of
  // non-negative doubles is the max of their bit patterns)
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    wmax = fmax(wmax, __shfl_down(wmax, off, 64));
    mmax = fmax(mmax, __shfl_down(mmax, off, 64));
    bad |= __shfl_down(bad, off, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    atomicMax(&ctl[slot].wmax_bits, (unsigned long long)__double_as_longlong(wmax));
    atomicMax(&ctl[slot].mmax_bits, (unsigned long long)__double_as_longlong(mmax));
    if (bad) atomicOr(&ctl[slot].bad_input, 1);
  }
}

__global__ void k_tv_check(const Vol* __restrict__ vols, Ctl* __restrict__ ctl, int slot) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const Vol& V = vols[slot];
  Ctl& C = ctl[slot];
  const double wmax = __longlong_as_double((long long)C.wmax_bits);
  const double mmax = __longlong_as_double((long long)C.mmax_bits);
  const double L2 = wmax * wmax * V.knorm * V.knorm +
                    mmax * mmax * 4.0 * (V.inv_dx * V.inv_dx + V.inv_dy * V.inv_dy + V.inv_dz * V.inv_dz);
  if (C.bad_input) {
    C.status = 1;
    C.stop = 1;
  } else if (!(V.tau * V.sigma * L2 < 1.0)) {
    C.status = 2;
    C.stop = 1;
  }
}

}  // namespace

hipError_t launch_tv_setup(const Vol* vols, Ctl* ctl, int slot, size_t npts, int precision, hipStream_t st) {
  size_t blocks = (npts + kThreads - 1) / kThreads;
  if (blocks > 4096) blocks = 4096;
  if (blocks == 0) blocks = 1;
  if (precision == 1)
    hipLaunchKernelGGL(k_tv_pack<double>, dim3((unsigned)blocks), dim3(kThreads), 0, st, vols, ctl, slot);
  else
    hipLaunchKernelGGL(k_tv_pack<float>, dim3((unsigned)blocks), dim3(kThreads), 0, st, vols, ctl, slot);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_tv_check, dim3(1), dim3(64), 0, st, vols, ctl, slot);
  return hipGetLastError();
}

}  // namespace pdk
