// pd_tv_row.hpp - row kernels of the weighted TV model of Eq. (1),
//
//     minimise over chi   lam/2 ||W (D chi - delta)||^2 + ||M G chi||_1,
//
// solved by the PD pseudocode of Sec. II-A with K = [W D; M G] (lam on the
// data term; G the in-plane forward difference divided by the voxel size,
// with the last difference along each axis zero; isotropic gradient norm).
// One iteration runs as four launches over the slice pairs of every TV
// volume of one shape, with all duals in the image domain:
//
//   column kernel (COL_TV):  X' <- F_y^-1 (D / (nx ny)) F_y X'
//   ROW_TV_DUAL:    u = F_x^-1 X'  (= D chibar_n)
//                   p <- (p + sigma W (u - delta)) / (1 + sigma / lam)
//                   q <- v / max(1, |v|),   v = q + sigma M G chibar_n
//                   X' = F_x (W p)
//   column kernel (COL_TV)
//   ROW_TV_PRIMAL:  u = F_x^-1 X'  (= D W p_{n+1})
//                   chi'   = chi - tau u - tau G* (M q_{n+1})
//                   chibar = chi' + theta (chi' - chi)
//                   X' = F_x chibar  (first half of the next iteration)
//
// G needs the row below a workgroup's rows and G* the row above: both are
// read from the chibar / q buffers, which the previous launch completed, so
// rows owned by other workgroups are never read while being written.  W, M,
// delta and every dual are real per slice, so the pair packing z = a + i b
// carries them unchanged (the projection is taken per slice: .x for slice
// 2p, .y for slice 2p+1).
#pragma once

#include "pd_fft.hpp"
#include "pd_internal.hpp"

namespace pdk {

// EXT as for the L1 model's row kernel (partial last row group; Bluestein rows).
template <typename T, int NX, int S, int MODE, int EXT>
__global__ __launch_bounds__(kThreads) void k_row_tv(const Vol* __restrict__ vols,
                                                     const Range* __restrict__ ranges, int nranges,
                                                     Ctl* __restrict__ ctl, int groups, int it) {
  using F = AxisFft<T, NX, S, kThreads, false, EXT>;
  constexpr int QI = F::template QF<+1>();  // inverse first radix == forward last radix
  constexpr int QO = F::template QL<+1>();  // inverse last radix == forward first radix
  __shared__ cpx<T> lds[F::LDS_ELEMS];
  __shared__ cpx<T> tw_s[F::TW_MAX];

  const int tid = threadIdx.x;
  int slot, pair, g;
  find_work(ranges, nranges, groups, slot, pair, g);
  const Vol& V = vols[slot];
  if (ctl[slot].stop || it >= V.iters) return;
  const int ny = V.ny;
  const int len = EXT == 2 ? V.nx : NX;     // true row length (and row stride)
  const int r0 = g * S;
  const size_t base = (size_t)pair * (size_t)len * ny + (size_t)r0 * len;
  auto inb = [&](int s, int n) -> bool {
    if constexpr (EXT == 0) return true;
    else return r0 + s < ny && n < len;
  };
  stage_twiddles(tw_s, gmem((const cpx<T>*)V.twx), F::tw_count(len), tid, kThreads);
  __syncthreads();
  const cpx<T>* tw = tw_s;

  cpx<T> a[F::template nq<QI>()][QI];
  cpx<T> b[F::template nq<QO>()][QO];
  cpx<T>* __restrict__ ex = gmem((cpx<T>*)V.ex) + base;
#pragma unroll
  for (int q = 0; q < F::template nq<QI>(); ++q)
#pragma unroll
    for (int r = 0; r < QI; ++r) {
      int s, n;
      if constexpr (EXT != 0) a[q][r] = mk((T)0, (T)0);
      if (F::template pos<QI>(tid, q, r, s, n) && inb(s, n)) a[q][r] = ex[(size_t)s * len + n];
    }
  F::template run<+1>(a, b, lds, tw, tid, len);

  const T sig = (T)V.sigma;
  const T idx = (T)V.inv_dx, idy = (T)V.inv_dy;
  const cpx<T>* __restrict__ msk = gmem((const cpx<T>*)V.msk) + base;
  bool store_ex = true;
  if constexpr (MODE == ROW_TV_DUAL) {
    const T damp = (T)(1.0 / (1.0 + V.sigma / V.lam));
    cpx<T>* __restrict__ pd = gmem((cpx<T>*)V.pdual) + base;
    cpx<T>* __restrict__ qxp = gmem((cpx<T>*)V.qx) + base;
    cpx<T>* __restrict__ qyp = gmem((cpx<T>*)V.qy) + base;
    const cpx<T>* __restrict__ wg = gmem((const cpx<T>*)V.wgt) + base;
    const cpx<T>* __restrict__ dl = gmem((const cpx<T>*)V.dpk) + base;
    const cpx<T>* __restrict__ cb = gmem((const cpx<T>*)V.chibar) + base;
#pragma unroll
    for (int q = 0; q < F::template nq<QO>(); ++q)
#pragma unroll
      for (int r = 0; r < QO; ++r) {
        int s, n;
        if (F::template pos<QO>(tid, q, r, s, n) && inb(s, n)) {
          const ptrdiff_t o = (ptrdiff_t)s * len + n;
          const cpx<T> w = wg[o], d = dl[o], p0 = pd[o], u = b[q][r];
          const cpx<T> pn = mk((p0.x + sig * w.x * (u.x - d.x)) * damp, (p0.y + sig * w.y * (u.y - d.y)) * damp);
          pd[o] = pn;
          // G chibar_n: forward differences, zero at the last column / row
          const cpx<T> c0 = cb[o];
          const cpx<T> cr = n + 1 < len ? cb[o + 1] : c0;
          const cpx<T> cd = r0 + s + 1 < ny ? cb[o + len] : c0;
          const cpx<T> m = msk[o], qx0 = qxp[o], qy0 = qyp[o];
          const T vxa = qx0.x + sig * m.x * ((cr.x - c0.x) * idx);
          const T vya = qy0.x + sig * m.x * ((cd.x - c0.x) * idy);
          const T vxb = qx0.y + sig * m.y * ((cr.y - c0.y) * idx);
          const T vyb = qy0.y + sig * m.y * ((cd.y - c0.y) * idy);
          const T sa = fmax((T)1, sqrt(vxa * vxa + vya * vya));
          const T sb = fmax((T)1, sqrt(vxb * vxb + vyb * vyb));
          qxp[o] = mk(vxa / sa, vxb / sb);
          qyp[o] = mk(vya / sa, vyb / sb);
          b[q][r] = mk(w.x * pn.x, w.y * pn.y);
        }
      }
  } else {  // ROW_TV_PRIMAL
    const T tau = (T)V.tau, theta = (T)V.theta;
    const bool pad_imag = V.half_last && pair == V.P - 1;
    cpx<T>* __restrict__ chi = gmem((cpx<T>*)V.chi) + base;
    cpx<T>* __restrict__ chibar = gmem((cpx<T>*)V.chibar) + base;
    const cpx<T>* __restrict__ qxp = gmem((const cpx<T>*)V.qx) + base;
    const cpx<T>* __restrict__ qyp = gmem((const cpx<T>*)V.qy) + base;
#pragma unroll
    for (int q = 0; q < F::template nq<QO>(); ++q)
#pragma unroll
      for (int r = 0; r < QO; ++r) {
        int s, n;
        if (F::template pos<QO>(tid, q, r, s, n) && inb(s, n)) {
          const ptrdiff_t o = (ptrdiff_t)s * len + n;
          const int row = r0 + s;
          const cpx<T> x0 = chi[o], u = b[q][r];
          // G* (M q): element i takes +(M q)[i-1] and -(M q)[i] per axis,
          // where i-1 and i are differences G computes
          const cpx<T> m0 = msk[o], qx0 = qxp[o], qy0 = qyp[o];
          T ta = 0, tb = 0;
          if (n + 1 < len) {
            ta -= m0.x * qx0.x * idx;
            tb -= m0.y * qx0.y * idx;
          }
          if (n >= 1) {
            const cpx<T> ml = msk[o - 1], ql = qxp[o - 1];
            ta += ml.x * ql.x * idx;
            tb += ml.y * ql.y * idx;
          }
          if (row + 1 < ny) {
            ta -= m0.x * qy0.x * idy;
            tb -= m0.y * qy0.y * idy;
          }
          if (row >= 1) {
            const cpx<T> mu = msk[o - len], qu = qyp[o - len];
            ta += mu.x * qu.x * idy;
            tb += mu.y * qu.y * idy;
          }
          const T na = x0.x - tau * u.x - tau * ta;
          const T nb = pad_imag ? (T)0 : x0.y - tau * u.y - tau * tb;
          chi[o] = mk(na, nb);
          const cpx<T> cbn = mk(na + theta * (na - x0.x), nb + theta * (nb - x0.y));
          chibar[o] = cbn;
          b[q][r] = cbn;
        }
      }
    store_ex = it != V.final_it;
  }
  if (store_ex) {
    F::sync_before_reuse();
    F::template run<-1>(b, a, lds, tw, tid, len);
#pragma unroll
    for (int q = 0; q < F::template nq<QI>(); ++q)
#pragma unroll
      for (int r = 0; r < QI; ++r) {
        int s, n;
        if (F::template pos<QI>(tid, q, r, s, n) && inb(s, n)) ex[(size_t)s * len + n] = a[q][r];
      }
  }
}

}  // namespace pdk
