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
//
// The model in three dimensions (ROW_TV3_*: D the 3-D dipole kernel, G the
// 3-D forward difference, the z difference divided by the slice thickness
// and zero at the last slice): the image-domain fields keep the pair layout,
// but the 3-D transform needs each slice's row spectrum on its own plane, so
// the exchange buffer holds nz planes and the column kernels run
//   F_y per plane, (F_z, D / (nx ny nz), F_z^-1) on the z view, F_y^-1 per plane
// in place of COL_TV.  The row kernel of pair p reads planes 2p and 2p+1 as
// Z = X'_2p + i X'_2p+1: both are row spectra of real rows, so one inverse
// transform returns the pair (slice 2p in the real, 2p+1 in the imaginary
// part).  After the forward transform of the pair it splits the spectrum by
// the symmetry of real rows, A(k) = (Z(k) + conj Z(-k)) / 2 and
// B(k) = (Z(k) - conj Z(-k)) / 2i, through LDS.  The z difference of slice
// 2p+1 reads the next pair's real part, G*_z of slice 2p the previous pair's
// imaginary part, both completed by the previous launch.
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
  constexpr bool Z3 = MODE == ROW_TV3_DUAL || MODE == ROW_TV3_PRIMAL;
  constexpr bool DUAL = MODE == ROW_TV_DUAL || MODE == ROW_TV3_DUAL;
  // one-radix plans: each row's transform stays inside one wave (the mirror
  // split below keeps its own workgroup barriers)
  constexpr bool WL = F::kWaveLocal;
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
  const size_t plane = (size_t)len * ny;
  const size_t base = (size_t)pair * plane + (size_t)r0 * len;
  auto inb = [&](int s, int n) -> bool {
    if constexpr (EXT == 0) return true;
    else return r0 + s < ny && n < len;
  };
  stage_twiddles(tw_s, gmem((const cpx<T>*)V.twx), F::tw_count(len), tid, kThreads);
  __syncthreads();
  const cpx<T>* tw = tw_s;

  // 3-D: slices 2p and 2p+1 (the second absent for the last pair of odd nz);
  // z differences 2p -> 2p+1 and 2p+1 -> 2p+2 exist while both ends do
  const bool has_b = !Z3 || 2 * pair + 1 < V.nz;
  const bool za_ok = Z3 && has_b;
  const bool zb_ok = Z3 && 2 * pair + 2 < V.nz;
  cpx<T> a[F::template nq<QI>()][QI];
  cpx<T> b[F::template nq<QO>()][QO];
  cpx<T>* __restrict__ ex = gmem((cpx<T>*)V.ex) + (Z3 ? (size_t)(2 * pair) * plane + (size_t)r0 * len : base);
#pragma unroll
  for (int q = 0; q < F::template nq<QI>(); ++q)
#pragma unroll
    for (int r = 0; r < QI; ++r) {
      int s, n;
      if constexpr (EXT != 0) a[q][r] = mk((T)0, (T)0);
      if (F::template pos<QI>(tid, q, r, s, n) && inb(s, n)) {
        const size_t o = (size_t)s * len + n;
        a[q][r] = ex[o];
        if constexpr (Z3) {   // Z = X'_2p + i X'_2p+1
          if (has_b) {
            const cpx<T> xb = ex[o + plane];
            a[q][r] = mk(a[q][r].x - xb.y, a[q][r].y + xb.x);
          }
        }
      }
    }
  F::template run<+1, WL>(a, b, lds, tw, tid, len);

  const T sig = (T)V.sigma;
  const T idx = (T)V.inv_dx, idy = (T)V.inv_dy, idz = (T)V.inv_dz;
  const cpx<T>* __restrict__ msk = gmem((const cpx<T>*)V.msk) + base;
  bool store_ex = true;
  if constexpr (DUAL) {
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
          if constexpr (Z3) {
            cpx<T>* __restrict__ qzp = gmem((cpx<T>*)V.qz) + base;
            const cpx<T> qz0 = qzp[o];
            const T gza = za_ok ? (c0.y - c0.x) * idz : (T)0;
            const T gzb = zb_ok ? (cb[o + (ptrdiff_t)plane].x - c0.y) * idz : (T)0;
            const T vza = qz0.x + sig * m.x * gza;
            const T vzb = qz0.y + sig * m.y * gzb;
            const T sa = fmax((T)1, sqrt(vxa * vxa + vya * vya + vza * vza));
            const T sb = fmax((T)1, sqrt(vxb * vxb + vyb * vyb + vzb * vzb));
            qxp[o] = mk(vxa / sa, vxb / sb);
            qyp[o] = mk(vya / sa, vyb / sb);
            qzp[o] = mk(vza / sa, vzb / sb);
          } else {
            const T sa = fmax((T)1, sqrt(vxa * vxa + vya * vya));
            const T sb = fmax((T)1, sqrt(vxb * vxb + vyb * vyb));
            qxp[o] = mk(vxa / sa, vxb / sb);
            qyp[o] = mk(vya / sa, vyb / sb);
          }
          b[q][r] = mk(w.x * pn.x, w.y * pn.y);
        }
      }
  } else {  // ROW_TV_PRIMAL, ROW_TV3_PRIMAL
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
          if constexpr (Z3) {   // differences 2p -> 2p+1, 2p+1 -> 2p+2 and 2p-1 -> 2p
            const cpx<T>* __restrict__ qzp = gmem((const cpx<T>*)V.qz) + base;
            const cpx<T> qz0 = qzp[o];
            if (za_ok) {
              const T f = m0.x * qz0.x * idz;
              ta -= f;
              tb += f;
            }
            if (zb_ok) tb -= m0.y * qz0.y * idz;
            if (pair >= 1) {
              const cpx<T> mp = msk[o - (ptrdiff_t)plane], qp = qzp[o - (ptrdiff_t)plane];
              ta += mp.y * qp.y * idz;
            }
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
    F::template sync_before_reuse<WL>();
    F::template run<-1, WL>(b, a, lds, tw, tid, len);
    if constexpr (Z3) {
      // split the pair's row spectrum into the two slices' spectra: Z(-k)
      // sits in another lane, so the row goes through LDS
      __syncthreads();
#pragma unroll
      for (int q = 0; q < F::template nq<QI>(); ++q)
#pragma unroll
        for (int r = 0; r < QI; ++r) {
          int s, n;
          if (F::template pos<QI>(tid, q, r, s, n)) lds[F::lidx(s, n)] = a[q][r];
        }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < F::template nq<QI>(); ++q)
#pragma unroll
        for (int r = 0; r < QI; ++r) {
          int s, n;
          if (F::template pos<QI>(tid, q, r, s, n) && inb(s, n)) {
            const cpx<T> z = a[q][r], zm = lds[F::lidx(s, n == 0 ? 0 : len - n)];
            const size_t o = (size_t)s * len + n;
            ex[o] = mk((z.x + zm.x) * (T)0.5, (z.y - zm.y) * (T)0.5);
            if (has_b) ex[o + plane] = mk((z.y + zm.y) * (T)0.5, (zm.x - z.x) * (T)0.5);
          }
        }
    } else {
#pragma unroll
      for (int q = 0; q < F::template nq<QI>(); ++q)
#pragma unroll
        for (int r = 0; r < QI; ++r) {
          int s, n;
          if (F::template pos<QI>(tid, q, r, s, n) && inb(s, n)) ex[(size_t)s * len + n] = a[q][r];
        }
    }
  }
}

}  // namespace pdk
