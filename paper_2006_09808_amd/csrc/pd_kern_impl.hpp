// pd_kern_impl.hpp - the two kernels of one primal-dual iteration and their
// set-up / check variants, templated on precision and transform length.
// Included by one pd_kern_<N>.hip translation unit per transform length.
//
// One iteration of the PD pseudocode (Sec. II-A) on a slice pair z = a + i b
// runs as two launches, with the dual kept in the frequency domain:
//
//  column kernel (length ny transforms over column strips):
//     Xhat = F_y X'                       X' = row transform of chibar_n
//     Yhat <- (Yhat + sigma (D Xhat - F delta)) / (1 + sigma)     dual prox
//     X'   <- F_y^-1 (D Yhat / (nx ny))                          (A y, column half)
//  row kernel (length nx transforms over rows):
//     u      = F_x^-1 X'                  u = A y_{n+1}
//     chi'   = soft(chi - tau u, tau lam) primal prox
//     chibar = chi' + theta (chi' - chi)  over-relaxation
//     X'     = F_x chibar                 row half of the next forward FFT
//
// Because F is linear and D is real, F y_n equals the frequency-domain dual
// by induction from y_0 = 0, so each iteration needs one forward and one
// inverse 2-D FFT instead of the image-domain form's two of each.
#pragma once

#include "pd_fft.hpp"
#include "pd_internal.hpp"

namespace pdk {

template <typename T>
__device__ __forceinline__ T clampv(T v, T lo, T hi) {
  return v < lo ? lo : (v > hi ? hi : v);
}

// Block-wide reduction of NV doubles over NT threads (sum, or max for entries
// with MAXMASK bit set); fixed tree, so the result is deterministic.  Result
// valid in thread 0.  Uses its own LDS.
template <int NV, int MAXMASK, int NT = kThreads>
__device__ __forceinline__ void block_reduce(double (&v)[NV], int tid) {
  static_assert(NT % 64 == 0, "whole waves");
  __shared__ double red[NV][NT / 64];
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    double x = v[i];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      double o = __shfl_down(x, off, 64);
      x = ((MAXMASK >> i) & 1) ? fmax(x, o) : x + o;
    }
    if ((tid & 63) == 0) red[i][tid >> 6] = x;
  }
  __syncthreads();
  if (tid == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      double x = red[i][0];
#pragma unroll
      for (int w = 1; w < NT / 64; ++w) x = ((MAXMASK >> i) & 1) ? fmax(x, red[i][w]) : x + red[i][w];
      v[i] = x;
    }
  }
}

// ---------------------------------------------------------------------------
// Column kernel: strips of S columns, transforms of length NY.
// EXT = 0: nx is a multiple of S and the columns have length NY.
// EXT = 1: as 0, but the last strip may be partial (columns >= nx skipped).
// EXT = 2: columns of any length ny <= (NY + 1) / 2 through the Bluestein
//          engine on length-NY transforms; the last strip may be partial.
// ---------------------------------------------------------------------------
template <typename T, int NY, int S, int MODE, int EXT, int PV = 0>
__global__ __launch_bounds__(kThreads) void k_col(const Vol* __restrict__ vols,
                                                  const Range* __restrict__ ranges, int nranges,
                                                  Ctl* __restrict__ ctl, int groups, int it) {
  using F = AxisFft<T, NY, S, kThreads, true, EXT, PV>;
  constexpr int QA = F::template QF<-1>();  // forward first radix == inverse last radix
  constexpr int QB = F::template QL<-1>();  // forward last radix == inverse first radix
  __shared__ cpx<T> lds[F::LDS_ELEMS];
  __shared__ cpx<T> tw_s[F::TW_MAX];

  const int tid = threadIdx.x;
  int slot, pair, g;
  find_work(ranges, nranges, groups, slot, pair, g);
  const Vol& V = vols[slot];
  if constexpr (MODE == COL_ITER) {
    if (ctl[slot].stop || it >= V.iters || V.check_only) return;
  } else if constexpr (MODE == COL_CHECK) {
    if (ctl[slot].stop || it != V.iters - 1 || !V.check_last) return;
  } else if constexpr (MODE == COL_TV) {
    if (ctl[slot].stop || it >= V.iters) return;
  } else if constexpr (MODE == COL_FWD || MODE == COL_INV) {
    if (it >= 0 && (ctl[slot].stop || it >= V.iters || V.check_only)) return;
  } else if constexpr (MODE == COL_FWD_CHK) {
    if (ctl[slot].stop || it != V.iters - 1 || !V.check_last) return;
  }
  const int nx = V.nx;
  const int len = EXT == 2 ? V.ny : NY;     // true column length
  const int c0 = g * S;
  const size_t base = (size_t)pair * (size_t)nx * len;
  // element (s, n) of the strip exists (always, for EXT == 0)
  auto inb = [&](int s, int n) -> bool {
    if constexpr (EXT == 0) return true;
    else return c0 + s < nx && n < len;
  };
  stage_twiddles(tw_s, gmem((const cpx<T>*)V.twy), F::tw_count(len), tid, kThreads);
  __syncthreads();
  const cpx<T>* tw = tw_s;
  const cpx<T>* __restrict__ src =
      gmem((const cpx<T>*)(MODE == COL_CHECK || MODE == COL_FWD_CHK ? V.ex2 : V.ex)) + base + c0;

  cpx<T> a[F::template nq<QA>()][QA];
  cpx<T> b[F::template nq<QB>()][QB];
  if constexpr (MODE == COL_INV) {
    // inverse column transform alone, in place: input in the inverse's
    // first-pass layout (QB), output in its last-pass layout (QA)
#pragma unroll
    for (int q = 0; q < F::template nq<QB>(); ++q)
#pragma unroll
      for (int r = 0; r < QB; ++r) {
        int s, n;
        if constexpr (EXT != 0) b[q][r] = mk((T)0, (T)0);
        if (F::template pos<QB>(tid, q, r, s, n) && inb(s, n)) b[q][r] = src[(size_t)n * nx + s];
      }
    F::template run<+1>(b, a, lds, tw, tid, len);
    cpx<T>* dst = gmem((cpx<T>*)V.ex) + base + c0;
#pragma unroll
    for (int q = 0; q < F::template nq<QA>(); ++q)
#pragma unroll
      for (int r = 0; r < QA; ++r) {
        int s, n;
        if (F::template pos<QA>(tid, q, r, s, n) && inb(s, n)) dst[(size_t)n * nx + s] = a[q][r];
      }
    return;
  }
#pragma unroll
  for (int q = 0; q < F::template nq<QA>(); ++q)
#pragma unroll
    for (int r = 0; r < QA; ++r) {
      int s, n;
      if constexpr (EXT != 0) a[q][r] = mk((T)0, (T)0);
      if (F::template pos<QA>(tid, q, r, s, n) && inb(s, n)) a[q][r] = src[(size_t)n * nx + s];
    }
  // COL_ITER: the dual prox's operands (Yhat, F delta, D) do not depend on
  // the transform, so they are loaded before it and their latency overlaps
  // the FFT's LDS passes instead of following them.  Not for transforms
  // longer than 512 points or Bluestein transforms: there the extra
  // registers leave one wave per SIMD, which costs more than the overlap
  // gains.
  constexpr int NQB = F::template nq<QB>();
  constexpr bool kPre = MODE == COL_ITER && NY <= 512 && EXT != 2;
  cpx<T> yv[kPre ? NQB : 1][kPre ? QB : 1], ev[kPre ? NQB : 1][kPre ? QB : 1];
  T dv[kPre ? NQB : 1][kPre ? QB : 1];
  if constexpr (kPre) {
    const cpx<T>* __restrict__ yh = gmem((const cpx<T>*)V.yhat) + base + c0;
    const cpx<T>* __restrict__ dh = gmem((const cpx<T>*)V.dhat) + base + c0;
    const T* __restrict__ dt = gmem((const T*)V.dtab) + c0;
#pragma unroll
    for (int q = 0; q < NQB; ++q)
#pragma unroll
      for (int r = 0; r < QB; ++r) {
        int s, n;
        yv[q][r] = ev[q][r] = mk((T)0, (T)0);
        dv[q][r] = (T)0;
        if (F::template pos<QB>(tid, q, r, s, n) && inb(s, n)) {
          const size_t o = (size_t)n * nx + s;
          yv[q][r] = yh[o];
          ev[q][r] = dh[o];
          dv[q][r] = dt[o];
        }
      }
  }
  F::template run<-1>(a, b, lds, tw, tid, len);
  if constexpr (MODE == COL_FWD || MODE == COL_FWD_CHK) {
    // forward column transform alone, in place
    cpx<T>* dst = gmem((cpx<T>*)(MODE == COL_FWD_CHK ? V.ex2 : V.ex)) + base + c0;
#pragma unroll
    for (int q = 0; q < F::template nq<QB>(); ++q)
#pragma unroll
      for (int r = 0; r < QB; ++r) {
        int s, n;
        if (F::template pos<QB>(tid, q, r, s, n) && inb(s, n)) dst[(size_t)n * nx + s] = b[q][r];
      }
    return;
  }

  const T* __restrict__ dtab = gmem((const T*)V.dtab) + c0;
  if constexpr (MODE == COL_SETUP) {
    cpx<T>* dh = gmem((cpx<T>*)V.dhat) + base + c0;
#pragma unroll
    for (int q = 0; q < F::template nq<QB>(); ++q)
#pragma unroll
      for (int r = 0; r < QB; ++r) {
        int s, n;
        if (F::template pos<QB>(tid, q, r, s, n) && inb(s, n)) dh[(size_t)n * nx + s] = b[q][r];
      }
    return;
  } else if constexpr (MODE == COL_CHECK) {
    const cpx<T>* __restrict__ dh = gmem((const cpx<T>*)V.dhat) + base + c0;
    const cpx<T>* __restrict__ yh = gmem((const cpx<T>*)V.yhat) + base + c0;
    double acc[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < F::template nq<QB>(); ++q)
#pragma unroll
      for (int r = 0; r < QB; ++r) {
        int s, n;
        if (F::template pos<QB>(tid, q, r, s, n) && inb(s, n)) {
          size_t o = (size_t)n * nx + s;
          T d = dtab[(size_t)n * nx + s];
          cpx<T> e = dh[o], y = yh[o];
          double rx = (double)(d * b[q][r].x - e.x), ry = (double)(d * b[q][r].y - e.y);
          acc[0] += rx * rx + ry * ry;
          acc[1] += (double)y.x * (double)y.x + (double)y.y * (double)y.y;
          acc[2] += (double)y.x * (double)e.x + (double)y.y * (double)e.y;
        }
      }
    block_reduce<3, 0>(acc, tid);
    if (tid == 0) {
      double* out = gmem(V.part_col) + ((size_t)pair * groups + g) * 3;
      out[0] = acc[0];
      out[1] = acc[1];
      out[2] = acc[2];
    }
    return;
  } else {
    const T invN = (T)(1.0 / ((double)nx * (double)len));
    if constexpr (MODE == COL_ITER) {
      const T sig = (T)V.sigma;
      const T inv1ps = (T)(1.0 / (1.0 + V.sigma));
      cpx<T>* __restrict__ yh = gmem((cpx<T>*)V.yhat) + base + c0;
#pragma unroll
      for (int q = 0; q < F::template nq<QB>(); ++q)
#pragma unroll
        for (int r = 0; r < QB; ++r) {
          int s, n;
          if (F::template pos<QB>(tid, q, r, s, n) && inb(s, n)) {
            size_t o = (size_t)n * nx + s;
            T d;
            cpx<T> y, e;
            if constexpr (kPre) {
              d = dv[q][r];
              y = yv[q][r];
              e = ev[q][r];
            } else {
              d = dtab[o];
              y = yh[o];
              e = gmem((const cpx<T>*)V.dhat)[base + c0 + o];
            }
            cpx<T> yn = mk((y.x + sig * (d * b[q][r].x - e.x)) * inv1ps,
                           (y.y + sig * (d * b[q][r].y - e.y)) * inv1ps);
            yh[o] = yn;
            T dn = d * invN;
            b[q][r] = mk(dn * yn.x, dn * yn.y);
          }
        }
    } else {  // COL_APPLY, COL_TV: multiply by D / (nx ny)
#pragma unroll
      for (int q = 0; q < F::template nq<QB>(); ++q)
#pragma unroll
        for (int r = 0; r < QB; ++r) {
          int s, n;
          if (F::template pos<QB>(tid, q, r, s, n) && inb(s, n)) {
            T dn = dtab[(size_t)n * nx + s] * invN;
            b[q][r] = mk(dn * b[q][r].x, dn * b[q][r].y);
          }
        }
    }
    F::sync_before_reuse();
    F::template run<+1>(b, a, lds, tw, tid, len);
    cpx<T>* dst = gmem((cpx<T>*)V.ex) + base + c0;
#pragma unroll
    for (int q = 0; q < F::template nq<QA>(); ++q)
#pragma unroll
      for (int r = 0; r < QA; ++r) {
        int s, n;
        if (F::template pos<QA>(tid, q, r, s, n) && inb(s, n)) dst[(size_t)n * nx + s] = a[q][r];
      }
  }
}

// ---------------------------------------------------------------------------
// Row kernel: S rows per workgroup, transforms of length NX.
// ---------------------------------------------------------------------------
// EXT as for the column kernel, along rows: 1 = the last row group may be
// partial, 2 = rows of any length nx <= (NX + 1) / 2 through Bluestein.
template <typename T, int NX, int S, int MODE, int EXT, int PV = 0>
__global__ __launch_bounds__(kThreads) void k_row(const Vol* __restrict__ vols,
                                                  const Range* __restrict__ ranges, int nranges,
                                                  Ctl* __restrict__ ctl, int groups, int it) {
  using F = AxisFft<T, NX, S, kThreads, false, EXT, PV>;
  constexpr int QI = F::template QF<+1>();  // inverse first radix == forward last radix
  constexpr int QO = F::template QL<+1>();  // inverse last radix == forward first radix
  // one-radix plans: each row's transform stays inside one wave, so its
  // passes need no workgroup barrier
  constexpr bool WL = F::kWaveLocal;
  __shared__ cpx<T> lds[F::LDS_ELEMS];
  __shared__ cpx<T> tw_s[F::TW_MAX];

  const int tid = threadIdx.x;
  int slot, pair, g;
  find_work(ranges, nranges, groups, slot, pair, g);
  const Vol& V = vols[slot];
  if constexpr (MODE == ROW_ITER) {
    if (ctl[slot].stop || it >= V.iters || V.check_only) return;
  }
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
  // imaginary part held at zero: the padding slice of an odd stack, or every
  // plane of an unpacked (3-D kernel) volume
  const bool pad_imag = V.unpacked || (V.half_last && pair == V.P - 1);
  const size_t plane = (size_t)len * ny;
  const size_t slice0 = (size_t)(V.unpacked ? pair : 2 * pair);   // first caller slice of this plane

  cpx<T> a[F::template nq<QI>()][QI];
  cpx<T> b[F::template nq<QO>()][QO];

  if constexpr (MODE == ROW_FWD_PLANAR) {
    const T* __restrict__ in = gmem((const T*)V.user_in) + slice0 * plane + (size_t)r0 * len;
#pragma unroll
    for (int q = 0; q < F::template nq<QO>(); ++q)
#pragma unroll
      for (int r = 0; r < QO; ++r) {
        int s, n;
        if constexpr (EXT != 0) b[q][r] = mk((T)0, (T)0);
        if (F::template pos<QO>(tid, q, r, s, n) && inb(s, n)) {
          size_t o = (size_t)s * len + n;
          b[q][r] = mk(in[o], pad_imag ? (T)0 : in[plane + o]);
        }
      }
    F::template run<-1, WL>(b, a, lds, tw, tid, len);
    cpx<T>* dst = gmem((cpx<T>*)V.ex) + base;
#pragma unroll
    for (int q = 0; q < F::template nq<QI>(); ++q)
#pragma unroll
      for (int r = 0; r < QI; ++r) {
        int s, n;
        if (F::template pos<QI>(tid, q, r, s, n) && inb(s, n)) dst[(size_t)s * len + n] = a[q][r];
      }
    return;
  } else {
    const cpx<T>* __restrict__ src = gmem((const cpx<T>*)V.ex) + base;
#pragma unroll
    for (int q = 0; q < F::template nq<QI>(); ++q)
#pragma unroll
      for (int r = 0; r < QI; ++r) {
        int s, n;
        if constexpr (EXT != 0) a[q][r] = mk((T)0, (T)0);
        if (F::template pos<QI>(tid, q, r, s, n) && inb(s, n)) a[q][r] = src[(size_t)s * len + n];
      }
    // ROW_ITER: chi_n is loaded before the inverse transform, so its latency
    // overlaps the FFT (not for transforms longer than 512 points or
    // Bluestein transforms, as in the column kernel); c then carries
    // chi_{n+1} for the check transform
    constexpr bool kPre = MODE == ROW_ITER && NX <= 512 && EXT != 2;
    cpx<T> c[MODE == ROW_ITER ? F::template nq<QO>() : 1][MODE == ROW_ITER ? QO : 1];
    if constexpr (MODE == ROW_ITER && !kPre) {
#pragma unroll
      for (int q = 0; q < F::template nq<QO>(); ++q)
#pragma unroll
        for (int r = 0; r < QO; ++r) c[q][r] = mk((T)0, (T)0);
    }
    if constexpr (kPre) {
      const cpx<T>* __restrict__ chi0 = gmem((const cpx<T>*)V.chi) + base;
#pragma unroll
      for (int q = 0; q < F::template nq<QO>(); ++q)
#pragma unroll
        for (int r = 0; r < QO; ++r) {
          int s, n;
          c[q][r] = mk((T)0, (T)0);
          if (F::template pos<QO>(tid, q, r, s, n) && inb(s, n)) c[q][r] = chi0[(size_t)s * len + n];
        }
    }
    F::template run<+1, WL>(a, b, lds, tw, tid, len);

    if constexpr (MODE == ROW_INV_PLANAR) {
      T* __restrict__ out = gmem((T*)V.user_out) + slice0 * plane + (size_t)r0 * len;
#pragma unroll
      for (int q = 0; q < F::template nq<QO>(); ++q)
#pragma unroll
        for (int r = 0; r < QO; ++r) {
          int s, n;
          if (F::template pos<QO>(tid, q, r, s, n) && inb(s, n)) {
            size_t o = (size_t)s * len + n;
            out[o] = b[q][r].x;
            if (!pad_imag) out[plane + o] = b[q][r].y;
          }
        }
      return;
    } else {  // ROW_ITER
      const T tau = (T)V.tau;
      const T tl = (T)(V.tau * V.lam);
      const T theta = (T)V.theta;
      const bool check = V.check_last && it == V.iters - 1;
      const bool last = (it == V.final_it);
      cpx<T>* __restrict__ chi = gmem((cpx<T>*)V.chi) + base;
      double acc[2] = {0.0, 0.0};
#pragma unroll
      for (int q = 0; q < F::template nq<QO>(); ++q)
#pragma unroll
        for (int r = 0; r < QO; ++r) {
          int s, n;
          if (F::template pos<QO>(tid, q, r, s, n) && inb(s, n)) {
            size_t o = (size_t)s * len + n;
            const cpx<T> x0 = kPre ? c[q][r] : chi[o];
            cpx<T> u = b[q][r];
            T vx = x0.x - tau * u.x, vy = x0.y - tau * u.y;
            T nx_ = vx - clampv(vx, -tl, tl);
            T ny_ = vy - clampv(vy, -tl, tl);
            if (pad_imag) {
              ny_ = (T)0;
              u.y = (T)0;
            }
            cpx<T> xn = mk(nx_, ny_);
            chi[o] = xn;
            c[q][r] = xn;
            b[q][r] = mk(nx_ + theta * (nx_ - x0.x), ny_ + theta * (ny_ - x0.y));
            if (check) {
              acc[0] += fabs((double)nx_) + fabs((double)ny_);
              acc[1] = fmax(acc[1], fmax(fabs((double)u.x), fabs((double)u.y)));
            }
          }
        }
      if (check) {
        block_reduce<2, 2>(acc, tid);
        if (tid == 0) {
          double* out = gmem(V.part_row) + ((size_t)pair * groups + g) * 2;
          out[0] = acc[0];
          out[1] = acc[1];
        }
      }
      if (!last) {
        F::template sync_before_reuse<WL>();
        F::template run<-1, WL>(b, a, lds, tw, tid, len);
        cpx<T>* dst = gmem((cpx<T>*)V.ex) + base;
#pragma unroll
        for (int q = 0; q < F::template nq<QI>(); ++q)
#pragma unroll
          for (int r = 0; r < QI; ++r) {
            int s, n;
            if (F::template pos<QI>(tid, q, r, s, n) && inb(s, n)) dst[(size_t)s * len + n] = a[q][r];
          }
      }
      if (check) {
        F::template sync_before_reuse<WL>();
        F::template run<-1, WL>(c, a, lds, tw, tid, len);
        cpx<T>* dst = gmem((cpx<T>*)V.ex2) + base;
#pragma unroll
        for (int q = 0; q < F::template nq<QI>(); ++q)
#pragma unroll
          for (int r = 0; r < QI; ++r) {
            int s, n;
            if (F::template pos<QI>(tid, q, r, s, n) && inb(s, n)) dst[(size_t)s * len + n] = a[q][r];
          }
      }
    }
  }
}

}  // namespace pdk

#include "pd_tv_row.hpp"

namespace pdk {

// ---------------------------------------------------------------------------
// per-length launchers
// ---------------------------------------------------------------------------
template <int N, typename T, int S, int EXT>
hipError_t launch_col_t(int mode, int grid, int groups, const Vol* vols, const Range* ranges, int nranges, Ctl* ctl,
                        int it, hipStream_t st) {
  dim3 gr(grid), bl(kThreads);
  switch (mode) {
    case COL_ITER: hipLaunchKernelGGL((k_col<T, N, S, COL_ITER, EXT>), gr, bl, 0, st, vols, ranges, nranges, ctl, groups, it); break;
    case COL_CHECK: hipLaunchKernelGGL((k_col<T, N, S, COL_CHECK, EXT>), gr, bl, 0, st, vols, ranges, nranges, ctl, groups, it); break;
    case COL_SETUP: hipLaunchKernelGGL((k_col<T, N, S, COL_SETUP, EXT>), gr, bl, 0, st, vols, ranges, nranges, ctl, groups, it); break;
    case COL_APPLY: hipLaunchKernelGGL((k_col<T, N, S, COL_APPLY, EXT>), gr, bl, 0, st, vols, ranges, nranges, ctl, groups, it); break;
    case COL_TV: hipLaunchKernelGGL((k_col<T, N, S, COL_TV, EXT>), gr, bl, 0, st, vols, ranges, nranges, ctl, groups, it); break;
    case COL_FWD: hipLaunchKernelGGL((k_col<T, N, S, COL_FWD, EXT>), gr, bl, 0, st, vols, ranges, nranges, ctl, groups, it); break;
    case COL_INV: hipLaunchKernelGGL((k_col<T, N, S, COL_INV, EXT>), gr, bl, 0, st, vols, ranges, nranges, ctl, groups, it); break;
    case COL_FWD_CHK: hipLaunchKernelGGL((k_col<T, N, S, COL_FWD_CHK, EXT>), gr, bl, 0, st, vols, ranges, nranges, ctl, groups, it); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int N, typename T, int S, int EXT>
hipError_t launch_row_t(int mode, int grid, int groups, const Vol* vols, const Range* ranges, int nranges, Ctl* ctl,
                        int it, hipStream_t st) {
  dim3 gr(grid), bl(kThreads);
  switch (mode) {
    case ROW_ITER: hipLaunchKernelGGL((k_row<T, N, S, ROW_ITER, EXT>), gr, bl, 0, st, vols, ranges, nranges, ctl, groups, it); break;
    case ROW_FWD_PLANAR: hipLaunchKernelGGL((k_row<T, N, S, ROW_FWD_PLANAR, EXT>), gr, bl, 0, st, vols, ranges, nranges, ctl, groups, it); break;
    case ROW_INV_PLANAR: hipLaunchKernelGGL((k_row<T, N, S, ROW_INV_PLANAR, EXT>), gr, bl, 0, st, vols, ranges, nranges, ctl, groups, it); break;
    case ROW_TV_DUAL: hipLaunchKernelGGL((k_row_tv<T, N, S, ROW_TV_DUAL, EXT>), gr, bl, 0, st, vols, ranges, nranges, ctl, groups, it); break;
    case ROW_TV_PRIMAL: hipLaunchKernelGGL((k_row_tv<T, N, S, ROW_TV_PRIMAL, EXT>), gr, bl, 0, st, vols, ranges, nranges, ctl, groups, it); break;
    case ROW_TV3_DUAL: hipLaunchKernelGGL((k_row_tv<T, N, S, ROW_TV3_DUAL, EXT>), gr, bl, 0, st, vols, ranges, nranges, ctl, groups, it); break;
    case ROW_TV3_PRIMAL: hipLaunchKernelGGL((k_row_tv<T, N, S, ROW_TV3_PRIMAL, EXT>), gr, bl, 0, st, vols, ranges, nranges, ctl, groups, it); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// EXT (0, 1, 2) from a runtime value
template <int N, typename T, int S>
hipError_t launch_col_x(int ext, int mode, int grid, int groups, const Vol* vols, const Range* ranges, int nranges,
                        Ctl* ctl, int it, hipStream_t st) {
  switch (ext) {
    case 0: return launch_col_t<N, T, S, 0>(mode, grid, groups, vols, ranges, nranges, ctl, it, st);
    case 1: return launch_col_t<N, T, S, 1>(mode, grid, groups, vols, ranges, nranges, ctl, it, st);
    case 2: return launch_col_t<N, T, S, 2>(mode, grid, groups, vols, ranges, nranges, ctl, it, st);
    default: return hipErrorInvalidValue;
  }
}
template <int N, typename T, int S>
hipError_t launch_row_x(int ext, int mode, int grid, int groups, const Vol* vols, const Range* ranges, int nranges,
                        Ctl* ctl, int it, hipStream_t st) {
  switch (ext) {
    case 0: return launch_row_t<N, T, S, 0>(mode, grid, groups, vols, ranges, nranges, ctl, it, st);
    case 1: return launch_row_t<N, T, S, 1>(mode, grid, groups, vols, ranges, nranges, ctl, it, st);
    case 2: return launch_row_t<N, T, S, 2>(mode, grid, groups, vols, ranges, nranges, ctl, it, st);
    default: return hipErrorInvalidValue;
  }
}

// The iteration and check launches of FP32 whole-tile transforms with pass
// plan PV > 0 (the autotuner's alternatives); every other mode runs the
// default plan (a different plan computes the same DFT).
template <int N, int S, int PV>
hipError_t launch_col_pv(int mode, int grid, int groups, const Vol* vols, const Range* ranges, int nranges, Ctl* ctl,
                         int it, hipStream_t st) {
  dim3 gr(grid), bl(kThreads);
  switch (mode) {
    case COL_ITER: hipLaunchKernelGGL((k_col<float, N, S, COL_ITER, 0, PV>), gr, bl, 0, st, vols, ranges, nranges, ctl, groups, it); break;
    case COL_CHECK: hipLaunchKernelGGL((k_col<float, N, S, COL_CHECK, 0, PV>), gr, bl, 0, st, vols, ranges, nranges, ctl, groups, it); break;
    default: return launch_col_t<N, float, S, 0>(mode, grid, groups, vols, ranges, nranges, ctl, it, st);
  }
  return hipGetLastError();
}
template <int N, int S, int PV>
hipError_t launch_row_pv(int mode, int grid, int groups, const Vol* vols, const Range* ranges, int nranges, Ctl* ctl,
                         int it, hipStream_t st) {
  if (mode != ROW_ITER) return launch_row_t<N, float, S, 0>(mode, grid, groups, vols, ranges, nranges, ctl, it, st);
  hipLaunchKernelGGL((k_row<float, N, S, ROW_ITER, 0, PV>), dim3(grid), dim3(kThreads), 0, st, vols, ranges, nranges,
                     ctl, groups, it);
  return hipGetLastError();
}
// plan index from a runtime value (0 .. PlanCount<N> - 1)
template <int N, int S>
hipError_t launch_col_plan(int plan, int mode, int grid, int groups, const Vol* vols, const Range* ranges,
                           int nranges, Ctl* ctl, int it, hipStream_t st) {
  if constexpr (PlanCount<N>::value > 1)
    if (plan == 1) return launch_col_pv<N, S, 1>(mode, grid, groups, vols, ranges, nranges, ctl, it, st);
  if constexpr (PlanCount<N>::value > 2)
    if (plan == 2) return launch_col_pv<N, S, 2>(mode, grid, groups, vols, ranges, nranges, ctl, it, st);
  if (plan != 0) return hipErrorInvalidValue;
  return launch_col_t<N, float, S, 0>(mode, grid, groups, vols, ranges, nranges, ctl, it, st);
}
template <int N, int S>
hipError_t launch_row_plan(int plan, int mode, int grid, int groups, const Vol* vols, const Range* ranges,
                           int nranges, Ctl* ctl, int it, hipStream_t st) {
  if constexpr (PlanCount<N>::value > 1)
    if (plan == 1) return launch_row_pv<N, S, 1>(mode, grid, groups, vols, ranges, nranges, ctl, it, st);
  if constexpr (PlanCount<N>::value > 2)
    if (plan == 2) return launch_row_pv<N, S, 2>(mode, grid, groups, vols, ranges, nranges, ctl, it, st);
  if (plan != 0) return hipErrorInvalidValue;
  return launch_row_t<N, float, S, 0>(mode, grid, groups, vols, ranges, nranges, ctl, it, st);
}

// rows per row-kernel workgroup for length-N rows (FP32): the largest power
// of two with at most 4096 points per workgroup, clamped to [8, 64]
constexpr int row_s_big(int n) {
  int s = 8;
  while (s < 64 && 2 * s * n <= 4096) s *= 2;
  return s;
}

// widest column strip for length-N columns (FP32): the largest power of two
// with at most 4096 points per workgroup, clamped to [16, 64]; wider than 16
// only for N <= 128 (short transforms, e.g. along z)
constexpr int col_s_wide(int n) {
  int s = 16;
  while (s < 64 && 2 * s * n <= 4096) s *= 2;
  return s;
}

}  // namespace pdk

// Defines launch_col_<N> / launch_row_<N>: transforms of length N, tile
// width `cols` / `rows`, EXT `ext` (0: plain; 1: partial last tile; 2:
// Bluestein transforms of any length <= (N + 1) / 2 on length-N transforms),
// pass plan `plan` (FP32 whole tiles only; 0 elsewhere).  FP32 EXT 0 has two
// tile sizes (three columns wide for N <= 128); every other combination uses
// tiles of 8.
#define PD_INSTANTIATE(N)                                                                         \
  namespace pdk {                                                                                 \
  hipError_t launch_col_##N(int mode, int cols, int grid, int groups, const Vol* vols,            \
                            const Range* ranges, int nranges, Ctl* ctl, int it, int precision,    \
                            int ext, int plan, hipStream_t st) {                                  \
    if (plan < 0 || plan >= PlanCount<N>::value || (plan != 0 && (precision == 1 || ext != 0)))    \
      return hipErrorInvalidValue;                                                                \
    if (precision == 1) {                                                                         \
      if (cols != 8) return hipErrorInvalidValue;                                                 \
      return launch_col_x<N, double, 8>(ext, mode, grid, groups, vols, ranges, nranges, ctl, it, st); \
    }                                                                                             \
    if (ext == 0 && cols == 16 && N <= 512)                                                       \
      return launch_col_plan<N, (N <= 512 ? 16 : 8)>(plan, mode, grid, groups, vols, ranges, nranges, ctl, it, st); \
    constexpr int SW = col_s_wide(N);                                                             \
    if (SW > 16 && ext == 0 && cols == SW)                                                        \
      return launch_col_plan<N, SW>(plan, mode, grid, groups, vols, ranges, nranges, ctl, it, st); \
    if (ext == 0 && cols == 8)                                                                    \
      return launch_col_plan<N, 8>(plan, mode, grid, groups, vols, ranges, nranges, ctl, it, st); \
    if (cols == 8) return launch_col_x<N, float, 8>(ext, mode, grid, groups, vols, ranges, nranges, ctl, it, st); \
    return hipErrorInvalidValue;                                                                  \
  }                                                                                               \
  hipError_t launch_row_##N(int mode, int rows, int grid, int groups, const Vol* vols,            \
                            const Range* ranges, int nranges, Ctl* ctl, int it, int precision,    \
                            int ext, int plan, hipStream_t st) {                                  \
    if (plan < 0 || plan >= PlanCount<N>::value || (plan != 0 && (precision == 1 || ext != 0)))    \
      return hipErrorInvalidValue;                                                                \
    if (precision == 1) {                                                                         \
      if (rows != 8) return hipErrorInvalidValue;                                                 \
      return launch_row_x<N, double, 8>(ext, mode, grid, groups, vols, ranges, nranges, ctl, it, st); \
    }                                                                                             \
    constexpr int SB = row_s_big(N);                                                              \
    if (ext == 0 && rows == SB)                                                                   \
      return launch_row_plan<N, SB>(plan, mode, grid, groups, vols, ranges, nranges, ctl, it, st); \
    if (ext == 0 && rows == 8)                                                                    \
      return launch_row_plan<N, 8>(plan, mode, grid, groups, vols, ranges, nranges, ctl, it, st); \
    if (rows == 8) return launch_row_x<N, float, 8>(ext, mode, grid, groups, vols, ranges, nranges, ctl, it, st); \
    return hipErrorInvalidValue;                                                                  \
  }                                                                                               \
  }
