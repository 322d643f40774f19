// pd_resident_tv.hpp - the weighted TV model of Eq. (1) iterated for K
// iterations in one persistent launch.
//
// The two-launch form of the TV model (pd_tv_row.hpp) runs four launches per
// iteration; two of them are the column halves of the transforms that apply
// D (F_y, D / (nx ny), F_y^-1), which move only the exchange field and whose
// time is set by each workgroup's chain of loads, LDS passes and stores
// rather than by their bytes.  Here a team of TEAM workgroups owns one slice
// pair, as in the resident kernel of the L1 model (pd_resident.hpp, whose
// team formation, exchange buffer access and team barrier it uses): member m
// holds the D values of its CT columns in registers for the whole launch and
// does the column halves on the exchange buffer in the L2 of its XCD, and the
// row halves on its RT rows.  Unlike the L1 model the TV model's state (chi,
// chibar, p, q_x, q_y, W, M, delta: seven image-domain fields per slice and
// the exchange) does not fit on chip, so the row phases stream it from and
// to HBM as the two-launch row kernels do, except the mask M: constant and
// read by both row phases, it is staged once per launch in LDS for the
// member's rows and the row above them (the primal phase's G* reads it).
// One iteration:
//
//   column phase  X' <- F_y^-1 (D / (nx ny)) F_y X'      (X' = F_x chibar_n)
//   row phase     u = F_x^-1 X' = D chibar_n
//                 p <- (p + sigma W (u - delta)) / (1 + sigma / lam)
//                 q <- v / max(1, |v|),  v = q + sigma M G chibar_n
//                 X' = F_x (W p)
//   column phase  (as above: X' = F_x^-1 ... gives D W p after the row transform)
//   row phase     u = F_x^-1 X' = D W p_{n+1}
//                 chi' = chi - tau u - tau G* (M q_{n+1})
//                 chibar = chi' + theta (chi' - chi);  X' = F_x chibar
//
// with a team barrier after every phase.  Rows of other members are read
// only across a barrier from their last writer: chibar's row below the
// member's rows (written in the previous primal phase) and q_y's row above
// (written in this iteration's dual phase).  All state loads and stores use
// the exchange buffer's device-scope access (loads skip the CU's L1), so a
// line another CU wrote is never read stale.  The update formulas are the
// two-launch row kernels' (ROW_TV_DUAL / ROW_TV_PRIMAL), point for point.
// On a barrier give-up the launch stops where it is; the host restarts its
// requests from the beginning on the two-launch path.
#pragma once

#include "pd_resident.hpp"

namespace pdk {

// State loads and stores of the row phases, with the exchange buffer's
// device-scope access (loads skip the CU's L1).  (Marking them non-temporal,
// to keep the exchange field in L2 ahead of the streamed state, measured 50%
// slower.)
__device__ __forceinline__ cpx<float> st_ld(__amdgpu_buffer_rsrc_t r, unsigned voff) { return buf_ld(r, voff, 0); }
__device__ __forceinline__ void st_st(__amdgpu_buffer_rsrc_t r, unsigned voff, cpx<float> v) { buf_st(r, voff, 0, v); }

template <int NX, int NY, int TEAM, int NT, int PV>
struct ResidentTv {
  using AX = TeamAxes<NX, NY, TEAM, NT, PV>;
  static constexpr int RT = AX::RT;   // rows per workgroup (row phases)
  static constexpr int CT = AX::CT;   // columns per workgroup (column phases)
  using FR = typename AX::FR;
  using FC = typename AX::FC;
  static constexpr int G = AX::G;
  static constexpr bool kBLK = AX::kBLK;
  static constexpr bool kWL = AX::kWL;
  static constexpr int LDS = FR::LDS_ELEMS > FC::LDS_ELEMS ? FR::LDS_ELEMS : FC::LDS_ELEMS;
  static constexpr int QI = FR::template QF<+1>();
  static constexpr int QO = FR::template QL<+1>();
  static constexpr int QA = FC::template QF<-1>();
  static constexpr int QB = FC::template QL<-1>();
  static constexpr int NQI = FR::template nq<QI>();
  static constexpr int NQO = FR::template nq<QO>();
  static constexpr int NQA = FC::template nq<QA>();
  static constexpr int NQB = FC::template nq<QB>();
  static constexpr int kTeam = TEAM;
  static constexpr int kThreadsPerGroup = NT;
  // shared memory: FFT staging, the twiddles of both axes, M of rows
  // r0 - 1 .. r0 + RT - 1 ([RT + 1][NX], slot 0 the row above), the barrier flag
  static constexpr size_t OFF_TW = (size_t)LDS * sizeof(cpx<float>);
  static constexpr size_t OFF_M = OFF_TW + (size_t)(NX + NY) * sizeof(cpx<float>);
  static constexpr size_t OFF_FLAG = OFF_M + (size_t)(RT + 1) * NX * sizeof(cpx<float>);
  static constexpr size_t SMEM = OFF_FLAG + 16;
  static_assert(NX == NY, "square slices");

  static __device__ __forceinline__ void run(unsigned char* smem, const Vol& V, int pair, int m, unsigned* cnt,
                                             bool fenced, int* abort_flag, unsigned spin_limit);
};

template <int NX, int NY, int TEAM, int NT, int PV>
__global__ __launch_bounds__(NT) void k_resident_tv(const Vol* __restrict__ vols, const Range* __restrict__ ranges,
                                                    int nranges, Ctl* __restrict__ ctl,
                                                    unsigned* __restrict__ counters, int* __restrict__ abort_flag,
                                                    int nteams, int force_fenced, unsigned spin_limit) {
  using R = ResidentTv<NX, NY, TEAM, NT, PV>;
  __shared__ __attribute__((aligned(16))) unsigned char smem[R::SMEM];
  if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
  const int rounds = (int)gridDim.x / (kXcds * TEAM);
  int xcd, ticket;
  bool fenced;
  if (!form_team<NT>(counters, rounds * kXcds, TEAM * rounds, force_fenced, abort_flag, spin_limit, &xcd, &ticket,
                     &fenced))
    return;
  const int t = (ticket / TEAM) * kXcds + xcd;
  if (t >= nteams) return;
  int slot, pair, m;
  find_work_b(ranges, nranges, TEAM, t * TEAM + ticket % TEAM, slot, pair, m);
  const Vol& V = vols[slot];
  if (ctl[slot].stop || V.iters <= 0) return;   // uniform over the team
  R::run(smem, V, pair, m, counters + (size_t)t * kCounterStride, fenced, abort_flag, spin_limit);
}

template <int NX, int NY, int TEAM, int NT, int PV>
__device__ __forceinline__ void ResidentTv<NX, NY, TEAM, NT, PV>::run(unsigned char* smem, const Vol& V, int pair,
                                                                      int m, unsigned* cnt, bool fenced,
                                                                      int* abort_flag, unsigned spin_limit) {
  using R = ResidentTv<NX, NY, TEAM, NT, PV>;
  using T = float;
  cpx<T>* lds = (cpx<T>*)(smem);
  cpx<T>* tw_s = (cpx<T>*)(smem + OFF_TW);
  cpx<T>* m_s = (cpx<T>*)(smem + OFF_M);
  int& lds_flag = *(int*)(smem + OFF_FLAG);
  const int tid = threadIdx.x;
  const int iters = V.iters;

  const size_t plane = (size_t)NX * NY;
  const size_t base = (size_t)pair * plane;
  const unsigned pbytes = (unsigned)(plane * sizeof(cpx<T>));
  const int r0 = m * R::RT;
  const int c0 = m * R::CT;
  stage_twiddles(tw_s, gmem((const cpx<T>*)V.twx), NX, tid, NT);
  stage_twiddles(tw_s + NX, gmem((const cpx<T>*)V.twy), NY, tid, NT);
  const cpx<T>* twx = tw_s;
  const cpx<T>* twy = tw_s + NX;
  // every field of this pair as one [ny][nx] complex plane
  const __amdgpu_buffer_rsrc_t rex = buf_rsrc(gmem((cpx<T>*)V.ex) + base, pbytes);
  const __amdgpu_buffer_rsrc_t rchi = buf_rsrc(gmem((cpx<T>*)V.chi) + base, pbytes);
  const __amdgpu_buffer_rsrc_t rcb = buf_rsrc(gmem((cpx<T>*)V.chibar) + base, pbytes);
  const __amdgpu_buffer_rsrc_t rp = buf_rsrc(gmem((cpx<T>*)V.pdual) + base, pbytes);
  const __amdgpu_buffer_rsrc_t rqx = buf_rsrc(gmem((cpx<T>*)V.qx) + base, pbytes);
  const __amdgpu_buffer_rsrc_t rqy = buf_rsrc(gmem((cpx<T>*)V.qy) + base, pbytes);
  const __amdgpu_buffer_rsrc_t rw = buf_rsrc(gmem((cpx<T>*)V.wgt) + base, pbytes);
  const __amdgpu_buffer_rsrc_t rm = buf_rsrc(gmem((cpx<T>*)V.msk) + base, pbytes);
  const __amdgpu_buffer_rsrc_t rd = buf_rsrc(gmem((cpx<T>*)V.dpk) + base, pbytes);
  const T* __restrict__ dtab = gmem((const T*)V.dtab);

  // D / (nx ny) of the member's columns at the forward-last-pass positions
  const T invN = (T)(1.0 / ((double)NX * (double)NY));
  T dk[R::NQB][R::QB];
#pragma unroll
  for (int q = 0; q < R::NQB; ++q)
#pragma unroll
    for (int r = 0; r < R::QB; ++r) {
      int s, n;
      dk[q][r] = (T)0;
      if (FC::template pos<R::QB>(tid, q, r, s, n)) dk[q][r] = dtab[(unsigned)(n * NX + c0 + s)] * invN;
    }
  // M of rows r0 - 1 .. r0 + RT - 1 (no row above the first member's rows)
  for (int i = tid; i < (R::RT + 1) * NX; i += NT) {
    const int row = r0 - 1 + i / NX;
    if (row >= 0) m_s[i] = st_ld(rm, (unsigned)((row * NX + i % NX) * 8));
  }
  __syncthreads();   // twiddle tables and M staged

  const T sig = (T)V.sigma, damp = (T)(1.0 / (1.0 + V.sigma / V.lam));
  const T tau = (T)V.tau, theta = (T)V.theta;
  const T idx = (T)V.inv_dx, idy = (T)V.inv_dy;
  const bool pad_imag = V.half_last && pair == V.P - 1;
  using AC = ExAddr<FC, R::QA, true, NY, NX>;    // column phase, forward first / inverse last pass
  using AR = ExAddr<FR, R::QI, false, NX, NX>;   // row phase, inverse first / forward last pass
  // Blocked exchange layout inside the launch (as in the L1 model's resident
  // kernel): the first column phase reads the [ny][nx] field and the last row
  // phase writes it, each relayout behind one extra team barrier.
  constexpr bool BLK = R::kBLK;
  constexpr bool WL = R::kWL;
  using ACB = ExBlk<FC, R::QA, true, NY, R::G>;
  using ARB = ExBlk<FR, R::QI, false, NY, R::G>;

  unsigned phase = 0;
  bool ok = true;
  for (int it = 0; it < iters && ok; ++it) {
    for (int half = 0; half < 2 && ok; ++half) {
      // ---------------- column phase: X' <- F_y^-1 (D / (nx ny)) F_y X' ----------------
      {
        cpx<T> a[R::NQA][R::QA];
        cpx<T> b[R::NQB][R::QB];
        const bool first = it == 0 && half == 0;
        if constexpr (BLK) {
          if (!first) ex_load<ACB>(a, rex, tid, c0);
          else ex_load<AC>(a, rex, tid, c0);
        } else {
          ex_load<AC>(a, rex, tid, c0);
        }
        FC::template run<-1, BLK>(a, b, lds, twy, tid);
#pragma unroll
        for (int q = 0; q < R::NQB; ++q)
#pragma unroll
          for (int r = 0; r < R::QB; ++r) b[q][r] = mk(dk[q][r] * b[q][r].x, dk[q][r] * b[q][r].y);
        FC::template sync_before_reuse<BLK>();
        FC::template run<+1, BLK>(b, a, lds, twy, tid);
        if constexpr (BLK) {
          if (first) {
            ok = team_barrier(cnt, (++phase) * TEAM, abort_flag, &lds_flag, fenced, spin_limit);
            if (!ok) break;
          }
          ex_store<ACB>(a, rex, tid, c0);
        } else {
          ex_store<AC>(a, rex, tid, c0);
        }
      }
      ok = team_barrier(cnt, (++phase) * TEAM, abort_flag, &lds_flag, fenced, spin_limit);
      if (!ok) break;
      // ---------------- row phase ----------------
      const bool last_update = half == 1 && it == V.final_it;
      {
        cpx<T> a[R::NQI][R::QI];
        cpx<T> b[R::NQO][R::QO];
        if constexpr (BLK) ex_load<ARB>(a, rex, tid, r0);
        else ex_load<AR>(a, rex, tid, r0);
        FR::template run<+1, WL>(a, b, lds, twx, tid);
        if (half == 0) {
          // dual: u = D chibar_n in b
#pragma unroll
          for (int q = 0; q < R::NQO; ++q)
#pragma unroll
            for (int r = 0; r < R::QO; ++r) {
              int s, n;
              if (FR::template pos<R::QO>(tid, q, r, s, n)) {
                const int row = r0 + s;
                const unsigned o = (unsigned)((row * NX + n) * 8);
                const cpx<T> w = st_ld(rw, o), d = st_ld(rd, o), p0 = st_ld(rp, o), u = b[q][r];
                const cpx<T> pn = mk((p0.x + sig * w.x * (u.x - d.x)) * damp, (p0.y + sig * w.y * (u.y - d.y)) * damp);
                st_st(rp, o, pn);
                // G chibar_n: forward differences, zero at the last column / row
                const cpx<T> c0v = st_ld(rcb, o);
                const cpx<T> cr = n + 1 < NX ? st_ld(rcb, o + 8) : c0v;
                const cpx<T> cd = row + 1 < NY ? st_ld(rcb, o + NX * 8) : c0v;
                const cpx<T> mm = m_s[(s + 1) * NX + n], qx0 = st_ld(rqx, o), qy0 = st_ld(rqy, o);
                const T vxa = qx0.x + sig * mm.x * ((cr.x - c0v.x) * idx);
                const T vya = qy0.x + sig * mm.x * ((cd.x - c0v.x) * idy);
                const T vxb = qx0.y + sig * mm.y * ((cr.y - c0v.y) * idx);
                const T vyb = qy0.y + sig * mm.y * ((cd.y - c0v.y) * idy);
                const T sa = fmax((T)1, sqrt(vxa * vxa + vya * vya));
                const T sb = fmax((T)1, sqrt(vxb * vxb + vyb * vyb));
                st_st(rqx, o, mk(vxa / sa, vxb / sb));
                st_st(rqy, o, mk(vya / sa, vyb / sb));
                b[q][r] = mk(w.x * pn.x, w.y * pn.y);
              }
            }
        } else {
          // primal: u = D W p_{n+1} in b
#pragma unroll
          for (int q = 0; q < R::NQO; ++q)
#pragma unroll
            for (int r = 0; r < R::QO; ++r) {
              int s, n;
              if (FR::template pos<R::QO>(tid, q, r, s, n)) {
                const int row = r0 + s;
                const unsigned o = (unsigned)((row * NX + n) * 8);
                const cpx<T> x0 = st_ld(rchi, o), u = b[q][r];
                // G* (M q): element i takes +(M q)[i-1] and -(M q)[i] per axis
                const cpx<T> m0 = m_s[(s + 1) * NX + n], qx0 = st_ld(rqx, o), qy0 = st_ld(rqy, o);
                T ta = 0, tb = 0;
                if (n + 1 < NX) {
                  ta -= m0.x * qx0.x * idx;
                  tb -= m0.y * qx0.y * idx;
                }
                if (n >= 1) {
                  const cpx<T> ml = m_s[(s + 1) * NX + n - 1], ql = st_ld(rqx, o - 8);
                  ta += ml.x * ql.x * idx;
                  tb += ml.y * ql.y * idx;
                }
                if (row + 1 < NY) {
                  ta -= m0.x * qy0.x * idy;
                  tb -= m0.y * qy0.y * idy;
                }
                if (row >= 1) {
                  const cpx<T> mu = m_s[s * NX + n], qu = st_ld(rqy, o - NX * 8);
                  ta += mu.x * qu.x * idy;
                  tb += mu.y * qu.y * idy;
                }
                const T na = x0.x - tau * u.x - tau * ta;
                const T nb = pad_imag ? (T)0 : x0.y - tau * u.y - tau * tb;
                st_st(rchi, o, mk(na, nb));
                const cpx<T> cbn = mk(na + theta * (na - x0.x), nb + theta * (nb - x0.y));
                st_st(rcb, o, cbn);
                b[q][r] = cbn;
              }
            }
        }
        if (!last_update) {
          FR::template sync_before_reuse<WL>();
          FR::template run<-1, WL>(b, a, lds, twx, tid);
          const bool end = half == 1 && it == iters - 1;   // the launch's last exchange store
          if constexpr (BLK) {
            if (end) {
              ok = team_barrier(cnt, (++phase) * TEAM, abort_flag, &lds_flag, fenced, spin_limit);
              if (!ok) break;
              ex_store<AR>(a, rex, tid, r0);
            } else {
              ex_store<ARB>(a, rex, tid, r0);
            }
          } else {
            ex_store<AR>(a, rex, tid, r0);
          }
        }
      }
      if (!(half == 1 && it == iters - 1)) ok = team_barrier(cnt, (++phase) * TEAM, abort_flag, &lds_flag, fenced,
                                                             spin_limit);
    }
  }
}

template <int NX, int NY, int TEAM, int NT, int PV>
hipError_t launch_resident_tv_t(int nteams, const Vol* vols, const Range* ranges, int nranges, Ctl* ctl,
                                unsigned* counters, int* abort_flag, int fenced, unsigned spin_limit,
                                hipStream_t st) {
  const int rounds = (nteams + kXcds - 1) / kXcds;
  const int grid = rounds * kXcds * TEAM;
  hipLaunchKernelGGL((k_resident_tv<NX, NY, TEAM, NT, PV>), dim3(grid), dim3(NT), 0, st, vols, ranges, nranges,
                     ctl, counters, abort_flag, nteams, fenced, spin_limit);
  return hipGetLastError();
}

template <int NX, int NY, int TEAM, int NT, int PV>
int resident_tv_max_teams_t() {
  int per_cu = 0, dev = 0, ncu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_resident_tv<NX, NY, TEAM, NT, PV>, NT,
                                                   0) != hipSuccess)
    return 0;
  int teams = per_cu * ncu / TEAM;
  return teams - teams % kXcds;
}

}  // namespace pdk

// Defines the TV model's resident variant of the square N x N slice shape.
#define PD_INSTANTIATE_RESIDENT_TV(N, TEAM, NT, PV)                                                      \
  namespace pdk {                                                                                        \
  hipError_t launch_resident_tv_##N(int nteams, const Vol* vols, const Range* ranges, int nranges,       \
                                    Ctl* ctl, unsigned* counters, int* abort_flag, int fenced,           \
                                    unsigned spin_limit, hipStream_t st) {                               \
    return launch_resident_tv_t<N, N, TEAM, NT, PV>(nteams, vols, ranges, nranges, ctl, counters,        \
                                                    abort_flag, fenced, spin_limit, st);                  \
  }                                                                                                      \
  int resident_tv_max_teams_##N() { return resident_tv_max_teams_t<N, N, TEAM, NT, PV>(); }             \
  int resident_tv_team_##N() { return TEAM; }                                                           \
  int resident_tv_threads_##N() { return NT; }                                                          \
  int resident_tv_plan_##N() { return PV; }                                                             \
  }
