// pd_resident.hpp - the iteration kept resident on chip for K iterations.
//
// A team of TEAM workgroups owns one slice pair of an NX x NY volume.  For
// the whole launch each workgroup keeps in registers
//   - its RT = NY/TEAM rows of chi (row phase), and
//   - its CT = NX/TEAM columns of Yhat, F delta and D (column phase),
// so the only memory traffic per iteration is the half-transformed field the
// row and column phases hand each other through the exchange buffer.  Each
// iteration is one column phase (forward column FFT, frequency-domain dual
// prox, inverse column FFT) and one row phase (inverse row FFT, soft
// threshold, over-relaxation, forward row FFT) of the PD pseudocode
// (Sec. II-A), with a team barrier after each phase.
//
// The kernel groups the workgroups of one XCD into teams (each workgroup
// reads the XCD it runs on, HW_REG_XCC_ID), so a team's exchange traffic
// stays in that XCD's L2, the coherence point of all its CUs.  Team barriers
// then only need each wave's stores to have reached L2 (s_waitcnt) and the
// exchange loads to skip the CU's L1 (sc1), with no L2 write-back.  If the
// workgroups are not spread evenly over the XCDs, teams are formed from
// workgroup indices instead and use agent-scope release/acquire fences (L2
// write-back and invalidate) for every barrier, which is correct wherever
// the workgroups run.  The launch is an ordinary one sized to the device's
// co-resident capacity (the occupancy calculator's workgroups per CU times
// the CUs), so on an otherwise idle device every workgroup is resident at
// once; a bounded spin turns a barrier that never completes (other work
// holding CUs) into an abort flag that every workgroup sees, so the grid
// always drains, and the host then reruns the requests on the two-launch
// path.
#pragma once

#include "pd_kern_impl.hpp"

namespace pdk {

// Raw buffer access: a per-thread 32-bit byte offset plus a wave-uniform one
// (an SGPR), so the strided exchange-buffer addresses cost no vector
// registers across the iteration loop.  Out-of-range offsets read 0 and drop
// writes (the resource carries the buffer size).
typedef unsigned u32x2_t __attribute__((__vector_size__(2 * sizeof(unsigned))));
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* p, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}
// Exchange loads are device-scope (sc1): they skip the CU's L1, whose lines
// may predate another member's store, and read the L2.
__device__ __forceinline__ cpx<float> buf_ld(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
  return __builtin_bit_cast(cpx<float>, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 16));
}
__device__ __forceinline__ void buf_st(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, cpx<float> v) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2_t, v), r, voff, soff, 0);
}

// Element (s, j + r N/Q) of a pass with radix Q: per-thread part (s, j) and
// the uniform part r.  Rows layout: element n of row s at s*ld + n; columns
// layout: element n of column s at n*ld + s.
template <typename F, int Q, bool COLS, int N, int LD>
struct ExAddr {
  static __device__ __forceinline__ bool voff(int tid, int q, int s0, unsigned& v) {
    int w = tid + q * F::kNT, s, j;
    F::template coords<Q>(w, s, j);
    if constexpr (COLS) v = (unsigned)((j * LD + s0 + s) * 8);
    else v = (unsigned)(((s0 + s) * LD + j) * 8);
    return F::template nbutter<Q>() % F::kNT == 0 || w < F::template nbutter<Q>();
  }
  static constexpr unsigned soff(int r) {
    return COLS ? (unsigned)(r * (N / Q) * LD * 8) : (unsigned)(r * (N / Q) * 8);
  }
};

// The blocked exchange layout of teams whose transforms are all wave-local:
// columns in groups of G, element (y, x) of the [NYD][*] plane at
// ((x / G) NYD + y) G + x mod G.  A column-phase wave transforms exactly one
// group (G columns of N/Q lanes each), so its loads and stores of a pass
// cover (N/Q) G consecutive elements; a row-phase wave holds G rows, and each
// of its accesses covers G x G consecutive elements per group.  Element
// (s, j + r N/Q) of a pass with radix Q: per-thread part (s, j), uniform r.
template <typename F, int Q, bool COLPHASE, int NYD, int G>
struct ExBlk {
  static constexpr int J = F::kN / Q;
  static_assert(J % G == 0 && 64 % G == 0, "groups of whole lane runs");
  static __device__ __forceinline__ bool voff(int tid, int q, int s0, unsigned& v) {
    int w = tid + q * F::kNT, s, j;
    F::template coords<Q>(w, s, j);
    if constexpr (COLPHASE) {
      const int x = s0 + s;
      v = (unsigned)((((x / G) * NYD + j) * G + x % G) * 8);
    } else {
      v = (unsigned)((((j / G) * NYD + s0 + s) * G + j % G) * 8);
    }
    return F::template nbutter<Q>() % F::kNT == 0 || w < F::template nbutter<Q>();
  }
  static constexpr unsigned soff(int r) {
    return COLPHASE ? (unsigned)(r * J * G * 8) : (unsigned)(r * J * NYD * 8);
  }
};

// Exchange loads / stores of a first or last pass's registers under address
// map A (ExAddr or ExBlk).
template <typename A, int NQ, int Q>
__device__ __forceinline__ void ex_load(cpx<float> (&a)[NQ][Q], __amdgpu_buffer_rsrc_t rs, int tid, int s0) {
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    unsigned v;
    if (A::voff(tid, q, s0, v)) {
#pragma unroll
      for (int r = 0; r < Q; ++r) a[q][r] = buf_ld(rs, v, A::soff(r));
    }
  }
}
template <typename A, int NQ, int Q>
__device__ __forceinline__ void ex_store(const cpx<float> (&a)[NQ][Q], __amdgpu_buffer_rsrc_t rs, int tid, int s0) {
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    unsigned v;
    if (A::voff(tid, q, s0, v)) {
#pragma unroll
      for (int r = 0; r < Q; ++r) buf_st(rs, v, A::soff(r), a[q][r]);
    }
  }
}

// Arrive at a team barrier and wait for `target` arrivals in total; thread 0
// only.  Returns false once the spin limit is hit or another workgroup
// aborted.  A spin limit of 0 gives up at once (a host-set test of the
// recovery path).
__device__ __forceinline__ bool arrive_wait(unsigned* cnt, unsigned add, unsigned target, unsigned mask,
                                            unsigned* seen, int* abort_flag, unsigned spin_limit) {
  if (spin_limit == 0) {
    __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return false;
  }
  unsigned v = __hip_atomic_fetch_add(cnt, add, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + add;
  unsigned spins = 0;
  while ((v & mask) < target) {
    __builtin_amdgcn_s_sleep(2);
    if (++spins > spin_limit || __hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
      __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
    v = __hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  *seen = v;
  return true;
}

// Team barrier: every earlier exchange store of every member is visible to
// every later exchange load (sc1) of every member.  `fenced` selects the
// agent-scope protocol (members on different XCDs).  Returns false in all
// threads once any workgroup has aborted.
__device__ __forceinline__ bool team_barrier(unsigned* cnt, unsigned target, int* abort_flag, int* lds_flag,
                                             bool fenced, unsigned spin_limit) {
  // this wave's stores have reached L2 (the compiler may not move memory
  // operations across the signal fences)
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0);
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __syncthreads();
  if (threadIdx.x == 0) {
    if (fenced) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    unsigned seen;
    int ok = arrive_wait(cnt, 1u, target, 0xffffffffu, &seen, abort_flag, spin_limit) ? 1 : 0;
    if (fenced) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    *lds_flag = ok;
  }
  __syncthreads();
  return *lds_flag != 0;
}

// The transform engines of a team member that owns NY/TEAM rows and NX/TEAM
// columns of a slice pair.  Column transforms run on the rows engine (each
// column's butterflies on consecutive lanes of one wave) when that engine is
// wave-local on both axes: then every transform stays inside its wave, and
// the exchange uses the blocked layout (ExBlk) within a launch.  Otherwise
// the column engine (columns across threads, every pass behind a workgroup
// barrier) and the [ny][nx] layout throughout.
template <int NX, int NY, int TEAM, int NT, int PV>
struct TeamAxes {
  static constexpr int RT = NY / TEAM;   // rows per workgroup (row phase)
  static constexpr int CT = NX / TEAM;   // columns per workgroup (column phase)
  using FR = Fft<float, NX, RT, NT, false, PV>;   // PV: FFT pass plan of both axes
  using FCW = Fft<float, NY, CT, NT, false, PV>;
  static constexpr int JC = FCW::kWaveLocal ? NY / FCW::template QF<-1>() : 1;   // lanes per column
  static constexpr int G = 64 / JC;                                               // columns per wave
  static constexpr bool kBLK = NX == NY && FR::kWaveLocal && FCW::kWaveLocal && JC >= 8 && JC % G == 0 &&
                               CT % G == 0;
  using FC = std::conditional_t<kBLK, FCW, Fft<float, NY, CT, NT, true, PV>>;
  // the row transforms of a wave's rows never leave the wave: their passes
  // need no workgroup barrier (the team barriers still order the phases)
  static constexpr bool kWL = FR::kWaveLocal;
};

template <int NX, int NY, int TEAM, int NT, int PV>
struct Resident {
  using AX = TeamAxes<NX, NY, TEAM, NT, PV>;
  static constexpr int RT = AX::RT;
  static constexpr int CT = AX::CT;
  using FR = typename AX::FR;
  using FC = typename AX::FC;
  static constexpr int G = AX::G;
  static constexpr bool kBLK = AX::kBLK;
  static constexpr int LDS = FR::LDS_ELEMS > FC::LDS_ELEMS ? FR::LDS_ELEMS : FC::LDS_ELEMS;
  // row phase: inverse first radix QI (exchange in), inverse last radix QO
  // (chi state; forward first radix)
  static constexpr int QI = FR::template QF<+1>();
  static constexpr int QO = FR::template QL<+1>();
  // column phase: forward first radix QA (exchange in/out), forward last
  // radix QB (dual state)
  static constexpr int QA = FC::template QF<-1>();
  static constexpr int QB = FC::template QL<-1>();
  static constexpr int NQI = FR::template nq<QI>();
  static constexpr int NQO = FR::template nq<QO>();
  static constexpr int NQA = FC::template nq<QA>();
  static constexpr int NQB = FC::template nq<QB>();
  static constexpr bool kWL = AX::kWL;
  // waves per SIMD the register allocation must allow (the launch bound's
  // second argument): two wherever the member's state fits in 256 registers
  // per lane, so that a variant's co-resident capacity does not hinge on the
  // allocator landing one register under the limit; the 192x192 variants and
  // the 8 x 8 x 4 plan at 256x256 need more and run at one wave per SIMD
  static constexpr int kMinWaves = (NX == 192 || (NX == 256 && PV == 1)) ? 1 : 2;
  static constexpr int kTeam = TEAM;
  static constexpr int kThreadsPerGroup = NT;
  // shared memory of one team member, carved from one byte buffer: the FFT
  // staging area, F delta of the member's columns (blocked layout: [column]
  // [row] with rows padded by 16 entries, so the two column runs of a half
  // wave fall on different banks; else [row][column]), the twiddles of the
  // row (NX) and column (NY) transforms, the barrier flag
  static constexpr int DH_LD = NY + 16;
  static constexpr int DH_ELEMS = kBLK ? CT * DH_LD : CT * NY;
  static __device__ __forceinline__ int dhi(int s, int n) {
    if constexpr (kBLK) return s * DH_LD + n;
    else return n * CT + s;
  }
  static constexpr size_t OFF_DH = (size_t)LDS * sizeof(cpx<float>);
  static constexpr size_t OFF_TW = OFF_DH + (size_t)DH_ELEMS * sizeof(cpx<float>);
  static constexpr size_t OFF_FLAG = OFF_TW + (size_t)(NX + NY) * sizeof(cpx<float>);
  static constexpr size_t SMEM = OFF_FLAG + 16;

  static __device__ __forceinline__ void run(unsigned char* smem, const Vol& V, int pair, int m, unsigned* cnt,
                                             bool fenced, int* abort_flag, unsigned spin_limit);
};

// counters: one barrier counter per team slot, then kXcds per-XCD tickets and
// the grid arrival counter, kCounterStride words apart; zeroed before every
// launch.
//
// Team formation.  Every workgroup reads the XCD it runs on and takes a
// ticket among that XCD's workgroups; after one grid-wide arrival all of
// them know whether each XCD received exactly its quota of `quota`
// workgroups (the dispatcher deals them out round robin, from whichever XCD
// is next).  If so, a workgroup is member `ticket - first` of the team of its
// XCD whose ticket range holds its ticket, and every team lives on one XCD;
// otherwise the workgroups fall back to XCD b mod 8 and ticket b / 8 (b the
// workgroup index), with agent-scope fences at every barrier.  Gives the
// workgroup's XCD (or b mod 8) and ticket, and whether barriers must fence;
// false if the launch aborted before any state was touched.
template <int NT>
__device__ __forceinline__ bool form_team(unsigned* counters, int ticket_base, int quota, int force_fenced,
                                          int* abort_flag, unsigned spin_limit, int* xcd_out, int* ticket_out,
                                          bool* fenced_out) {
  __shared__ int s_xcd, s_ticket, s_fenced;
  unsigned* tickets = counters + (size_t)ticket_base * kCounterStride;   // per-XCD tickets, grid counter
  const int tid = threadIdx.x;
  if (tid == 0) {
    const unsigned here = __builtin_amdgcn_s_getreg((3 << 11) | 20);   // HW_REG_XCC_ID, bits [3:0]
    unsigned ticket = 0xffffffffu;
    if (here < (unsigned)kXcds) ticket = __hip_atomic_fetch_add(tickets + here * kCounterStride, 1u,
                                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    unsigned seen = 0;
    int fen = 1;
    if (!arrive_wait(tickets + kXcds * kCounterStride, 1u, gridDim.x, 0xffffffffu, &seen, abort_flag, spin_limit)) {
      fen = -1;
    } else {
      bool balanced = true;
      for (int x = 0; x < kXcds; ++x)
        balanced &= __hip_atomic_load(tickets + x * kCounterStride, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ==
                    (unsigned)quota;
      const int b = (int)blockIdx.x;
      if (balanced && !force_fenced) {
        s_xcd = (int)here;
        s_ticket = (int)ticket;
        fen = 0;
      } else {
        s_xcd = b % kXcds;
        s_ticket = b / kXcds;
        fen = 1;
      }
    }
    s_fenced = fen;
  }
  __syncthreads();
  if (s_fenced < 0) return false;
  *xcd_out = s_xcd;
  *ticket_out = s_ticket;
  *fenced_out = s_fenced != 0;
  return true;
}

// MW: waves per SIMD the register allocation must allow (0: the variant's
// kMinWaves).  A 192x192 variant with MW = 2 spills part of its state to
// scratch but holds twice the pairs of its one-wave twin: the faster choice
// once a step's pairs exceed what one launch of the twin holds.
template <int NX, int NY, int TEAM, int NT, int PV, int MW = 0>
__global__ __launch_bounds__(NT, (MW > 0 ? MW : Resident<NX, NY, TEAM, NT, PV>::kMinWaves)) void k_resident(const Vol* __restrict__ vols, const Range* __restrict__ ranges,
                                                 int nranges, Ctl* __restrict__ ctl, unsigned* __restrict__ counters,
                                                 int* __restrict__ abort_flag, int nteams, int force_fenced,
                                                 unsigned spin_limit) {
  using R = Resident<NX, NY, TEAM, NT, PV>;
  __shared__ __attribute__((aligned(16))) unsigned char smem[R::SMEM];
  // a launch earlier in the same round gave up: this one does nothing (the
  // host restarts every request of the round's resident launches)
  if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
  // one team size: team t = (ticket / TEAM) * 8 + XCD
  const int rounds = (int)gridDim.x / (kXcds * TEAM);
  int xcd, ticket;
  bool fenced;
  if (!form_team<NT>(counters, rounds * kXcds, TEAM * rounds, force_fenced, abort_flag, spin_limit, &xcd, &ticket,
                     &fenced))
    return;                                   // aborted before any state was touched
  const int t = (ticket / TEAM) * kXcds + xcd;
  if (t >= nteams) return;                    // padding team of the last XCD round
  int slot, pair, m;
  find_work_b(ranges, nranges, TEAM, t * TEAM + ticket % TEAM, slot, pair, m);
  const Vol& V = vols[slot];
  if (ctl[slot].stop || V.iters <= 0 || V.check_only) return;   // uniform over the team
  R::run(smem, V, pair, m, counters + (size_t)t * kCounterStride, fenced, abort_flag, spin_limit);
}

// The K iterations of one team member on slice pair `pair` of volume V:
// member m of TEAM, barrier counter cnt.
template <int NX, int NY, int TEAM, int NT, int PV>
__device__ __forceinline__ void Resident<NX, NY, TEAM, NT, PV>::run(unsigned char* smem, const Vol& V, int pair,
                                                                    int m, unsigned* cnt, bool fenced,
                                                                    int* abort_flag, unsigned spin_limit) {
  using R = Resident<NX, NY, TEAM, NT, PV>;
  using T = float;
  cpx<T>* lds = (cpx<T>*)(smem);
  cpx<T>* dh_s = (cpx<T>*)(smem + OFF_DH);
  cpx<T>* tw_s = (cpx<T>*)(smem + OFF_TW);
  int& lds_flag = *(int*)(smem + OFF_FLAG);
  const int tid = threadIdx.x;
  const int iters = V.iters;
  const bool check = V.check_last != 0;
  const bool final_step = V.final_it == iters - 1;

  const size_t plane = (size_t)NX * NY;
  const size_t base = (size_t)pair * plane;
  const int r0 = m * R::RT;
  const int c0 = m * R::CT;
  stage_twiddles(tw_s, gmem((const cpx<T>*)V.twx), NX, tid, NT);
  stage_twiddles(tw_s + NX, gmem((const cpx<T>*)V.twy), NY, tid, NT);
  const cpx<T>* twx = tw_s;
  const cpx<T>* twy = tw_s + NX;
  cpx<T>* __restrict__ ex = gmem((cpx<T>*)V.ex) + base;
  cpx<T>* __restrict__ ex2 = gmem((cpx<T>*)V.ex2) + base;
  cpx<T>* __restrict__ chi_g = gmem((cpx<T>*)V.chi) + base;
  cpx<T>* __restrict__ yh_g = gmem((cpx<T>*)V.yhat) + base;
  const cpx<T>* __restrict__ dh_g = gmem((const cpx<T>*)V.dhat) + base;
  const T* __restrict__ dtab = gmem((const T*)V.dtab);
  const T tau = (T)V.tau, tl = (T)(V.tau * V.lam), theta = (T)V.theta;
  const T sig = (T)V.sigma, inv1ps = (T)(1.0 / (1.0 + V.sigma));
  const T invN = (T)(1.0 / ((double)NX * (double)NY));
  const bool pad_imag = V.half_last && pair == V.P - 1;

  // ---- resident state ----
  cpx<T> chi[R::NQO][R::QO];                 // rows r0.., inverse-last-pass positions
  cpx<T> yh[R::NQB][R::QB];                  // columns c0.., forward-last-pass positions
  T dk[R::NQB][R::QB];
#pragma unroll
  for (int q = 0; q < R::NQO; ++q)
#pragma unroll
    for (int r = 0; r < R::QO; ++r) {
      int s, n;
      if (FR::template pos<R::QO>(tid, q, r, s, n)) chi[q][r] = chi_g[(unsigned)((r0 + s) * NX + n)];
    }
#pragma unroll
  for (int q = 0; q < R::NQB; ++q)
#pragma unroll
    for (int r = 0; r < R::QB; ++r) {
      int s, n;
      if (FC::template pos<R::QB>(tid, q, r, s, n)) {
        const unsigned o = (unsigned)(n * NX + c0 + s);
        yh[q][r] = yh_g[o];
        dh_s[R::dhi(s, n)] = dh_g[o];
        dk[q][r] = dtab[o];
      }
    }

  __syncthreads();   // twiddle tables staged

  // exchange-buffer resources of this pair (the whole [ny][nx] plane)
  const __amdgpu_buffer_rsrc_t rex = buf_rsrc(ex, (unsigned)(plane * sizeof(cpx<T>)));
  const __amdgpu_buffer_rsrc_t rex2 = buf_rsrc(ex2, (unsigned)(plane * sizeof(cpx<T>)));
  using AC = ExAddr<FC, R::QA, true, NY, NX>;    // column phase, forward first / inverse last pass
  using AR = ExAddr<FR, R::QI, false, NX, NX>;   // row phase, inverse first / forward last pass
  // Blocked layout (kBLK) inside a launch; a launch still takes and leaves
  // the exchange in the [ny][nx] layout every other kernel uses.  The field
  // is rewritten in place, so one extra team barrier before the first
  // blocked store (every member has read the [ny][nx] input) and one before
  // the last iteration's [ny][nx] stores (every member has read the blocked
  // field).
  constexpr bool BLK = R::kBLK;
  using ACB = ExBlk<FC, R::QA, true, NY, R::G>;
  using ARB = ExBlk<FR, R::QI, false, NY, R::G>;

  unsigned phase = 0;
  bool ok = true;
  double acc_r[2] = {0.0, 0.0};
  for (int it = 0; it < iters && ok; ++it) {
    const bool last = it == iters - 1;
    // ---------------- column phase ----------------
    {
      cpx<T> a[R::NQA][R::QA];
      cpx<T> b[R::NQB][R::QB];
      if constexpr (BLK) {
        if (it > 0) ex_load<ACB>(a, rex, tid, c0);
        else ex_load<AC>(a, rex, tid, c0);
      } else {
        ex_load<AC>(a, rex, tid, c0);
      }
      FC::template run<-1, BLK>(a, b, lds, twy, tid);
#pragma unroll
      for (int q = 0; q < R::NQB; ++q)
#pragma unroll
        for (int r = 0; r < R::QB; ++r) {
          int s, n;
          if (FC::template pos<R::QB>(tid, q, r, s, n)) {
            T d = dk[q][r];
            cpx<T> y = yh[q][r], e = dh_s[R::dhi(s, n)];
            cpx<T> yn = mk((y.x + sig * (d * b[q][r].x - e.x)) * inv1ps,
                           (y.y + sig * (d * b[q][r].y - e.y)) * inv1ps);
            yh[q][r] = yn;
            T dn = d * invN;
            b[q][r] = mk(dn * yn.x, dn * yn.y);
          }
        }
      FC::template sync_before_reuse<BLK>();
      FC::template run<+1, BLK>(b, a, lds, twy, tid);
      if constexpr (BLK) {
        if (it == 0) {
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
    {
      cpx<T> a[R::NQI][R::QI];
      cpx<T> b[R::NQO][R::QO];
      if constexpr (BLK) ex_load<ARB>(a, rex, tid, r0);
      else ex_load<AR>(a, rex, tid, r0);
      FR::template run<+1, kWL>(a, b, lds, twx, tid);
      const bool do_check = check && last;
#pragma unroll
      for (int q = 0; q < R::NQO; ++q)
#pragma unroll
        for (int r = 0; r < R::QO; ++r) {
          int s, n;
          if (FR::template pos<R::QO>(tid, q, r, s, n)) {
            cpx<T> x0 = chi[q][r];
            cpx<T> u = b[q][r];
            T vx = x0.x - tau * u.x, vy = x0.y - tau * u.y;
            T nx_ = vx - clampv(vx, -tl, tl);
            T ny_ = vy - clampv(vy, -tl, tl);
            if (pad_imag) {
              ny_ = (T)0;
              u.y = (T)0;
            }
            chi[q][r] = mk(nx_, ny_);
            b[q][r] = mk(nx_ + theta * (nx_ - x0.x), ny_ + theta * (ny_ - x0.y));
            if (do_check) {
              acc_r[0] += fabs((double)nx_) + fabs((double)ny_);
              acc_r[1] = fmax(acc_r[1], fmax(fabs((double)u.x), fabs((double)u.y)));
            }
          }
        }
      if (!(last && final_step)) {
        FR::template sync_before_reuse<kWL>();
        FR::template run<-1, kWL>(b, a, lds, twx, tid);
      }
      if (BLK && last && (!final_step || do_check)) {
        ok = team_barrier(cnt, (++phase) * TEAM, abort_flag, &lds_flag, fenced, spin_limit);
        if (!ok) break;
      }
      if (!(last && final_step)) {
        if constexpr (BLK) {
          if (!last) ex_store<ARB>(a, rex, tid, r0);
          else ex_store<AR>(a, rex, tid, r0);
        } else {
          ex_store<AR>(a, rex, tid, r0);
        }
      }
      if (do_check) {
        block_reduce<2, 2, NT>(acc_r, tid);
        if (tid == 0) {
          double* out = gmem(V.part_row) + ((size_t)pair * TEAM + m) * 2;
          out[0] = acc_r[0];
          out[1] = acc_r[1];
        }
        // chi is final for this launch: write it back now and transform it
        // in place for the residual
#pragma unroll
        for (int q = 0; q < R::NQO; ++q)
#pragma unroll
          for (int r = 0; r < R::QO; ++r) {
            int s, n;
            if (FR::template pos<R::QO>(tid, q, r, s, n)) chi_g[(unsigned)((r0 + s) * NX + n)] = chi[q][r];
          }
        FR::template sync_before_reuse<kWL>();
        FR::template run<-1, kWL>(chi, a, lds, twx, tid);
        ex_store<AR>(a, rex2, tid, r0);
      }
    }
    if (!last || check) {
      ok = team_barrier(cnt, (++phase) * TEAM, abort_flag, &lds_flag, fenced, spin_limit);
      if (!ok) break;
    }
  }

  if (ok && check) {
    // residual of F chi against F delta, and the dual's norms, per workgroup
    cpx<T> a[R::NQA][R::QA];
    cpx<T> b[R::NQB][R::QB];
    ex_load<AC>(a, rex2, tid, c0);   // stored in the [ny][nx] layout above
    FC::template run<-1, BLK>(a, b, lds, twy, tid);
    double acc[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < R::NQB; ++q)
#pragma unroll
      for (int r = 0; r < R::QB; ++r) {
        int s, n;
        if (FC::template pos<R::QB>(tid, q, r, s, n)) {
          T d = dk[q][r];
          cpx<T> e = dh_s[R::dhi(s, n)], y = yh[q][r];
          double rx = (double)(d * b[q][r].x - e.x), ry = (double)(d * b[q][r].y - e.y);
          acc[0] += rx * rx + ry * ry;
          acc[1] += (double)y.x * (double)y.x + (double)y.y * (double)y.y;
          acc[2] += (double)y.x * (double)e.x + (double)y.y * (double)e.y;
        }
      }
    block_reduce<3, 0, NT>(acc, tid);
    if (tid == 0) {
      double* out = gmem(V.part_col) + ((size_t)pair * TEAM + m) * 3;
      out[0] = acc[0];
      out[1] = acc[1];
      out[2] = acc[2];
    }
  }

  // a team barrier gave up: the state of this launch's requests is dropped
  // (they restart on the two-launch path), so nothing is written back
  if (!ok) return;
  // ---- write the state back (chi already written on a check) ----
  if (!check) {
#pragma unroll
    for (int q = 0; q < R::NQO; ++q)
#pragma unroll
      for (int r = 0; r < R::QO; ++r) {
        int s, n;
        if (FR::template pos<R::QO>(tid, q, r, s, n)) chi_g[(unsigned)((r0 + s) * NX + n)] = chi[q][r];
      }
  }
#pragma unroll
  for (int q = 0; q < R::NQB; ++q)
#pragma unroll
    for (int r = 0; r < R::QB; ++r) {
      int s, n;
      if (FC::template pos<R::QB>(tid, q, r, s, n)) yh_g[(unsigned)(n * NX + c0 + s)] = yh[q][r];
    }
}

// ---------------------------------------------------------------------------
// One launch over teams of several slice shapes (uneven volumes iterated
// together).  Bodies... is a list of Resident<N, N, TEAM, NT, PV> types with
// one block size NT; a team names the body it runs.  The launch's table (in
// the range array) starts with kXcds + 1 entries whose `first` is the index
// of each XCD's first team (the last entry: the team count), followed by
// the teams as Range{slot, first ticket on its XCD, pair, body}, grouped by
// XCD in ascending ticket order.  Every XCD receives `quota` workgroups; the
// host places the teams so that each XCD's teams fit in its quota.
// ---------------------------------------------------------------------------
template <typename... Bodies>
constexpr size_t max_smem() {
  size_t m = 16;
  ((m = Bodies::SMEM > m ? Bodies::SMEM : m), ...);
  return m;
}
template <int I, typename B, typename... Rest>
__device__ __forceinline__ int body_team(int body) {
  if (body == I) return B::kTeam;
  if constexpr (sizeof...(Rest) > 0) return body_team<I + 1, Rest...>(body);
  else return 0;
}
template <int I, typename B, typename... Rest>
__device__ __forceinline__ void body_run(int body, unsigned char* smem, const Vol& V, int pair, int m, unsigned* cnt,
                                         bool fenced, int* abort_flag, unsigned spin_limit) {
  if (body == I) {
    B::run(smem, V, pair, m, cnt, fenced, abort_flag, spin_limit);
    return;
  }
  if constexpr (sizeof...(Rest) > 0) body_run<I + 1, Rest...>(body, smem, V, pair, m, cnt, fenced, abort_flag, spin_limit);
}

// Two waves per SIMD, as every body reaches alone: the register budget is
// that of the largest body, not of their union.
template <int NT, typename... Bodies>
__global__ __launch_bounds__(NT, 2) void k_resident_multi(const Vol* __restrict__ vols, const Range* __restrict__ table,
                                                       Ctl* __restrict__ ctl, unsigned* __restrict__ counters,
                                                       int* __restrict__ abort_flag, int ticket_base, int quota,
                                                       int force_fenced, unsigned spin_limit) {
  static_assert(((Bodies::kThreadsPerGroup == NT) && ...), "one block size per launch");
  __shared__ __attribute__((aligned(16))) unsigned char smem[max_smem<Bodies...>()];
  if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
  int xcd, ticket;
  bool fenced;
  if (!form_team<NT>(counters, ticket_base, quota, force_fenced, abort_flag, spin_limit, &xcd, &ticket, &fenced))
    return;
  const Range* teams = table + kXcds + 1;
  int lo = table[xcd].first, hi = table[xcd + 1].first - 1;
  if (lo > hi || teams[lo].first > ticket) return;        // no team holds this ticket: padding
  while (lo < hi) {                                        // last team of the XCD starting at or before the ticket
    const int mid = (lo + hi + 1) >> 1;
    if (teams[mid].first <= ticket) lo = mid;
    else hi = mid - 1;
  }
  const Range& T = teams[lo];
  const int m = ticket - T.first;
  if (m >= body_team<0, Bodies...>(T.pad)) return;        // padding after the XCD's last team
  const Vol& V = vols[T.slot];
  if (ctl[T.slot].stop || V.iters <= 0 || V.check_only) return;   // uniform over the team
  body_run<0, Bodies...>(T.pad, smem, V, T.pair0, m, counters + (size_t)lo * kCounterStride, fenced, abort_flag,
                         spin_limit);
}

// Launch of `nteams` teams, rounded up to whole rounds of one team per XCD
// (grid = a multiple of 8 TEAM workgroups; the padding teams exit at once).
// The caller keeps nteams within resident_max_teams, the co-resident
// capacity.
template <int NX, int NY, int TEAM, int NT, int PV, int MW = 0>
hipError_t launch_resident_t(int nteams, const Vol* vols, const Range* ranges, int nranges, Ctl* ctl,
                             unsigned* counters, int* abort_flag, int fenced, unsigned spin_limit, hipStream_t st) {
  const int rounds = (nteams + kXcds - 1) / kXcds;
  const int grid = rounds * kXcds * TEAM;
  hipLaunchKernelGGL((k_resident<NX, NY, TEAM, NT, PV, MW>), dim3(grid), dim3(NT), 0, st, vols, ranges, nranges,
                     ctl, counters, abort_flag, nteams, fenced, spin_limit);
  return hipGetLastError();
}

template <int NX, int NY, int TEAM, int NT, int PV, int MW = 0>
int resident_max_teams_t() {
  int per_cu = 0, dev = 0, ncu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_resident<NX, NY, TEAM, NT, PV, MW>, NT,
                                                   0) != hipSuccess)
    return 0;
  int teams = per_cu * ncu / TEAM;
  return teams - teams % kXcds;
}

}  // namespace pdk

// Defines resident variant V of the square N x N slice shape: its launcher,
// its co-resident team capacity, its team size, block size and FFT pass plan
// (MW: the waves per SIMD its registers must allow, 0 for the default).
#define PD_INSTANTIATE_RESIDENT_MW(N, V, TEAM, NT, PV, MW)                                              \
  namespace pdk {                                                                                        \
  hipError_t launch_resident_##N##_##V(int nteams, const Vol* vols, const Range* ranges, int nranges,    \
                                       Ctl* ctl, unsigned* counters, int* abort_flag, int fenced,        \
                                       unsigned spin_limit, hipStream_t st) {                            \
    return launch_resident_t<N, N, TEAM, NT, PV, MW>(nteams, vols, ranges, nranges, ctl, counters,       \
                                                     abort_flag, fenced, spin_limit, st);                 \
  }                                                                                                      \
  int resident_max_teams_##N##_##V() { return resident_max_teams_t<N, N, TEAM, NT, PV, MW>(); }         \
  int resident_team_##N##_##V() { return TEAM; }                                                        \
  int resident_threads_##N##_##V() { return NT; }                                                       \
  int resident_plan_##N##_##V() { return PV; }                                                          \
  }
#define PD_INSTANTIATE_RESIDENT(N, V, TEAM, NT, PV) PD_INSTANTIATE_RESIDENT_MW(N, V, TEAM, NT, PV, 0)
