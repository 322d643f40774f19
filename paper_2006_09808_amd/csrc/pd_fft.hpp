// pd_fft.hpp - register/LDS building blocks of the batched mixed-radix FFT
// used by every transform of the primal-dual iteration (gfx950, wave64).
//
// A length-N transform runs as a sequence of Stockham autosort passes.  A
// pass of radix Q after passes whose radices multiply to p takes, for each
// butterfly j in [0, N/Q), the Q inputs at j + r N/Q, multiplies input r by
// w^(r k) (k = j mod p, w = exp(s 2 pi i / (p Q)), s = -1 forward, +1
// inverse), applies a Q-point DFT in registers and writes output r to
// (j - k) Q + k + r p.  The first pass therefore reads at stride N/Q and the
// last pass writes at stride N/Q, both with consecutive butterflies at
// consecutive addresses, so a transform reads its input from and writes its
// output to global memory in coalesced order and only the passes in between
// go through LDS.  Running the passes of a forward transform in the reverse
// order of the inverse's makes one transform's output registers exactly the
// next transform's input registers, which is how the kernels fuse an inverse
// FFT, a point-wise update and a forward FFT without an LDS round trip.
//
// Small DFTs (2, 3, 4) are written out; larger register DFTs are built as
// A x B Cooley-Tukey products with compile-time twiddles.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <type_traits>
#include <utility>

namespace pdk {

template <typename T>
struct alignas(2 * sizeof(T)) cpx {
  T x, y;
};

template <typename T>
__device__ __forceinline__ cpx<T> mk(T x, T y) {
  cpx<T> r;
  r.x = x;
  r.y = y;
  return r;
}
template <typename T>
__device__ __forceinline__ cpx<T> operator+(cpx<T> a, cpx<T> b) { return mk(a.x + b.x, a.y + b.y); }
template <typename T>
__device__ __forceinline__ cpx<T> operator-(cpx<T> a, cpx<T> b) { return mk(a.x - b.x, a.y - b.y); }
template <typename T>
__device__ __forceinline__ cpx<T> cmul(cpx<T> a, cpx<T> b) {
  return mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
template <typename T>
__device__ __forceinline__ cpx<T> cmulc(cpx<T> a, cpx<T> b) {
  return mk(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
template <typename T>
__device__ __forceinline__ cpx<T> scl(cpx<T> a, T s) { return mk(a.x * s, a.y * s); }
// multiply by DIR * i  (DIR = -1: by -i; DIR = +1: by +i)
template <int DIR, typename T>
__device__ __forceinline__ cpx<T> mul_i(cpx<T> a) {
  if constexpr (DIR < 0) return mk(a.y, -a.x);
  else return mk(-a.y, a.x);
}

// ---------------------------------------------------------------------------
// compile-time trigonometry (Taylor series on a reduced argument)
// ---------------------------------------------------------------------------
constexpr double kPi = 3.14159265358979323846264338327950288;

constexpr double ce_sin_red(double x) {
  double x2 = x * x, term = x, sum = x;
  for (int n = 1; n <= 30; ++n) {
    term *= -x2 / ((2.0 * n) * (2.0 * n + 1.0));
    sum += term;
  }
  return sum;
}
constexpr double ce_cos_red(double x) {
  double x2 = x * x, term = 1.0, sum = 1.0;
  for (int n = 1; n <= 30; ++n) {
    term *= -x2 / ((2.0 * n - 1.0) * (2.0 * n));
    sum += term;
  }
  return sum;
}
// cos / sin of 2 pi m / R, argument reduced to (-pi, pi]
constexpr double ce_cos_frac(int m, int R) {
  m %= R;
  if (m < 0) m += R;
  if (2 * m > R) m -= R;
  return ce_cos_red(2.0 * kPi * m / R);
}
constexpr double ce_sin_frac(int m, int R) {
  m %= R;
  if (m < 0) m += R;
  if (2 * m > R) m -= R;
  return ce_sin_red(2.0 * kPi * m / R);
}

template <int I, int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    static_for<I + 1, N>(f);
  }
}

// a * w^m with w = exp(DIR 2 pi i / R), m and R compile-time
template <int R, int M, int DIR, typename T>
__device__ __forceinline__ cpx<T> twc(cpx<T> a) {
  constexpr int m = ((M % R) + R) % R;
  if constexpr (m == 0) {
    return a;
  } else if constexpr (2 * m == R) {
    return mk(-a.x, -a.y);
  } else if constexpr (4 * m == R) {
    return mul_i<DIR>(a);
  } else if constexpr (4 * m == 3 * R) {
    return mul_i<-DIR>(a);
  } else {
    constexpr T c = (T)ce_cos_frac(m, R);
    constexpr T s = (T)(DIR * ce_sin_frac(m, R));
    return mk(a.x * c - a.y * s, a.x * s + a.y * c);
  }
}

// ---------------------------------------------------------------------------
// register DFTs, natural order in and out, unnormalised
// ---------------------------------------------------------------------------
template <int R, int DIR, typename T>
struct Dft;

template <int A, int B, int DIR, typename T>
__device__ __forceinline__ void dft_ab(cpx<T>* x);

template <int DIR, typename T>
struct Dft<1, DIR, T> {
  static __device__ __forceinline__ void run(cpx<T>*) {}
};
template <int DIR, typename T>
struct Dft<2, DIR, T> {
  static __device__ __forceinline__ void run(cpx<T>* x) {
    cpx<T> a = x[0], b = x[1];
    x[0] = a + b;
    x[1] = a - b;
  }
};
template <int DIR, typename T>
struct Dft<3, DIR, T> {
  static __device__ __forceinline__ void run(cpx<T>* x) {
    constexpr T c = (T)-0.5;
    constexpr T s = (T)(DIR * 0.866025403784438646763723170752936183);  // DIR sin(2pi/3)
    cpx<T> t1 = x[1] + x[2], t2 = x[1] - x[2];
    cpx<T> m = mk(x[0].x + c * t1.x, x[0].y + c * t1.y);
    cpx<T> r = mk(-s * t2.y, s * t2.x);  // i s t2
    x[0] = x[0] + t1;
    x[1] = m + r;
    x[2] = m - r;
  }
};
template <int DIR, typename T>
struct Dft<4, DIR, T> {
  static __device__ __forceinline__ void run(cpx<T>* x) {
    cpx<T> a0 = x[0] + x[2], a1 = x[0] - x[2];
    cpx<T> b0 = x[1] + x[3], b1 = mul_i<DIR>(x[1] - x[3]);
    x[0] = a0 + b0;
    x[2] = a0 - b0;
    x[1] = a1 + b1;
    x[3] = a1 - b1;
  }
};
template <int DIR, typename T>
struct Dft<6, DIR, T> {
  static __device__ __forceinline__ void run(cpx<T>* x) { dft_ab<2, 3, DIR, T>(x); }
};
template <int DIR, typename T>
struct Dft<8, DIR, T> {
  static __device__ __forceinline__ void run(cpx<T>* x) { dft_ab<2, 4, DIR, T>(x); }
};
template <int DIR, typename T>
struct Dft<12, DIR, T> {
  static __device__ __forceinline__ void run(cpx<T>* x) { dft_ab<4, 3, DIR, T>(x); }
};
template <int DIR, typename T>
struct Dft<16, DIR, T> {
  static __device__ __forceinline__ void run(cpx<T>* x) { dft_ab<4, 4, DIR, T>(x); }
};
template <int DIR, typename T>
struct Dft<24, DIR, T> {
  static __device__ __forceinline__ void run(cpx<T>* x) { dft_ab<8, 3, DIR, T>(x); }
};

// R = A B: B-point DFTs over x[a + A b], twiddle w_R^(a kb), A-point DFTs,
// output index kb + B ka.
template <int A, int B, int DIR, typename T>
__device__ __forceinline__ void dft_ab(cpx<T>* x) {
  constexpr int R = A * B;
  cpx<T> y[R];
  static_for<0, A>([&](auto ia) {
    constexpr int a = decltype(ia)::value;
    cpx<T> t[B];
    static_for<0, B>([&](auto ib) {
      constexpr int b = decltype(ib)::value;
      t[b] = x[a + A * b];
    });
    Dft<B, DIR, T>::run(t);
    static_for<0, B>([&](auto ik) {
      constexpr int kb = decltype(ik)::value;
      y[a * B + kb] = twc<R, a * kb, DIR>(t[kb]);
    });
  });
  static_for<0, B>([&](auto ik) {
    constexpr int kb = decltype(ik)::value;
    cpx<T> t[A];
    static_for<0, A>([&](auto ia) {
      constexpr int a = decltype(ia)::value;
      t[a] = y[a * B + kb];
    });
    Dft<A, DIR, T>::run(t);
    static_for<0, A>([&](auto ia) {
      constexpr int ka = decltype(ia)::value;
      x[kb + B * ka] = t[ka];
    });
  });
}

// ---------------------------------------------------------------------------
// per-length pass plans (radices in inverse-transform order; the forward
// transform runs them reversed).  Plan<N, 0> is the default of each length;
// Plan<N, 1..> are alternative factorisations of the same length, among which
// the autotuner chooses for the two-launch kernels.  Each plan computes the
// same DFT; only the rounding and the speed differ.
// ---------------------------------------------------------------------------
template <int N, int PV = 0>
struct Plan;
template <int N>
struct PlanCount {
  static constexpr int value = 1;
};
#define PD_PLAN(N_, PV_, M_, A_, B_, C_)                         \
  template <>                                                    \
  struct Plan<N_, PV_> {                                         \
    static constexpr int M = M_;                                 \
    static constexpr int r(int i) { return i == 0 ? A_ : i == 1 ? B_ : C_; } \
  };
#define PD_PLAN_COUNT(N_, K_)                                    \
  template <>                                                    \
  struct PlanCount<N_> {                                         \
    static constexpr int value = K_;                             \
  };
PD_PLAN(8, 0, 1, 8, 1, 1)
PD_PLAN(16, 0, 1, 16, 1, 1)
PD_PLAN(24, 0, 2, 8, 3, 1)
PD_PLAN(32, 0, 2, 8, 4, 1)
PD_PLAN(48, 0, 2, 16, 3, 1)
PD_PLAN(64, 0, 2, 8, 8, 1)
PD_PLAN(64, 1, 2, 16, 4, 1)
PD_PLAN(64, 2, 2, 4, 16, 1)
PD_PLAN_COUNT(64, 3)
PD_PLAN(96, 0, 2, 8, 12, 1)
PD_PLAN(96, 1, 2, 12, 8, 1)
PD_PLAN(96, 2, 2, 24, 4, 1)
PD_PLAN_COUNT(96, 3)
PD_PLAN(128, 0, 2, 16, 8, 1)
PD_PLAN(128, 1, 2, 8, 16, 1)
PD_PLAN(128, 2, 3, 8, 4, 4)
PD_PLAN_COUNT(128, 3)
PD_PLAN(192, 0, 2, 16, 12, 1)
PD_PLAN(192, 1, 2, 12, 16, 1)
PD_PLAN(192, 2, 2, 24, 8, 1)
PD_PLAN_COUNT(192, 3)
PD_PLAN(256, 0, 2, 16, 16, 1)
PD_PLAN(256, 1, 3, 8, 8, 4)
PD_PLAN(256, 2, 3, 4, 4, 16)
PD_PLAN_COUNT(256, 3)
PD_PLAN(288, 0, 2, 12, 24, 1)
PD_PLAN(288, 1, 2, 24, 12, 1)
PD_PLAN_COUNT(288, 2)
PD_PLAN(384, 0, 2, 16, 24, 1)
PD_PLAN(384, 1, 2, 24, 16, 1)
PD_PLAN(384, 2, 3, 8, 6, 8)
PD_PLAN_COUNT(384, 3)
PD_PLAN(512, 0, 3, 8, 8, 8)
PD_PLAN(512, 1, 3, 16, 8, 4)
PD_PLAN(512, 2, 3, 4, 8, 16)
PD_PLAN_COUNT(512, 3)
PD_PLAN(576, 0, 2, 24, 24, 1)
PD_PLAN(576, 1, 3, 12, 8, 6)
PD_PLAN_COUNT(576, 2)
PD_PLAN(768, 0, 3, 24, 8, 4)
PD_PLAN(768, 1, 3, 16, 8, 6)
PD_PLAN(768, 2, 3, 12, 8, 8)
PD_PLAN_COUNT(768, 3)
#undef PD_PLAN
#undef PD_PLAN_COUNT

// radix of the i-th executed pass: inverse runs r(0..M-1), forward r(M-1..0)
template <int N, int DIR, int PV = 0>
constexpr int pass_radix(int i) {
  return DIR > 0 ? Plan<N, PV>::r(i) : Plan<N, PV>::r(Plan<N, PV>::M - 1 - i);
}
// product of the radices executed before pass i
template <int N, int DIR, int PV = 0>
constexpr int pass_prod(int i) {
  int p = 1;
  for (int t = 0; t < i; ++t) p *= pass_radix<N, DIR, PV>(t);
  return p;
}
constexpr int cdiv(int a, int b) { return (a + b - 1) / b; }

// ---------------------------------------------------------------------------
// Batched FFT engine: S sequences of length N per workgroup of NT threads.
// COLS = true: sequence index fastest across threads (column strips, element
// n of sequence s at lds[n*(S+1)+s]); COLS = false: element index fastest
// (rows, lds[s*LDN + n + n/32]).  Butterfly w of a pass with N/Q butterflies
// per sequence belongs to thread w mod NT.
// ---------------------------------------------------------------------------
template <typename T, int N, int S, int NT, bool COLS, int PV = 0>
struct Fft {
  static constexpr int kNT = NT;
  static constexpr int kN = N;
  static constexpr int LDN = N + N / 32 + 1;                 // padded row (rows layout)
  static constexpr int LDS_ELEMS = COLS ? N * (S + 1) : S * LDN;

  static __device__ __forceinline__ int lidx(int s, int n) {
    if constexpr (COLS) return n * (S + 1) + s;
    else return s * LDN + n + (n >> 5);
  }
  template <int Q>
  static __device__ __forceinline__ void coords(int w, int& s, int& j) {
    constexpr int J = N / Q;
    if constexpr (COLS) {
      s = w % S;
      j = w / S;
    } else {
      s = w / J;
      j = w % J;
    }
  }
  template <int Q>
  static constexpr int nbutter() { return S * (N / Q); }
  template <int Q>
  static constexpr int nq() { return cdiv(S * (N / Q), NT); }

  // twiddle r*k of a pass with product p and radix Q, from the forward
  // table tw[m] = exp(-2 pi i m / N); conjugated for the inverse.
  template <int DIR, int P, int Q>
  static __device__ __forceinline__ cpx<T> tw_mul(cpx<T> a, const cpx<T>* __restrict__ tw, int r, int k) {
    constexpr int stride = N / (P * Q);
    cpx<T> w = tw[r * k * stride];
    if constexpr (DIR > 0) return cmulc(a, w);
    else return cmul(a, w);
  }

  // first pass (p = 1, no twiddles): v holds inputs at j + r N/Q; DFT and
  // store the Stockham outputs to LDS.
  template <int DIR, int Q>
  static __device__ __forceinline__ void first_to_lds(cpx<T> (&v)[nq<Q>()][Q], cpx<T>* lds, int tid) {
#pragma unroll
    for (int q = 0; q < nq<Q>(); ++q) {
      int w = tid + q * NT;
      if (nbutter<Q>() % NT == 0 || w < nbutter<Q>()) {
        int s, j;
        coords<Q>(w, s, j);
        Dft<Q, DIR, T>::run(v[q]);
#pragma unroll
        for (int r = 0; r < Q; ++r) lds[lidx(s, j * Q + r)] = v[q][r];
      }
    }
  }

  // Rows layout with one radix in every pass and N/Q butterflies per row
  // dividing the wave: row s belongs to the N/Q consecutive threads from
  // s N/Q on, inside one wave, in every pass, and its LDS row is touched by
  // no other wave.  The passes of such a transform then only need the lanes
  // of one wave ordered (LDS executes a wave's accesses in issue order), not
  // a workgroup barrier.
  static constexpr bool uniform_plan() {
    for (int i = 1; i < Plan<N, PV>::M; ++i)
      if (Plan<N, PV>::r(i) != Plan<N, PV>::r(0)) return false;
    return true;
  }
  static constexpr bool kWaveLocal = !COLS && uniform_plan() && (N / Plan<N, PV>::r(0)) <= 64 &&
                                     64 % (N / Plan<N, PV>::r(0)) == 0 && NT % 64 == 0;

  // order the LDS accesses between two passes: the whole workgroup, or with
  // WL the lanes of each wave (kWaveLocal engines only)
  template <bool WL>
  static __device__ __forceinline__ void lds_sync() {
    if constexpr (WL) {
      static_assert(kWaveLocal, "wave-local passes need a wave-local engine");
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
      __syncthreads();
    }
  }

  // a pass after the first: read LDS, twiddle, DFT; if LAST keep the
  // outputs (positions j + r N/Q) in v, else write them back to LDS.
  template <int DIR, int PI, bool LAST, bool WL = false>
  static __device__ __forceinline__ void pass_from_lds(
      cpx<T> (&v)[nq<pass_radix<N, DIR, PV>(PI)>()][pass_radix<N, DIR, PV>(PI)], cpx<T>* lds,
      const cpx<T>* __restrict__ tw, int tid) {
    constexpr int Q = pass_radix<N, DIR, PV>(PI);
    constexpr int P = pass_prod<N, DIR, PV>(PI);
    lds_sync<WL>();
#pragma unroll
    for (int q = 0; q < nq<Q>(); ++q) {
      int w = tid + q * NT;
      if (nbutter<Q>() % NT == 0 || w < nbutter<Q>()) {
        int s, j;
        coords<Q>(w, s, j);
#pragma unroll
        for (int r = 0; r < Q; ++r) v[q][r] = lds[lidx(s, j + r * (N / Q))];
      }
    }
    if constexpr (!LAST) lds_sync<WL>();
#pragma unroll
    for (int q = 0; q < nq<Q>(); ++q) {
      int w = tid + q * NT;
      if (nbutter<Q>() % NT == 0 || w < nbutter<Q>()) {
        int s, j;
        coords<Q>(w, s, j);
        int k = j % P;
#pragma unroll
        for (int r = 1; r < Q; ++r) v[q][r] = tw_mul<DIR, P, Q>(v[q][r], tw, r, k);
        Dft<Q, DIR, T>::run(v[q]);
        if constexpr (!LAST) {
#pragma unroll
          for (int r = 0; r < Q; ++r) lds[lidx(s, (j - k) * Q + k + r * P)] = v[q][r];
        }
      }
    }
  }

  static constexpr int M = Plan<N, PV>::M;
  static_assert(pass_prod<N, -1, PV>(Plan<N, PV>::M) == N, "the pass radices of a plan multiply to its length");
  template <int DIR>
  static constexpr int QF() { return pass_radix<N, DIR, PV>(0); }
  template <int DIR>
  static constexpr int QL() { return pass_radix<N, DIR, PV>(M - 1); }

  // Whole transform: `in` holds the inputs of the first pass (positions
  // j + r N/QF), `out` receives the outputs of the last pass (positions
  // j + r N/QL).  in and out may be the same array when QF == QL.  Starts
  // with a barrier-free LDS write, so the caller must have synchronised
  // any earlier LDS readers (call sync_before_reuse()).
  // Twiddle-table entries the transform reads (tw[m] = exp(-2 pi i m / N)).
  static constexpr int TW_MAX = N;
  static __host__ __device__ constexpr int tw_count(int /*len*/) { return N; }

  // With WL (kWaveLocal engines) the passes order only each wave's lanes,
  // and the caller's sync_before_reuse<true>() suffices between transforms.
  template <int DIR, bool WL = false>
  static __device__ __forceinline__ void run(cpx<T> (&in)[nq<QF<DIR>()>()][QF<DIR>()],
                                             cpx<T> (&out)[nq<QL<DIR>()>()][QL<DIR>()],
                                             cpx<T>* lds, const cpx<T>* __restrict__ tw, int tid,
                                             int /*len*/ = N) {
    if constexpr (M == 1) {
#pragma unroll
      for (int q = 0; q < nq<QF<DIR>()>(); ++q) {
        Dft<QF<DIR>(), DIR, T>::run(in[q]);
#pragma unroll
        for (int r = 0; r < QF<DIR>(); ++r) out[q][r] = in[q][r];
      }
    } else {
      first_to_lds<DIR, QF<DIR>()>(in, lds, tid);
      if constexpr (M == 3) {
        constexpr int Q1 = pass_radix<N, DIR, PV>(1);
        cpx<T> mid[nq<Q1>()][Q1];
        pass_from_lds<DIR, 1, false, WL>(mid, lds, tw, tid);
      }
      pass_from_lds<DIR, M - 1, true, WL>(out, lds, tw, tid);
    }
  }

  template <bool WL = false>
  static __device__ __forceinline__ void sync_before_reuse() {
    if constexpr (M > 1) lds_sync<WL>();
  }

  // position (sequence, element) of register (q, r) of a first/last pass
  // with radix Q
  template <int Q>
  static __device__ __forceinline__ bool pos(int tid, int q, int r, int& s, int& n) {
    int w = tid + q * NT;
    int j;
    coords<Q>(w, s, j);
    n = j + r * (N / Q);
    return nbutter<Q>() % NT == 0 || w < nbutter<Q>();
  }
};

// ---------------------------------------------------------------------------
// Bluestein (chirp-z) engine: a length-`len` DFT of any len <= (M + 1) / 2,
// computed with two length-M transforms of the engine above.  With the chirp
// c_n = exp(-i pi n^2 / len),
//     X_k = c_k sum_n (x_n c_n) conj(c_(k-n)),
// a linear convolution that a cyclic one of length M >= 2 len - 1 computes
// exactly: X = c . F_M^-1( F_M(c . x, zero-padded) . B ), B = F_M(b) / M with
// b_m = conj(c_m) for |m| < len (indices mod M) and 0 elsewhere.  The inverse
// transform conjugates every chirp (its B is F_M(c) / M).  Input and output
// use the same register layout (the forward length-M transform's first-pass
// positions); positions n >= len are padding: zero on input, ignored on output.
//
// Table `tw` (staged in LDS): [M twiddles of length M][len chirp values]
// [M entries of B for the forward DFT][M entries of B for the inverse DFT].
// ---------------------------------------------------------------------------
template <typename T, int M, int S, int NT, bool COLS>
struct Blue {
  using F0 = Fft<T, M, S, NT, COLS>;
  static constexpr int kNT = NT;
  static constexpr bool kWaveLocal = false;   // its chirp tables are shared across rows
  static constexpr int LDS_ELEMS = F0::LDS_ELEMS;
  static constexpr int L0 = F0::template QF<-1>();   // forward first-pass radix
  static constexpr int L1 = F0::template QL<-1>();   // forward last-pass radix
  template <int DIR>
  static constexpr int QF() { return L0; }
  template <int DIR>
  static constexpr int QL() { return L0; }
  template <int Q>
  static constexpr int nq() { return F0::template nq<Q>(); }
  static constexpr int TW_MAX = M + (M + 1) / 2 + 2 * M;
  static __host__ __device__ constexpr int tw_count(int len) { return 3 * M + len; }

  template <int Q>
  static __device__ __forceinline__ bool pos(int tid, int q, int r, int& s, int& n) {
    return F0::template pos<Q>(tid, q, r, s, n);
  }
  static __device__ __forceinline__ int lidx(int s, int n) { return F0::lidx(s, n); }

  template <int DIR, bool WL = false>
  static __device__ __forceinline__ void run(cpx<T> (&in)[nq<L0>()][L0], cpx<T> (&out)[nq<L0>()][L0], cpx<T>* lds,
                                             const cpx<T>* __restrict__ tw, int tid, int len) {
    static_assert(!WL, "Bluestein transforms synchronise the workgroup");
    const cpx<T>* __restrict__ chirp = tw + M;
    const cpx<T>* __restrict__ bh = tw + M + len + (DIR < 0 ? 0 : M);
    // a_n = x_n c_n (conj(c_n) for the inverse), zero beyond len
#pragma unroll
    for (int q = 0; q < nq<L0>(); ++q)
#pragma unroll
      for (int r = 0; r < L0; ++r) {
        int s, n;
        const bool ok = F0::template pos<L0>(tid, q, r, s, n);
        if (ok && n < len) in[q][r] = DIR < 0 ? cmul(in[q][r], chirp[n]) : cmulc(in[q][r], chirp[n]);
        else in[q][r] = mk((T)0, (T)0);
      }
    cpx<T> mid[nq<L1>()][L1];
    F0::template run<-1>(in, mid, lds, tw, tid);
#pragma unroll
    for (int q = 0; q < nq<L1>(); ++q)
#pragma unroll
      for (int r = 0; r < L1; ++r) {
        int s, k;
        if (F0::template pos<L1>(tid, q, r, s, k)) mid[q][r] = cmul(mid[q][r], bh[k]);
      }
    F0::sync_before_reuse();
    F0::template run<+1>(mid, out, lds, tw, tid);
#pragma unroll
    for (int q = 0; q < nq<L0>(); ++q)
#pragma unroll
      for (int r = 0; r < L0; ++r) {
        int s, n;
        if (F0::template pos<L0>(tid, q, r, s, n) && n < len)
          out[q][r] = DIR < 0 ? cmul(out[q][r], chirp[n]) : cmulc(out[q][r], chirp[n]);
      }
  }

  template <bool WL = false>
  static __device__ __forceinline__ void sync_before_reuse() {
    static_assert(!WL, "Bluestein transforms synchronise the workgroup");
    __syncthreads();
  }
};

// Engine of a kernel's transform axis: EXT < 2 the plain length-N engine with
// pass plan PV, EXT == 2 the Bluestein engine on length-N transforms (default
// plan).
template <typename T, int N, int S, int NT, bool COLS, int EXT, int PV = 0>
using AxisFft = std::conditional_t<EXT == 2, Blue<T, N, S, NT, COLS>, Fft<T, N, S, NT, COLS, PV>>;

}  // namespace pdk
