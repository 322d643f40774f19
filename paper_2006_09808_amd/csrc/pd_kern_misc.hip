// pd_kern_misc.hip - duality-gap reduction, output unpacking, buffer fill,
// and the per-length dispatch of the column/row kernels.
#include "pd_fft.hpp"
#include "pd_internal.hpp"

namespace pdk {

#define PD_DECL(N)                                                                                   \
  hipError_t launch_col_##N(int, int, int, int, const Vol*, const Range*, int, Ctl*, int, int, int, int, hipStream_t); \
  hipError_t launch_row_##N(int, int, int, int, const Vol*, const Range*, int, Ctl*, int, int, int, int, hipStream_t);
PD_DECL(8)
PD_DECL(16)
PD_DECL(24)
PD_DECL(32)
PD_DECL(48)
PD_DECL(64)
PD_DECL(96)
PD_DECL(128)
PD_DECL(192)
PD_DECL(256)
PD_DECL(288)
PD_DECL(384)
PD_DECL(512)
PD_DECL(576)
PD_DECL(768)
#undef PD_DECL

#define PD_DECL_RES(N, V)                                                                                   \
  hipError_t launch_resident_##N##_##V(int, const Vol*, const Range*, int, Ctl*, unsigned*, int*, int,    \
                                       unsigned, hipStream_t);                                           \
  int resident_max_teams_##N##_##V();                                                                    \
  int resident_team_##N##_##V();                                                                         \
  int resident_threads_##N##_##V();                                                                      \
  int resident_plan_##N##_##V();
#define PD_RES_LIST(X)                                                                                  \
  X(64, 0) X(64, 1) X(64, 2) X(128, 0) X(128, 1) X(128, 2) X(128, 3) X(128, 4) X(192, 0) X(192, 1)    \
  X(192, 2) X(192, 3)                                                                                   \
  X(256, 0) X(256, 1) X(256, 2) X(256, 3)
PD_RES_LIST(PD_DECL_RES)
#undef PD_DECL_RES

#define PD_RES_ENTRY(N, V) \
  {N, launch_resident_##N##_##V, resident_max_teams_##N##_##V, resident_team_##N##_##V, resident_threads_##N##_##V, \
   resident_plan_##N##_##V},
static const ResidentVariant kResident[] = {PD_RES_LIST(PD_RES_ENTRY)};
#undef PD_RES_ENTRY
#undef PD_RES_LIST

int resident_variant_count(int n) {
  int k = 0;
  for (const auto& r : kResident) k += r.n == n;
  return k;
}

const ResidentVariant* resident_variant(int n, int v) {
  int k = 0;
  for (const auto& r : kResident)
    if (r.n == n && k++ == v) return &r;
  return nullptr;
}

bool size_supported(int n) {
  switch (n) {
    case 8: case 16: case 24: case 32: case 48: case 64: case 96:
    case 128: case 192: case 256: case 288: case 384: case 512: case 576: case 768:
      return true;
    default:
      return false;
  }
}

int blue_len(int n) {
  static const int lens[] = {8, 16, 24, 32, 48, 64, 96, 128, 192, 256, 288, 384, 512, 576, 768};
  if (n < 2) return 0;
  for (int m : lens)
    if (m >= 2 * n - 1) return m;
  return 0;
}

#define PD_CASE(N, KIND) \
  case N: return launch_##KIND##_##N(mode, g, grid, groups, vols, ranges, nranges, ctl, it, precision, ext, plan, st);

hipError_t launch_col_p(int n, int mode, int g, int grid, int groups, const Vol* vols, const Range* ranges,
                        int nranges, Ctl* ctl, int it, int precision, int ext, int plan, hipStream_t st) {
  switch (n) {
    PD_CASE(8, col) PD_CASE(16, col) PD_CASE(24, col) PD_CASE(32, col) PD_CASE(48, col)
    PD_CASE(64, col) PD_CASE(96, col) PD_CASE(128, col) PD_CASE(192, col) PD_CASE(256, col)
    PD_CASE(288, col) PD_CASE(384, col) PD_CASE(512, col) PD_CASE(576, col) PD_CASE(768, col)
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_row_p(int n, int mode, int g, int grid, int groups, const Vol* vols, const Range* ranges,
                        int nranges, Ctl* ctl, int it, int precision, int ext, int plan, hipStream_t st) {
  switch (n) {
    PD_CASE(8, row) PD_CASE(16, row) PD_CASE(24, row) PD_CASE(32, row) PD_CASE(48, row)
    PD_CASE(64, row) PD_CASE(96, row) PD_CASE(128, row) PD_CASE(192, row) PD_CASE(256, row)
    PD_CASE(288, row) PD_CASE(384, row) PD_CASE(512, row) PD_CASE(576, row) PD_CASE(768, row)
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_col(int n, int mode, int g, int grid, int groups, const Vol* vols, const Range* ranges,
                      int nranges, Ctl* ctl, int it, int precision, int ext, hipStream_t st) {
  return launch_col_p(n, mode, g, grid, groups, vols, ranges, nranges, ctl, it, precision, ext, 0, st);
}

hipError_t launch_row(int n, int mode, int g, int grid, int groups, const Vol* vols, const Range* ranges,
                      int nranges, Ctl* ctl, int it, int precision, int ext, hipStream_t st) {
  return launch_row_p(n, mode, g, grid, groups, vols, ranges, nranges, ctl, it, precision, ext, 0, st);
}

int plan_count(int n) {
  switch (n) {
    case 8: return PlanCount<8>::value;
    case 16: return PlanCount<16>::value;
    case 24: return PlanCount<24>::value;
    case 32: return PlanCount<32>::value;
    case 48: return PlanCount<48>::value;
    case 64: return PlanCount<64>::value;
    case 96: return PlanCount<96>::value;
    case 128: return PlanCount<128>::value;
    case 192: return PlanCount<192>::value;
    case 256: return PlanCount<256>::value;
    case 288: return PlanCount<288>::value;
    case 384: return PlanCount<384>::value;
    case 512: return PlanCount<512>::value;
    case 576: return PlanCount<576>::value;
    case 768: return PlanCount<768>::value;
    default: return 1;
  }
}
#undef PD_CASE

// ---------------------------------------------------------------------------
// Duality gap of one volume from the per-workgroup partial sums (FP64,
// fixed summation order).  P = 1/2 sum|D F chi - F delta|^2 / (nx ny)
// + lam sum|chi| (Parseval), Dual = -1/2 s^2 sum|Yhat|^2/(nx ny)
// - s Re sum Yhat conj(F delta)/(nx ny), s = min(1, lam / max|A y|).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_reduce(const Vol* __restrict__ vols,
                                                     const int* __restrict__ slots,
                                                     Ctl* __restrict__ ctl, int it) {
  const int tid = threadIdx.x;
  const int slot = slots[blockIdx.x];
  const Vol& V = vols[slot];
  if (ctl[slot].stop || it != V.iters - 1 || !V.check_last) return;
  const int nr = V.P * V.row_groups, nc = V.col_parts;
  double l1 = 0.0, mx = 0.0, res = 0.0, yy = 0.0, yd = 0.0;
  for (int i = tid; i < nr; i += kThreads) {
    l1 += V.part_row[2 * (size_t)i];
    mx = fmax(mx, V.part_row[2 * (size_t)i + 1]);
  }
  for (int i = tid; i < nc; i += kThreads) {
    res += V.part_col[3 * (size_t)i];
    yy += V.part_col[3 * (size_t)i + 1];
    yd += V.part_col[3 * (size_t)i + 2];
  }
  __shared__ double red[5][kThreads / 64];
  double v[5] = {l1, mx, res, yy, yd};
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    double x = v[k];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      double o = __shfl_down(x, off, 64);
      x = (k == 1) ? fmax(x, o) : x + o;
    }
    if ((tid & 63) == 0) red[k][tid >> 6] = x;
  }
  __syncthreads();
  if (tid != 0) return;
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    double x = red[k][0];
    for (int w = 1; w < kThreads / 64; ++w) x = (k == 1) ? fmax(x, red[k][w]) : x + red[k][w];
    v[k] = x;
  }
  const double invN = V.gap_norm;   // Parseval: 1 / points of one transform
  const double lam = V.lam;
  const double P = 0.5 * v[2] * invN + lam * v[0];
  const double m = v[1];
  const double s = (m == 0.0) ? 1.0 : fmin(1.0, lam / m);
  const double Dual = -0.5 * s * s * v[3] * invN - s * v[4] * invN;
  const double rel = (P - Dual) / fmax(P, 1e-300);
  Ctl& C = ctl[slot];
  C.primal = P;
  C.dual = Dual;
  C.rel_gap = rel;
  C.max_ay = m;
  C.stop_iter = V.done_base + it + 1;
  C.checks += 1;
  const bool finite = isfinite(P) && isfinite(Dual) && isfinite(m);
  if (!finite) {
    C.status = 1;
    C.stop = 1;
  } else if (it == V.final_it || (V.gap_tol > 0.0 && rel <= V.gap_tol)) {
    C.stop = 1;
  }
}

hipError_t launch_reduce(int nslots, const Vol* vols, const int* slots, Ctl* ctl, int it,
                         int /*precision*/, hipStream_t st) {
  if (nslots <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_reduce, dim3(nslots), dim3(kThreads), 0, st, vols, slots, ctl, it);
  return hipGetLastError();
}

// chi state (pair-interleaved) -> caller's planar [nz][ny][nx]
template <typename T>
__global__ __launch_bounds__(kThreads) void k_store_chi(const Vol* __restrict__ vols, int slot) {
  const Vol& V = vols[slot];
  const size_t plane = (size_t)V.nx * V.ny;
  const size_t total = (size_t)V.P * plane;
  const cpx<T>* __restrict__ chi = (const cpx<T>*)V.chi;
  T* __restrict__ out = (T*)V.user_out;
  const int nz = V.nz;
  for (size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x; i < total;
       i += (size_t)gridDim.x * kThreads) {
    size_t p = i / plane, o = i - p * plane;
    cpx<T> c = chi[i];
    if (V.unpacked) {
      out[p * plane + o] = c.x;
    } else {
      out[(2 * p) * plane + o] = c.x;
      if ((int)(2 * p + 1) < nz) out[(2 * p + 1) * plane + o] = c.y;
    }
  }
}

hipError_t launch_store_chi(const Vol* vols, int slot, size_t npts, int precision, hipStream_t st) {
  size_t blocks = (npts + kThreads - 1) / kThreads;
  if (blocks > 4096) blocks = 4096;
  if (blocks == 0) blocks = 1;
  if (precision == 1)
    hipLaunchKernelGGL(k_store_chi<double>, dim3((unsigned)blocks), dim3(kThreads), 0, st, vols, slot);
  else
    hipLaunchKernelGGL(k_store_chi<float>, dim3((unsigned)blocks), dim3(kThreads), 0, st, vols, slot);
  return hipGetLastError();
}

// zero fill (a kernel rather than a memset node, so it can live in a graph)
__global__ __launch_bounds__(kThreads) void k_zero(uint4* __restrict__ p, size_t n16, unsigned char* tail,
                                                   size_t ntail) {
  for (size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x; i < n16; i += (size_t)gridDim.x * kThreads)
    p[i] = make_uint4(0u, 0u, 0u, 0u);
  if (blockIdx.x == 0 && threadIdx.x < ntail) tail[threadIdx.x] = 0;
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t st) {
  if (bytes == 0) return hipSuccess;
  if (((uintptr_t)p & 15) != 0) return hipErrorInvalidValue;
  size_t n16 = bytes / 16, ntail = bytes - n16 * 16;
  size_t blocks = (n16 + kThreads - 1) / kThreads;
  if (blocks > 4096) blocks = 4096;
  if (blocks == 0) blocks = 1;
  hipLaunchKernelGGL(k_zero, dim3((unsigned)blocks), dim3(kThreads), 0, st, (uint4*)p, n16,
                     (unsigned char*)p + n16 * 16, ntail);
  return hipGetLastError();
}

}  // namespace pdk
