// pd_host.cpp - the C ABI: validation, arena allocation, per-shape kernel
// tables, and the scheduler that iterates every resident request together.
//
// Execution model (one context = one device stream + one worker thread):
//   pd_solve_batch validates and queues requests.  The worker admits queued
//   requests in FIFO order while a slot and arena space are free, runs their
//   set-up (F delta, zeroed state), then advances all resident requests by a
//   "step" of K iterations: per iteration one column-kernel and one row-kernel
//   launch per distinct slice shape, covering every pair of every resident
//   volume of that shape, plus the gap check kernels on check iterations.
//   Check results decide on the device whether a volume stops (kernels skip
//   stopped volumes), and the host retires stopped volumes at step end:
//   chi is unpacked into the caller's buffer, the arena space and slot are
//   released, and the next queued requests are admitted.  Every resident
//   volume keeps its primal, dual and exchange state in the arena between
//   steps (the paper's device residency, Sec. II-D).
#include "pd.h"
#include "pd_arena.hpp"
#include "pd_internal.hpp"

#include <algorithm>
#include <array>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <set>
#include <memory>
#include <mutex>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <thread>
#include <vector>

using namespace pdk;
using pdh::Arena;

namespace {

constexpr size_t kAlign = 256;
constexpr int kDefaultSlots = 256;
constexpr int kDefaultStep = 500;       // step cap while no request waits for admission
constexpr int kQueuedStep = 50;         // step cap while requests wait in the queue
constexpr int kMaxStep = 1 << 20;
constexpr int kMaxGraphs = 32;
// run-ahead: while no request waits, a round enqueues up to kRunAhead steps
// (stopping at kRunAheadIters iterations or at any volume's last iteration)
// before the host waits once; kernels skip volumes whose gap check already
// stopped them, so the steps after a stop cost a few empty launches only
constexpr int kRunAhead = 8;
constexpr int kRunAheadIters = 100;
constexpr double kIdleSpin = 200e-6;    // seconds the idle worker polls the queue before sleeping

inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
inline bool isfin(double x) { return std::isfinite(x); }

double now_s() {
  using namespace std::chrono;
  return duration_cast<duration<double>>(steady_clock::now().time_since_epoch()).count();
}

// ---------------------------------------------------------------------------
// dipole kernel grid (Eq. (1), operator D), FP64 on the host
// ---------------------------------------------------------------------------
double kfreq(int i, int n, double d) {
  int half = (n + 1) / 2;
  return (double)(i < half ? i : i - n) / ((double)n * d);
}

bool unit_b0(const double b[3], double out[3]) {
  double nb = std::sqrt(b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
  if (!isfin(nb) || nb == 0.0) return false;
  for (int i = 0; i < 3; ++i) out[i] = b[i] / nb;
  return true;
}

// D[ky][kx] = 1/3 - (k.b)^2/|k|^2, D(0) = 0, averaged between k and -k
void dipole_grid(int nx, int ny, const double b[3], const double vox[2], int kernel,
                 std::vector<double>& D) {
  D.assign((size_t)nx * ny, 1.0);
  if (kernel == PD_KERNEL_IDENTITY) return;
  double bu[3];
  unit_b0(b, bu);
  auto f = [&](double kx, double ky) {
    double k2 = kx * kx + ky * ky;
    if (k2 == 0.0) return 0.0;
    double kb = kx * bu[0] + ky * bu[1];
    return 1.0 / 3.0 - kb * kb / k2;
  };
  for (int j = 0; j < ny; ++j) {
    double ky = kfreq(j, ny, vox[1]), kym = kfreq((ny - j) % ny, ny, vox[1]);
    for (int i = 0; i < nx; ++i) {
      double kx = kfreq(i, nx, vox[0]), kxm = kfreq((nx - i) % nx, nx, vox[0]);
      D[(size_t)j * nx + i] = 0.5 * (f(kx, ky) + f(kxm, kym));
    }
  }
}

// 3-D kernel on the [nz][ny][nx] grid (kz with slice thickness dz), averaged
// between k and -k: f(index, value) for every grid point in index order (the
// grid is generated, not stored: it can hold 10^8 points)
template <typename Fn>
void dipole_grid3(int nx, int ny, int nz, const double b[3], const double vox[2], double dz, Fn&& out) {
  double bu[3];
  unit_b0(b, bu);
  auto f = [&](double kx, double ky, double kz) {
    double k2 = kx * kx + ky * ky + kz * kz;
    if (k2 == 0.0) return 0.0;
    double kb = kx * bu[0] + ky * bu[1] + kz * bu[2];
    return 1.0 / 3.0 - kb * kb / k2;
  };
  for (int l = 0; l < nz; ++l) {
    double kz = kfreq(l, nz, dz), kzm = kfreq((nz - l) % nz, nz, dz);
    for (int j = 0; j < ny; ++j) {
      double ky = kfreq(j, ny, vox[1]), kym = kfreq((ny - j) % ny, ny, vox[1]);
      for (int i = 0; i < nx; ++i) {
        double kx = kfreq(i, nx, vox[0]), kxm = kfreq((nx - i) % nx, nx, vox[0]);
        out(((size_t)l * ny + j) * nx + i, 0.5 * (f(kx, ky, kz) + f(kxm, kym, kzm)));
      }
    }
  }
}

double grid_norm(const std::vector<double>& D) {
  double m = 0.0;
  for (double d : D) m = std::max(m, std::fabs(d));
  return m;
}

// exp(-2 pi i m / n) for m < n, with the angle reduced to (-pi, pi]
void twiddles(int n, std::vector<double>& re, std::vector<double>& im) {
  re.resize(n);
  im.resize(n);
  const double pi = 3.14159265358979323846264338327950288;
  for (int m = 0; m < n; ++m) {
    int mm = (2 * m > n) ? m - n : m;
    double a = 2.0 * pi * (double)mm / (double)n;
    re[m] = std::cos(a);
    im[m] = -std::sin(a);
  }
}

// One axis of a slice: lengths with a direct plan are transformed as they
// are; any other length n (2 <= n <= 384) by the Bluestein engine on
// transforms of length blue_len(n).
inline bool axis_ok(int n) { return size_supported(n) || blue_len(n) > 0; }
inline bool axis_blue(int n) { return !size_supported(n); }
inline int axis_phys(int n) { return axis_blue(n) ? blue_len(n) : n; }
// twiddle-table entries of the axis: the length-n twiddles, or for Bluestein
// [M twiddles][n chirp values][M forward kernel][M inverse kernel]
inline size_t axis_tw_entries(int n) { return axis_blue(n) ? (size_t)3 * blue_len(n) + n : (size_t)n; }
inline int ceil_div(int a, int b) { return (a + b - 1) / b; }
// kernel variant for transforms along an axis of length n in tiles of `tile`
// sequences out of `other`: 2 Bluestein, 1 partial last tile, 0 plain
inline int axis_ext(int n, int other, int tile) { return axis_blue(n) ? 2 : (other % tile ? 1 : 0); }

// Bluestein table of a length-n axis on length-M transforms, interleaved
// (re, im): [M twiddles exp(-2 pi i m / M)][n chirp values c_k =
// exp(-i pi k^2 / n)][B_fwd][B_inv], B = F_M(b) / M with b_m = conj(c_|m|)
// (forward) or c_|m| (inverse) for |m| < n, indices mod M, 0 elsewhere.
// All in FP64 with exact integer argument reduction.
void bluestein_table(int n, int M, std::vector<double>& out) {
  const double pi = 3.14159265358979323846264338327950288;
  std::vector<double> re, im;
  twiddles(M, re, im);
  out.assign(2 * ((size_t)3 * M + n), 0.0);
  for (int m = 0; m < M; ++m) {
    out[2 * m] = re[m];
    out[2 * m + 1] = im[m];
  }
  std::vector<double> cr(n), ci(n);
  for (int q = 0; q < n; ++q) {
    long long r = ((long long)q * q) % (2LL * n);
    double a = pi * (double)r / (double)n;
    cr[q] = std::cos(a);
    ci[q] = -std::sin(a);
    out[2 * ((size_t)M + q)] = cr[q];
    out[2 * ((size_t)M + q) + 1] = ci[q];
  }
  for (int dir = 0; dir < 2; ++dir) {
    std::vector<double> br(M, 0.0), bi(M, 0.0);
    const double sgn = dir == 0 ? -1.0 : 1.0;   // forward: conj(c); inverse: c
    for (int q = 0; q < n; ++q) {
      br[q] = cr[q];
      bi[q] = sgn * ci[q];
      if (q > 0) {
        br[M - q] = cr[q];
        bi[M - q] = sgn * ci[q];
      }
    }
    const size_t off = (size_t)M + n + (size_t)dir * M;
    for (int kk = 0; kk < M; ++kk) {
      double sr = 0.0, si = 0.0;
      for (int m = 0; m < M; ++m) {
        long long e = ((long long)m * kk) % M;
        double w = -2.0 * pi * (double)e / (double)M;
        double wr = std::cos(w), wi = std::sin(w);
        sr += br[m] * wr - bi[m] * wi;
        si += br[m] * wi + bi[m] * wr;
      }
      out[2 * (off + kk)] = sr / M;
      out[2 * (off + kk) + 1] = si / M;
    }
  }
}

// work decomposition (must match the kernel instantiations)
int row_group_big(int nx) {   // the larger instantiated FP32 row group of length-nx rows
  int s = 8;
  while (s < 64 && 2 * s * nx <= 4096) s *= 2;
  return s;
}
int rows_per_wg(int nx, int ny, int precision) {
  if (precision == PD_FP64 || axis_blue(nx)) return 8;
  int s = row_group_big(nx);
  return (ny % s == 0) ? s : 8;
}
int col_group_wide(int ny) {   // the widest instantiated FP32 column strip (> 16 only for ny <= 128)
  int s = 16;
  while (s < 64 && 2 * s * ny <= 4096) s *= 2;
  return s;
}
int cols_per_wg(int nx, int ny, int precision) {
  if (precision == PD_FP64 || axis_blue(ny) || ny > 512) return 8;
  return (nx % 16 == 0) ? 16 : 8;
}

// instantiated tile sizes of the two-launch kernels: FP32 plain transforms
// over whole tiles have rows per row-kernel workgroup in {8, default} and
// columns per column-kernel workgroup in {8, 16, wide} (wide: 32 or 64 for
// columns of at most 128; 8 only for columns of 768); every other case (FP64,
// Bluestein, partial last tile) has tiles of 8
bool rows_valid(int r, int nx, int ny, int precision) {
  if (r <= 0) return false;
  if (precision == PD_FP64 || axis_blue(nx) || ny % r) return r == 8;
  return r == 8 || r == row_group_big(nx);
}
bool cols_valid(int cl, int nx, int ny, int precision) {
  if (cl <= 0) return false;
  if (precision == PD_FP64 || axis_blue(ny) || ny > 512 || nx % cl) return cl == 8;
  return cl == 8 || cl == 16 || cl == col_group_wide(ny);
}
// strip width of the 3-D kernel's z view (nx ny columns of length nz): the
// widest instantiated one that tiles the columns, so short z transforms get
// enough points per workgroup
int zcols_of(int nx, int ny, int nz, int precision) {
  for (int w : {col_group_wide(nz), 16})
    if (cols_valid(w, nx * ny, nz, precision)) return w;
  return 8;
}

struct Layout {
  int P, rows, cols, row_groups, col_groups;
  int ext_row, ext_col;             // kernel variants of the default tiles
  size_t field;                     // one [P][ny][nx] complex buffer
  size_t off_chi, off_yhat, off_dhat, off_ex, off_ex2, off_prow, off_pcol;
  // weighted TV model: over-relaxed primal, duals p, q_x, q_y (q_z), packed W, M, delta
  size_t off_chibar, off_p, off_qx, off_qy, off_qz, off_w, off_m, off_d;
  size_t total;
  bool separate_ex2;
  bool tv;
  bool unpacked;                    // 3-D kernel, L1 model: one slice per plane, P = nz
  bool tv3;                         // 3-D kernel, TV model: pairs, exchange of nz planes
  int planes;                       // planes of the exchange buffer (column kernels' "pairs")
  int zgroups, ext_z, zcols;        // 3-D kernel: z-transform workgroups, kernel variant, strip width
};

Layout layout_of(const pd_request& r, int precision) {
  Layout L{};
  size_t esz = precision == PD_FP64 ? 16 : 8;
  L.unpacked = r.kernel == PD_KERNEL_DIPOLE_3D && r.model != PD_MODEL_TV;
  L.tv3 = r.kernel == PD_KERNEL_DIPOLE_3D && r.model == PD_MODEL_TV;
  L.P = L.unpacked ? r.nz : (r.nz + 1) / 2;
  L.planes = L.tv3 ? r.nz : L.P;
  if (r.kernel == PD_KERNEL_DIPOLE_3D) {
    // z transforms: strips of 8 of the nx ny columns of the [nz][ny nx] view
    L.zcols = zcols_of(r.nx, r.ny, r.nz, precision);
    L.zgroups = ceil_div(r.nx * r.ny, L.zcols);
    L.ext_z = axis_ext(r.nz, r.nx * r.ny, L.zcols);
  }
  L.rows = rows_per_wg(r.nx, r.ny, precision);
  L.cols = cols_per_wg(r.nx, r.ny, precision);
  L.row_groups = ceil_div(r.ny, L.rows);
  L.col_groups = ceil_div(r.nx, L.cols);
  L.ext_row = axis_ext(r.nx, r.ny, L.rows);
  L.ext_col = axis_ext(r.ny, r.nx, L.cols);
  L.field = align_up((size_t)L.P * r.nx * r.ny * esz);
  size_t o = 0;
  if (r.model == PD_MODEL_TV) {
    // all state in the image domain; no gap partials (fixed iteration count)
    L.tv = true;
    L.off_chi = o; o += L.field;
    L.off_chibar = o; o += L.field;
    L.off_p = o; o += L.field;
    L.off_qx = o; o += L.field;
    L.off_qy = o; o += L.field;
    if (L.tv3) { L.off_qz = o; o += L.field; }
    L.off_w = o; o += L.field;
    L.off_m = o; o += L.field;
    L.off_d = o; o += L.field;
    L.off_ex = o; o += align_up((size_t)L.planes * r.nx * r.ny * esz);
    L.off_ex2 = L.off_ex;
    L.total = o;
    return L;
  }
  L.separate_ex2 = r.gap_tol > 0.0;
  L.off_chi = o; o += L.field;
  L.off_yhat = o; o += L.field;
  L.off_dhat = o; o += L.field;
  L.off_ex = o; o += L.field;
  if (L.separate_ex2) { L.off_ex2 = o; o += L.field; } else { L.off_ex2 = L.off_ex; }
  // gap partials: one entry per workgroup of any tile choice of the
  // two-launch kernels (8 rows or columns per workgroup at the least) or of
  // any resident team (at most 32 workgroups per pair)
  size_t pg = (size_t)std::max(std::max(ceil_div(r.ny, 8), ceil_div(r.nx, 8)), 32);
  L.off_prow = o; o += align_up((size_t)L.P * pg * 2 * sizeof(double));
  const size_t ncol = std::max((size_t)L.P * pg, (size_t)L.zgroups);
  L.off_pcol = o; o += align_up(ncol * 3 * sizeof(double));
  L.total = o;
  return L;
}

// D grid ([nz3][ny][nx], nz3 = 1 for the 2-D kernels) and the twiddle tables
// of x, y (and z for the 3-D kernel, nz3 > 1)
size_t table_bytes(int nx, int ny, int nz3, int precision) {
  size_t t = precision == PD_FP64 ? 8 : 4;
  size_t b = align_up((size_t)nx * ny * std::max(nz3, 1) * t) + align_up(axis_tw_entries(nx) * 2 * t) +
             align_up(axis_tw_entries(ny) * 2 * t);
  if (nz3 > 1) b += align_up(axis_tw_entries(nz3) * 2 * t);
  return b;
}
inline int nz3_of(const pd_request& r) { return r.kernel == PD_KERNEL_DIPOLE_3D ? r.nz : 0; }

// kernel, B0, voxel and (3-D kernel) slice thickness and z length
pd_status kernel_args(const pd_request* r) {
  if (r->kernel != PD_KERNEL_DIPOLE && r->kernel != PD_KERNEL_IDENTITY && r->kernel != PD_KERNEL_DIPOLE_3D)
    return PD_ERR_ARG;
  double bu[3];
  if (r->kernel != PD_KERNEL_IDENTITY && !unit_b0(r->b0, bu)) return PD_ERR_ARG;
  if (!isfin(r->voxel[0]) || !isfin(r->voxel[1]) || r->voxel[0] <= 0 || r->voxel[1] <= 0) return PD_ERR_ARG;
  if (r->kernel == PD_KERNEL_DIPOLE_3D) {
    if (!isfin(r->voxel_z) || r->voxel_z <= 0) return PD_ERR_ARG;
    if (!axis_ok(r->nz)) return PD_ERR_SIZE;
  }
  return PD_OK;
}

// max |D| per kernel grid, cached: validation runs on every submission and
// the grid has nx ny (nz) points
double cached_kernel_norm(const pd_request* r) {
  struct Key {
    int nx, ny, nz3, kernel;
    double b[3], vox[2], vz;
    bool operator<(const Key& o) const {
      return std::memcmp(this, &o, sizeof(Key)) < 0;
    }
  };
  static std::mutex mu;
  static std::map<Key, double> cache;
  Key k;
  std::memset(&k, 0, sizeof(k));   // padding takes part in the comparison
  k.nx = r->nx;
  k.ny = r->ny;
  k.nz3 = r->kernel == PD_KERNEL_DIPOLE_3D ? r->nz : 0;
  k.kernel = r->kernel;
  if (r->kernel != PD_KERNEL_IDENTITY) unit_b0(r->b0, k.b);
  k.vox[0] = r->voxel[0];
  k.vox[1] = r->voxel[1];
  k.vz = k.nz3 ? r->voxel_z : 0.0;
  {
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(k);
    if (it != cache.end()) return it->second;
  }
  double L = 0.0;
  if (r->kernel == PD_KERNEL_DIPOLE_3D) {
    dipole_grid3(r->nx, r->ny, r->nz, r->b0, r->voxel, r->voxel_z,
                 [&](size_t, double d) { L = std::max(L, std::fabs(d)); });
  } else {
    std::vector<double> D;
    dipole_grid(r->nx, r->ny, r->b0, r->voxel, r->kernel, D);
    L = grid_norm(D);
  }
  std::lock_guard<std::mutex> lk(mu);
  if (cache.size() > 4096) cache.clear();
  cache[k] = L;
  return L;
}

// check_ptrs: the device arrays must be given (a solve); pd_validate sizes a
// request before they exist and skips that test.
pd_status validate(const pd_request* r, int precision, double* norm_out, bool check_ptrs = true) {
  if (!r) return PD_ERR_ARG;
  if (precision != PD_FP32 && precision != PD_FP64) return PD_ERR_ARG;
  if (!axis_ok(r->nx) || !axis_ok(r->ny) || r->nz < 1) return PD_ERR_SIZE;
  pd_status ks = kernel_args(r);
  if (ks != PD_OK) return ks;
  if (!isfin(r->lambda) || r->lambda < 0) return PD_ERR_ARG;
  if (r->max_iter < 0) return PD_ERR_ARG;
  if (!isfin(r->gap_tol) || r->gap_tol < 0) return PD_ERR_ARG;
  if (r->gap_tol > 0 && r->check_every < 1) return PD_ERR_ARG;
  if (check_ptrs && (!r->delta || !r->chi)) return PD_ERR_ARG;
  if (r->model != PD_MODEL_L1 && r->model != PD_MODEL_TV) return PD_ERR_ARG;
  if (r->model == PD_MODEL_TV) {
    // lam weights the data term (it divides sigma in the dual prox); the
    // model runs a fixed number of iterations
    if ((check_ptrs && (!r->weight || !r->mask)) || r->gap_tol != 0.0 || !(r->lambda > 0)) return PD_ERR_ARG;
  }
  if (!isfin(r->tau) || !isfin(r->sigma) || r->tau <= 0 || r->sigma <= 0) return PD_ERR_STEP;
  if (!isfin(r->theta) || r->theta < 0 || r->theta > 1) return PD_ERR_STEP;
  const double L = cached_kernel_norm(r);
  // the TV model's condition also needs max|W| and max|M|: tested on the
  // device at admission
  if (r->model == PD_MODEL_L1 && !(r->tau * r->sigma * L * L < 1.0)) return PD_ERR_STEP;
  if (norm_out) *norm_out = L;
  return PD_OK;
}

// per kernel shape: D grid and the twiddles of both axes, in the arena
struct TableKey {
  int nx, ny, kernel;
  int nz3;                          // 3-D kernel: nz; else 0
  double b[3], vox[2], vz;
  bool operator<(const TableKey& o) const {
    if (nx != o.nx) return nx < o.nx;
    if (ny != o.ny) return ny < o.ny;
    if (kernel != o.kernel) return kernel < o.kernel;
    if (nz3 != o.nz3) return nz3 < o.nz3;
    if (vz != o.vz) return vz < o.vz;
    for (int i = 0; i < 3; ++i)
      if (b[i] != o.b[i]) return b[i] < o.b[i];
    for (int i = 0; i < 2; ++i)
      if (vox[i] != o.vox[i]) return vox[i] < o.vox[i];
    return false;
  }
};
struct Table {
  size_t off = 0, bytes = 0;
  int refs = 0;
  uint64_t last_use = 0;
  bool uploaded = false;
  void *d = nullptr, *twx = nullptr, *twy = nullptr, *twz = nullptr;
};

struct Job {
  uint64_t ticket = 0;
  pd_request req{};
  double t_submit = 0, t_start = 0, t_done = 0;
  int slot = -1;
  size_t off = 0;
  Layout L{};
  TableKey key{};
  Table tab{};              // copy of the shared table's device pointers
  int done_iters = 0;
  int run_iters = 0;        // iterations enqueued for it in the current round
  bool chi_stored = false;  // its result store is enqueued in the current round
  bool finished = false;
  bool in_resident = false; // some resident launch of the current round covers it
  double knorm = 0.0;       // max |D| of the request's kernel grid
  pd_result res{};
};

struct GroupKey {
  int nx, ny, model;
  int nz3;                          // 3-D kernel: nz (volumes batch only with equal nz); else 0
  bool operator<(const GroupKey& o) const {
    if (nx != o.nx) return nx < o.nx;
    if (ny != o.ny) return ny < o.ny;
    if (model != o.model) return model < o.model;
    return nz3 < o.nz3;
  }
};

}  // namespace

struct pd_ctx {
  pd_config cfg{};
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int device = 0;
  int precision = PD_FP32;
  int nslots = 0;

  std::mutex mu;               // queues, tickets, arena, tables
  std::condition_variable cv_work, cv_done;
  std::condition_variable cv_idle;   // signalled when the last in-flight API call leaves
  int calls = 0;               // API calls inside the context (CallGuard), under mu
  std::mutex exec_mu;          // GPU submission (worker steps vs. pd_apply_kernel)
  Arena arena;
  std::map<TableKey, Table> tables;
  uint64_t table_clock = 0;
  std::deque<std::shared_ptr<Job>> queue;
  std::vector<std::shared_ptr<Job>> active;
  std::map<uint64_t, std::shared_ptr<Job>> jobs;
  std::vector<int> free_slots;
  uint64_t next_ticket = 1;
  bool stopping = false;
  pd_status poisoned = PD_OK;
  std::thread worker;

  // control arrays: device copies carved from the arena, pinned host mirrors.
  // Entry nslots of vols/ctl/ranges is reserved for pd_apply_kernel.  The
  // step block [vols][slots][ranges] is contiguous on the device, so a step
  // uploads it in one copy from a pinned image of the same layout; likewise
  // [ctl][abort] comes back in one copy per round.
  size_t ctl_off = 0, ctl_bytes = 0;
  size_t off_slots = 0, off_ranges = 0;   // offsets inside the step block
  size_t off_abort = 0;                   // offset of the abort word after the ctl array
  char* h_stage[kRunAhead] = {};          // pinned step-block images, one per step of a round
  Vol* d_vols = nullptr;       // 2 (nslots + 1): plane views, then the 3-D kernel's z views from zoff
  int zoff = 0;
  std::atomic<int> n_queued{0};   // queue length, readable without the lock (worker's idle spin)
  Ctl* d_ctl = nullptr;        // nslots + 1
  int* d_slots = nullptr;      // nslots
  Range* d_ranges = nullptr;   // range_cap
  size_t range_cap = 0;        // entries of d_ranges / h_ranges; the last is pd_apply_kernel's
  unsigned* d_counters = nullptr;   // resident-launch counters, counter_bytes(kMaxTeamSlots)
  int* d_abort = nullptr;           // set by a resident launch whose barrier timed out
  int* h_abort = nullptr;      // inside the h_ctl block
  Vol* h_vols = nullptr;       // host mirror of the descriptors (set-up, operator and tuner paths)
  Ctl* h_ctl = nullptr;
  Range* h_ranges = nullptr;

  // autotuned choices per slice shape (nx, ny): resident variant and the
  // two-launch tile sizes (0: default)
  struct Tuned {
    int res_variant = 0;
    int rows = 0, cols = 0;
    int plan_x = 0, plan_y = 0;   // pass plans of the row (nx) and column (ny) transforms
  };
  std::map<std::pair<int, int>, Tuned> tuned;
  std::string tune_cache;      // file of the choices ("" = none)
  // shapes whose resident launch gave up at a team barrier: the two-launch
  // path only from then on (until pd_tune_set picks a resident variant
  // again).  Read and written under exec_mu.
  std::set<std::pair<int, int>> no_resident;
  unsigned spin_limit = kSpinLimit;   // resident barriers' polls before giving up
  void* scratch = nullptr;     // device address of this device's static scratch (pd_apply_kernel_noalloc)
  int multi_cap = 0;           // workgroups of the multi-shape resident launch one XCD holds at once
  int64_t aborted_rounds = 0, restarted_requests = 0;   // under exec_mu

  // captured step graphs of the two-launch path, keyed by launch plan
  struct GraphEntry {
    hipGraphExec_t exec = nullptr;
    int seen = 0;
    uint64_t last_use = 0;
  };
  std::map<std::string, GraphEntry> graphs;
  uint64_t graph_clock = 0;
  int64_t graph_replays = 0, graph_captures = 0;

  // kernel timing
  bool time_kernels = false;
  std::mutex tmu;
  static constexpr int kKinds = 8;        // column, row, resident, TV column, TV row, 3-D z transform,
                                          // multi-shape resident, TV resident
  int64_t t_launches[kKinds] = {};
  double t_ms[kKinds] = {};
  double t_points[kKinds] = {};           // iterations x slice-pair points processed
  std::vector<hipEvent_t> ev_pool;
};

namespace {

bool hip_ok(pd_ctx* c, hipError_t e) {
  if (e == hipSuccess) return true;
  c->poisoned = PD_ERR_HIP;
  return false;
}

// Every entry point that uses a context counts itself in for its whole
// duration, so pd_destroy, which may run on another thread, frees the
// context only after the calls already inside have left.  A call that
// arrives once pd_destroy has begun is refused (ok == false).
struct CallGuard {
  pd_ctx* c;
  bool ok;
  explicit CallGuard(pd_ctx* cc) : c(cc) {
    std::lock_guard<std::mutex> lk(c->mu);
    ok = !c->stopping;
    if (ok) ++c->calls;
  }
  ~CallGuard() {
    if (!ok) return;
    std::lock_guard<std::mutex> lk(c->mu);
    if (--c->calls == 0) c->cv_idle.notify_all();
  }
  CallGuard(const CallGuard&) = delete;
  CallGuard& operator=(const CallGuard&) = delete;
};

// Tables whose last user has retired stay in the arena (uploaded), so the
// next request of that kernel shape starts without rebuilding them; they are
// evicted, least recently used first, when an allocation needs the space.
// Caller holds c->mu.  Returns false if no unused table is left.
bool evict_unused_table(pd_ctx* c) {
  auto victim = c->tables.end();
  for (auto it = c->tables.begin(); it != c->tables.end(); ++it)
    if (it->second.refs == 0 && (victim == c->tables.end() || it->second.last_use < victim->second.last_use))
      victim = it;
  if (victim == c->tables.end()) return false;
  c->arena.release(victim->second.off, victim->second.bytes);
  c->tables.erase(victim);
  return true;
}

// Arena allocation that evicts unused tables while it does not fit.
bool arena_alloc(pd_ctx* c, size_t bytes, size_t* off) {
  while (!c->arena.alloc(bytes, off))
    if (!evict_unused_table(c)) return false;
  return true;
}

// Device pointers of a shape's table laid out from p: D grid, then the
// twiddles of x, y (and z), each 256-byte aligned (table_bytes in total).
void table_ptrs(Table& t, char* p, const TableKey& k, int precision) {
  const size_t tsz = precision == PD_FP64 ? 8 : 4;
  t.d = p;
  t.twx = p + align_up((size_t)k.nx * k.ny * std::max(k.nz3, 1) * tsz);
  t.twy = (char*)t.twx + align_up(axis_tw_entries(k.nx) * 2 * tsz);
  t.twz = k.nz3 > 1 ? (char*)t.twy + align_up(axis_tw_entries(k.ny) * 2 * tsz) : nullptr;
}

// Acquire (or share) the table of a shape; caller holds c->mu.
Table* acquire_table(pd_ctx* c, const TableKey& k, bool* fresh) {
  auto it = c->tables.find(k);
  if (it != c->tables.end()) {
    it->second.refs++;
    it->second.last_use = ++c->table_clock;
    *fresh = false;
    return &it->second;
  }
  Table t;
  t.bytes = table_bytes(k.nx, k.ny, k.nz3, c->precision);
  if (!arena_alloc(c, t.bytes, &t.off)) return nullptr;
  t.last_use = ++c->table_clock;
  table_ptrs(t, c->arena.ptr(t.off), k, c->precision);
  t.refs = 1;
  t.uploaded = false;
  *fresh = true;
  return &(c->tables[k] = t);
}

void release_table(pd_ctx* c, const TableKey& k) {
  auto it = c->tables.find(k);
  if (it == c->tables.end()) return;
  --it->second.refs;   // at zero the table stays cached (evict_unused_table)
}

template <typename T>
hipError_t upload_table(pd_ctx* c, const TableKey& k, const Table& t) {
  std::vector<double> re, im;
  std::vector<T> hd;
  if (k.nz3 > 1) {
    hd.resize((size_t)k.nx * k.ny * k.nz3);
    dipole_grid3(k.nx, k.ny, k.nz3, k.b, k.vox, k.vz, [&](size_t i, double d) { hd[i] = (T)d; });
  } else {
    std::vector<double> D;
    dipole_grid(k.nx, k.ny, k.b, k.vox, k.kernel, D);
    hd.resize(D.size());
    for (size_t i = 0; i < D.size(); ++i) hd[i] = (T)D[i];
  }
  hipError_t e = hipMemcpyAsync(t.d, hd.data(), hd.size() * sizeof(T), hipMemcpyHostToDevice, c->stream);
  if (e != hipSuccess) return e;
  std::vector<std::vector<T>> tws(3);
  for (int axis = 0; axis < (k.nz3 > 1 ? 3 : 2); ++axis) {
    int n = axis == 0 ? k.nx : axis == 1 ? k.ny : k.nz3;
    std::vector<T>& tw = tws[axis];
    if (!axis_blue(n)) {
      twiddles(n, re, im);
      tw.resize(2 * (size_t)n);
      for (int m = 0; m < n; ++m) {
        tw[2 * m] = (T)re[m];
        tw[2 * m + 1] = (T)im[m];
      }
    } else {
      std::vector<double> all;
      bluestein_table(n, blue_len(n), all);
      tw.resize(all.size());
      for (size_t m = 0; m < all.size(); ++m) tw[m] = (T)all[m];
    }
    e = hipMemcpyAsync(axis == 0 ? t.twx : axis == 1 ? t.twy : t.twz, tw.data(), tw.size() * sizeof(T),
                       hipMemcpyHostToDevice, c->stream);
    if (e != hipSuccess) return e;
  }
  // the host vectors die on return: wait for the copies
  return hipStreamSynchronize(c->stream);
}

TableKey key_of(const pd_request& r) {
  TableKey k{};
  k.nx = r.nx;
  k.ny = r.ny;
  k.kernel = r.kernel;
  k.nz3 = nz3_of(r);
  k.vz = k.nz3 ? r.voxel_z : 0.0;
  if (r.kernel != PD_KERNEL_IDENTITY) {
    unit_b0(r.b0, k.b);
  } else {
    k.b[0] = k.b[1] = k.b[2] = 0.0;
  }
  if (r.kernel != PD_KERNEL_IDENTITY) {
    k.vox[0] = r.voxel[0];
    k.vox[1] = r.voxel[1];
  } else {
    k.vox[0] = k.vox[1] = 0.0;
  }
  return k;
}

// Fill the kernel descriptor of a resident job (host mirror).
void fill_vol(pd_ctx* c, const Job& j, Vol& V) {
  std::memset(&V, 0, sizeof(V));
  const Table& t = j.tab;
  char* base = c->arena.ptr(j.off);
  V.chi = base + j.L.off_chi;
  V.yhat = base + j.L.off_yhat;
  V.dhat = base + j.L.off_dhat;
  V.ex = base + j.L.off_ex;
  V.ex2 = base + j.L.off_ex2;
  V.dtab = t.d;
  V.twx = t.twx;
  V.twy = t.twy;
  V.part_row = (double*)(base + j.L.off_prow);
  V.part_col = (double*)(base + j.L.off_pcol);
  V.user_in = j.req.delta;
  V.user_out = j.req.chi;
  V.tau = j.req.tau;
  V.sigma = j.req.sigma;
  V.lam = j.req.lambda;
  V.theta = j.req.theta;
  V.gap_tol = j.req.gap_tol;
  V.nx = j.req.nx;
  V.ny = j.req.ny;
  V.nz = j.req.nz;
  V.P = j.L.P;
  V.half_last = j.req.nz & 1;
  V.max_iter = j.req.max_iter;
  V.row_groups = j.L.row_groups;
  V.col_groups = j.L.col_groups;
  V.final_it = -1;
  V.model = j.req.model;
  if (j.L.tv) {
    V.chibar = base + j.L.off_chibar;
    V.pdual = base + j.L.off_p;
    V.qx = base + j.L.off_qx;
    V.qy = base + j.L.off_qy;
    if (j.L.tv3) {
      V.qz = base + j.L.off_qz;
      V.tv3 = 1;
      V.inv_dz = 1.0 / j.req.voxel_z;
    }
    V.wgt = base + j.L.off_w;
    V.msk = base + j.L.off_m;
    V.dpk = base + j.L.off_d;
    V.user_w = j.req.weight;
    V.user_m = j.req.mask;
    V.yhat = V.dhat = nullptr;
    V.part_row = V.part_col = nullptr;
  }
  V.inv_dx = 1.0 / j.req.voxel[0];
  V.inv_dy = 1.0 / j.req.voxel[1];
  V.knorm = j.knorm;
  V.unpacked = j.L.unpacked ? 1 : 0;
  if (j.L.unpacked) V.half_last = 0;
  V.gap_norm = 1.0 / ((double)j.req.nx * (double)j.req.ny * (j.L.unpacked ? (double)j.req.nz : 1.0));
  V.col_parts = j.L.unpacked ? j.L.zgroups : V.P * V.col_groups;
}

// The 3-D kernel's z view of a volume: the [nz][ny][nx] planes read as one
// slice of nz rows by nx ny columns, so the column kernel transforms along z
// (D table [nz][ny nx], twiddles of z).  Same buffers and controls as V.
void fill_zvol(const Job& j, const Vol& V, Vol& Z) {
  Z = V;
  Z.nx = j.req.nx * j.req.ny;
  Z.ny = j.req.nz;
  Z.P = 1;
  Z.half_last = 0;
  Z.unpacked = 0;
  Z.twx = nullptr;
  Z.twy = j.tab.twz;
  Z.row_groups = 0;
  Z.col_groups = j.L.zgroups;
}

// Reserve arena + slot for a queued job; caller holds c->mu.  Returns false
// if it does not fit now.
bool reserve(pd_ctx* c, Job& j) {
  if (c->free_slots.empty()) return false;
  size_t off;
  if (!arena_alloc(c, j.L.total, &off)) return false;
  bool fresh = false;
  Table* t = acquire_table(c, j.key, &fresh);
  if (!t) {
    c->arena.release(off, j.L.total);
    return false;
  }
  (void)fresh;
  j.off = off;
  j.tab = *t;
  j.slot = c->free_slots.back();
  c->free_slots.pop_back();
  return true;
}

void unreserve(pd_ctx* c, Job& j) {
  c->arena.release(j.off, j.L.total);
  release_table(c, j.key);
  if (j.slot >= 0 && j.slot < c->nslots) c->free_slots.push_back(j.slot);
  j.slot = -1;
}

hipEvent_t get_event(pd_ctx* c) {
  if (!c->ev_pool.empty()) {
    hipEvent_t e = c->ev_pool.back();
    c->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

void free_host(pd_ctx* c) {
  if (c->h_vols) (void)hipHostFree(c->h_vols);
  if (c->h_ctl) (void)hipHostFree(c->h_ctl);   // holds h_abort too
  if (c->h_ranges) (void)hipHostFree(c->h_ranges);
  for (char*& b : c->h_stage)
    if (b) (void)hipHostFree(b);
  c->h_vols = nullptr;
  c->h_ctl = nullptr;
  c->h_ranges = nullptr;
  c->h_abort = nullptr;
}

// ---------------------------------------------------------------------------
// set-up of a newly admitted job: zero state, F delta, zero partials
// ---------------------------------------------------------------------------
hipError_t setup_job(pd_ctx* c, Job& j) {
  Vol& V = c->h_vols[j.slot];
  fill_vol(c, j, V);
  hipError_t e = hipMemcpyAsync(c->d_vols + j.slot, &V, sizeof(Vol), hipMemcpyHostToDevice, c->stream);
  if (e != hipSuccess) return e;
  if (j.L.unpacked || j.L.tv3) {
    Vol& Z = c->h_vols[c->zoff + j.slot];
    fill_zvol(j, V, Z);
    if ((e = hipMemcpyAsync(c->d_vols + c->zoff + j.slot, &Z, sizeof(Vol), hipMemcpyHostToDevice, c->stream)) !=
        hipSuccess)
      return e;
  }
  char* base = c->arena.ptr(j.off);
  if ((e = launch_zero(base, j.L.total, c->stream)) != hipSuccess) return e;
  if ((e = launch_zero(c->d_ctl + j.slot, sizeof(Ctl), c->stream)) != hipSuccess) return e;
  return hipSuccess;
}

// Launch the transform set-up (F delta -> dhat) for the given jobs, whose Vol
// entries are already on the device.
hipError_t launch_setup(pd_ctx* c, const std::vector<Job*>& js) {
  hipError_t e;
  for (size_t k = 0; k < js.size(); ++k) c->h_ranges[k] = Range{js[k]->slot, 0, 0, 0};
  if ((e = hipMemcpyAsync(c->d_ranges, c->h_ranges, js.size() * sizeof(Range), hipMemcpyHostToDevice,
                          c->stream)) != hipSuccess)
    return e;
  for (size_t k = 0; k < js.size(); ++k) {
    Job* j = js[k];
    const Range* rg = c->d_ranges + k;
    int P = j->L.P;
    if (j->L.tv) {   // pack W, M, delta; step condition on the device
      e = launch_tv_setup(c->d_vols, c->d_ctl, j->slot, (size_t)P * j->req.nx * j->req.ny, c->precision, c->stream);
      if (e != hipSuccess) return e;
      continue;
    }
    // F_x of delta's rows -> ex, then F_y of ex's columns -> dhat
    e = launch_row(axis_phys(j->req.nx), ROW_FWD_PLANAR, j->L.rows, P * j->L.row_groups, j->L.row_groups, c->d_vols,
                   rg, 1, c->d_ctl, 0, c->precision, j->L.ext_row, c->stream);
    if (e != hipSuccess) return e;
    if (j->L.unpacked) {   // 3-D kernel: F_y in place, then F_z of the z view -> dhat
      e = launch_col(axis_phys(j->req.ny), COL_FWD, j->L.cols, P * j->L.col_groups, j->L.col_groups, c->d_vols, rg,
                     1, c->d_ctl, -1, c->precision, j->L.ext_col, c->stream);
      if (e != hipSuccess) return e;
      e = launch_col(axis_phys(j->req.nz), COL_SETUP, j->L.zcols, j->L.zgroups, j->L.zgroups, c->d_vols + c->zoff, rg, 1,
                     c->d_ctl, 0, c->precision, j->L.ext_z, c->stream);
      if (e != hipSuccess) return e;
      e = launch_zero(c->arena.ptr(j->off) + j->L.off_ex, j->L.field, c->stream);
      if (e != hipSuccess) return e;
      continue;
    }
    e = launch_col(axis_phys(j->req.ny), COL_SETUP, j->L.cols, P * j->L.col_groups, j->L.col_groups, c->d_vols,
                   rg, 1, c->d_ctl, 0, c->precision, j->L.ext_col, c->stream);
    if (e != hipSuccess) return e;
    // X'_0 = F_x chibar_0 = 0
    e = launch_zero(c->arena.ptr(j->off) + j->L.off_ex, j->L.field, c->stream);
    if (e != hipSuccess) return e;
  }
  // the pinned range array is reused by the step: wait for the copy
  return hipStreamSynchronize(c->stream);
}

// A failed HIP call of a step, named on stderr when PD_DEBUG is set
// (diagnostics only: the request's status reports PD_ERR_HIP).
inline hipError_t step_err(const char* what, hipError_t e) {
  if (e != hipSuccess && std::getenv("PD_DEBUG")) std::fprintf(stderr, "pd: %s: %s\n", what, hipGetErrorName(e));
  return e;
}

// HIP events of timed launches, read back after a round
struct StepEvents {
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> evs;
  std::vector<double> points;
};

// One scheduling step over all resident jobs: K iterations for every job,
// where K ends the step at every job's next gap check (or its last
// iteration), so checks and stop decisions only happen at step ends.  Each
// job starts the step at done_iters + run_iters (the steps already enqueued
// in this round).  The step's descriptors, slot list and range table are
// written to the pinned image `stage` and uploaded in one copy.  `last`: some
// job runs its last iteration (or only its check) in this step.
hipError_t enqueue_step(pd_ctx* c, std::vector<std::shared_ptr<Job>>& act, bool queued, char* stage,
                        StepEvents& tev, int& K_out, bool& last) {
  int K = c->cfg.step_iters > 0 ? c->cfg.step_iters : (queued ? kQueuedStep : kDefaultStep);
  Vol* s_vols = (Vol*)stage;
  int* s_slots = (int*)(stage + c->off_slots);
  Range* s_ranges = (Range*)(stage + c->off_ranges);
  bool any_check_only = false;
  for (auto& j : act) {
    if (j->req.max_iter == 0) {
      any_check_only |= !j->L.tv;   // a TV volume with no iteration just retires
      continue;
    }
    const int done = j->done_iters + j->run_iters;
    int rem = j->req.max_iter - done;
    int nc = j->req.gap_tol > 0 ? j->req.check_every - done % j->req.check_every : rem;
    K = std::min(K, std::min(rem, nc));
  }
  if (any_check_only) K = 1;
  K = std::max(K, 1);

  // descriptors
  std::map<GroupKey, std::vector<Job*>> groups;
  int nslot_list = 0;
  bool any_check = false;
  last = false;
  for (auto& j : act) {
    groups[GroupKey{j->req.nx, j->req.ny, j->req.model, nz3_of(j->req)}].push_back(j.get());
    Vol& V = c->h_vols[j->slot];
    fill_vol(c, *j, V);
    const int done = j->done_iters + j->run_iters;
    if (j->L.tv) {                  // fixed iteration count, no gap checks
      int rem = j->req.max_iter - done;
      V.iters = std::min(K, rem);
      V.done_base = done;
      V.final_it = (rem == V.iters) ? V.iters - 1 : -1;
      V.check_last = 0;
    } else if (j->req.max_iter == 0) {     // check-only step: gap of chi_0 = 0, y_0 = 0
      V.iters = 1;
      V.done_base = -1;
      V.final_it = 0;
      V.check_last = 1;
      V.check_only = 1;
    } else {
      int rem = j->req.max_iter - done;
      V.iters = std::min(K, rem);
      V.done_base = done;
      V.final_it = (rem == V.iters) ? V.iters - 1 : -1;
      int n = done + V.iters;
      V.check_last = (j->req.gap_tol > 0 && n % j->req.check_every == 0) || n == j->req.max_iter;
    }
    last |= V.final_it >= 0 || V.iters <= 0;
    any_check |= V.check_last != 0;
    s_slots[nslot_list++] = j->slot;
  }

  // launch plan: per shape either one resident launch per batch of pairs that
  // can be co-resident, or K x (column, row) launches covering every pair
  struct Launch {
    int nx, ny, rows, cols, rg, cg;
    bool resident;
    bool tv;                                 // weighted TV model (four launches per iteration)
    int px, py, er, ec;                      // transform lengths and kernel variants (row, column)
    int planx, plany;                        // pass plans of the row and column transforms
    bool z3;                                 // 3-D kernel: planes plus the z view
    int pz, ez, zg, zc, z_off, nzr;          // z: transform length, variant, groups per volume, strip, ranges
    int team;
    const ResidentVariant* rv;
    bool multi;                              // multi-shape resident launch (team table at range_off)
    int quota, nteams;                       // multi: workgroups per XCD, teams
    double multi_pts;                        // multi: slice-pair points of all its teams
    int range_off, nranges, npairs;          // resident: one range table
    int row_off, col_off;                    // two-launch path: row and column tables
    int ncolp;                               // two-launch path: planes of the column launches
  };
  std::vector<Launch> launches;
  size_t k = 0;
  auto push_range = [&](int slot, int first, int pair0) -> bool {
    if (k + 1 >= c->range_cap) return false;
    s_ranges[k++] = Range{slot, first, pair0, 0};
    return true;
  };
  bool fits = true;
  // The shape's chosen resident variant, or null for the two-launch path.
  auto chosen_rv = [&](const GroupKey& gk) -> const ResidentVariant* {
    const int nx = gk.nx, ny = gk.ny;
    const pd_ctx::Tuned tn = c->tuned.count({nx, ny}) ? c->tuned[{nx, ny}] : pd_ctx::Tuned{};
    return (c->precision == PD_FP32 && !(c->cfg.flags & PD_FLAG_NO_RESIDENT) && nx == ny && !any_check_only &&
            gk.model != PD_MODEL_TV && gk.nz3 == 0 && !c->no_resident.count({nx, ny}))
               ? resident_variant(nx, tn.res_variant)
               : nullptr;
  };
  // The TV model's resident launch for a 2-D TV group, or null for its
  // four-launch path.
  auto tv_rv = [&](const GroupKey& gk) -> const ResidentVariant* {
    return (c->precision == PD_FP32 && !(c->cfg.flags & PD_FLAG_NO_RESIDENT) && gk.nx == gk.ny &&
            gk.model == PD_MODEL_TV && gk.nz3 == 0 && !c->no_resident.count({gk.nx, gk.ny}))
               ? resident_tv_variant(gk.nx)
               : nullptr;
  };
  // Several resident shapes whose chosen variants' (shape, FFT plan) is a
  // body of the multi-shape launch share it (a body gives the same bits as
  // every variant of its plan), if their teams fit the range table.
  std::vector<Job*> multi_jobs;
  std::vector<int> multi_plan;   // FFT plan of each multi job's chosen variant
  const int multi_cap = c->multi_cap;
  {
    int shapes = 0;
    size_t entries = 0;
    for (auto& g : groups) {
      const ResidentVariant* rv = chosen_rv(g.first);
      if (!rv || multi_body(g.first.nx, rv->plan()) < 0 || multi_cap < multi_team(g.first.nx, rv->plan())) continue;
      ++shapes;
      for (Job* j : g.second) entries += (size_t)j->L.P;
    }
    // range entries: each team one, each launch (at most one per team)
    // kXcds + 1 headers, every other job at most four
    if (shapes >= 2 && entries * (kXcds + 2) + 4 * act.size() + 16 <= c->range_cap)
      for (auto& g : groups) {
        const ResidentVariant* rv = chosen_rv(g.first);
        if (!rv || multi_body(g.first.nx, rv->plan()) < 0 || multi_cap < multi_team(g.first.nx, rv->plan())) continue;
        for (Job* j : g.second) {
          multi_jobs.push_back(j);
          multi_plan.push_back(rv->plan());
        }
      }
  }
  for (auto& g : groups) {
    int nx = g.first.nx, ny = g.first.ny;
    const pd_ctx::Tuned tn = c->tuned.count({nx, ny}) ? c->tuned[{nx, ny}] : pd_ctx::Tuned{};
    const bool tv = g.first.model == PD_MODEL_TV;
    const bool z3 = g.first.nz3 > 0;
    if (!multi_jobs.empty() && std::find(multi_jobs.begin(), multi_jobs.end(), g.second.front()) != multi_jobs.end())
      continue;   // in the multi-shape launches below
    const ResidentVariant* rv = tv ? tv_rv(g.first) : chosen_rv(g.first);
    int maxt = rv ? std::min(rv->max_teams(), kMaxTeamSlots) : 0;
    if (rv && !tv) {
      // the chosen variant was timed at some slice count; when this step's
      // pairs need more than one of its co-resident launches, take the
      // variant of the same FFT plan with the most co-resident teams instead
      // (variants of one plan give the same bits, so a request's iterates do
      // not depend on the other requests of the step)
      int npairs = 0;
      for (Job* j : g.second) npairs += j->L.P;
      if (npairs > maxt)
        for (int v = 0; v < resident_variant_count(nx); ++v) {
          const ResidentVariant* cand = resident_variant(nx, v);
          if (cand->plan() != rv->plan()) continue;
          const int m = std::min(cand->max_teams(), kMaxTeamSlots);
          if (m > maxt) {
            rv = cand;
            maxt = m;
          }
        }
    }
    int team = rv ? rv->team() : 0;
    if (team && maxt > 0) {
      // split the shape's pairs into co-resident batches
      Launch L{};
      L.nx = nx;
      L.ny = ny;
      L.resident = true;
      L.tv = tv;
      L.team = team;
      L.rv = rv;
      L.range_off = (int)k;
      for (Job* j : g.second) {
        j->in_resident = true;
        int p = 0;
        while (p < j->L.P) {
          if (L.npairs == maxt) {
            L.nranges = (int)k - L.range_off;
            launches.push_back(L);
            L.range_off = (int)k;
            L.npairs = 0;
          }
          int take = std::min(j->L.P - p, maxt - L.npairs);
          fits &= push_range(j->slot, L.npairs * team, p);
          L.npairs += take;
          p += take;
        }
      }
      L.nranges = (int)k - L.range_off;
      if (L.npairs > 0) launches.push_back(L);
    } else {
      Launch L{};
      L.nx = nx;
      L.ny = ny;
      L.resident = false;
      L.tv = tv;
      L.row_off = (int)k;
      int np = 0;
      L.rows = rows_valid(tn.rows, nx, ny, c->precision) ? tn.rows : rows_per_wg(nx, ny, c->precision);
      L.cols = cols_valid(tn.cols, nx, ny, c->precision) ? tn.cols : cols_per_wg(nx, ny, c->precision);
      L.rg = ceil_div(ny, L.rows);
      L.cg = ceil_div(nx, L.cols);
      L.px = axis_phys(nx);
      L.py = axis_phys(ny);
      L.er = axis_ext(nx, ny, L.rows);
      L.ec = axis_ext(ny, nx, L.cols);
      // a tuned pass plan applies to FP32 whole-tile transforms of the L1
      // iteration; everything else runs the default plan
      const bool plain = c->precision == PD_FP32 && !tv && !z3;
      L.planx = (plain && L.er == 0 && tn.plan_x < plan_count(nx)) ? tn.plan_x : 0;
      L.plany = (plain && L.ec == 0 && tn.plan_y < plan_count(ny)) ? tn.plan_y : 0;
      for (Job* j : g.second) {
        Vol& V = c->h_vols[j->slot];
        V.row_groups = L.rg;
        V.col_groups = L.cg;
        fits &= push_range(j->slot, np * L.rg, 0);
        np += j->L.P;
      }
      L.npairs = np;
      L.nranges = (int)g.second.size();
      L.col_off = (int)k;
      np = 0;
      for (Job* j : g.second) {   // column launches run over the exchange planes
        fits &= push_range(j->slot, np * L.cg, 0);
        np += j->L.planes;
      }
      L.ncolp = np;
      if (z3) {   // one z-view range per volume
        Job* j0 = g.second.front();
        L.z3 = true;
        L.zg = j0->L.zgroups;
        L.zc = j0->L.zcols;
        L.pz = axis_phys(j0->req.nz);
        L.ez = j0->L.ext_z;
        L.z_off = (int)k;
        int nv = 0;
        for (Job* j : g.second) {
          fits &= push_range(j->slot, nv * L.zg, 0);
          ++nv;
        }
        L.nzr = nv;
      }
      launches.push_back(L);
    }
  }
  if (!multi_jobs.empty()) {
    // Multi-shape launches: every pair of the jobs is one team of its shape's
    // body; teams go to the least loaded XCD of the current launch (largest
    // teams first), and a team that no XCD of it can take opens the next
    // launch.  Each XCD's teams then get consecutive ticket ranges.
    struct TeamRec {
      int slot, pair, body, size, xcd;
    };
    std::vector<TeamRec> recs;
    for (size_t ji = 0; ji < multi_jobs.size(); ++ji) {
      Job* j = multi_jobs[ji];
      const int sz = multi_team(j->req.nx, multi_plan[ji]);
      const int body = multi_body(j->req.nx, multi_plan[ji]);
      for (int p = 0; p < j->L.P; ++p) recs.push_back(TeamRec{j->slot, p, body, sz, -1});
      j->in_resident = true;
      Vol& V = c->h_vols[j->slot];
      V.row_groups = V.col_groups = sz;
    }
    std::stable_sort(recs.begin(), recs.end(), [](const TeamRec& a, const TeamRec& b) { return a.size > b.size; });
    std::vector<std::vector<TeamRec>> per_launch(1);
    std::vector<std::array<int, kXcds>> load(1);
    load[0].fill(0);
    for (TeamRec t : recs) {
      auto& ld = load.back();
      int x = (int)(std::min_element(ld.begin(), ld.end()) - ld.begin());
      if (ld[x] + t.size > multi_cap) {
        per_launch.emplace_back();
        load.emplace_back();
        load.back().fill(0);
        x = 0;
      }
      t.xcd = x;
      load.back()[x] += t.size;
      per_launch.back().push_back(t);
    }
    for (size_t li = 0; li < per_launch.size(); ++li) {
      auto& ts = per_launch[li];
      std::stable_sort(ts.begin(), ts.end(), [](const TeamRec& a, const TeamRec& b) { return a.xcd < b.xcd; });
      Launch L{};
      L.nx = L.ny = 0;
      L.resident = true;
      L.multi = true;
      L.range_off = (int)k;
      L.nteams = (int)ts.size();
      L.quota = *std::max_element(load[li].begin(), load[li].end());
      // header: index of each XCD's first team, then the team count
      if (k + kXcds + 1 + ts.size() >= c->range_cap) {
        fits = false;
        break;
      }
      int ti = 0;
      for (int x = 0; x <= kXcds; ++x) {
        while (ti < (int)ts.size() && ts[ti].xcd < x) ++ti;
        s_ranges[k++] = Range{-1, ti, 0, 0};
      }
      int ticket = 0, prev = -1;
      double pts = 0.0;
      for (auto& t : ts) {
        if (t.xcd != prev) {
          ticket = 0;
          prev = t.xcd;
        }
        s_ranges[k++] = Range{t.slot, ticket, t.pair, t.body};
        ticket += t.size;
        pts += (double)c->h_vols[t.slot].nx * c->h_vols[t.slot].ny;
      }
      L.npairs = L.nteams;
      L.multi_pts = pts;
      launches.push_back(L);
    }
  }
  if (!fits) return hipErrorOutOfMemory;   // range table too small: cannot happen with range_cap
  // resident launches report gap partials per team member
  for (auto& L : launches)
    if (L.resident && !L.multi)
      for (int i = 0; i < L.nranges; ++i) {
        Vol& V = c->h_vols[s_ranges[L.range_off + i].slot];
        V.row_groups = V.col_groups = L.team;
      }
  for (auto& j : act) {
    Vol& V = c->h_vols[j->slot];
    V.col_parts = j->L.unpacked ? j->L.zgroups : V.P * V.col_groups;
    s_vols[j->slot] = V;
    if (j->L.unpacked || j->L.tv3) {
      fill_zvol(*j, V, c->h_vols[c->zoff + j->slot]);
      s_vols[c->zoff + j->slot] = c->h_vols[c->zoff + j->slot];
    }
    j->run_iters += std::max(V.iters, 0);
  }
  K_out = K;

  // descriptors of idle slots in the image are stale: no launch of this
  // step reads them (ranges and the slot list name active jobs only)
  hipError_t e;
  if ((e = hipMemcpyAsync(c->d_vols, stage, c->off_ranges + sizeof(Range) * k, hipMemcpyHostToDevice,
                          c->stream)) != hipSuccess)
    return e;

  auto& evs = tev.evs;
  auto& ev_points = tev.points;
  auto timed = [&](int kind, double points, auto&& fn) -> hipError_t {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (c->time_kernels) {
      e0 = get_event(c);
      e1 = get_event(c);
      if (e0) (void)hipEventRecord(e0, c->stream);
    }
    hipError_t r = fn();
    if (c->time_kernels && e0 && e1) {
      (void)hipEventRecord(e1, c->stream);
      evs.push_back({kind, {e0, e1}});
      ev_points.push_back(points);
    }
    return r;
  };

  // The step's launches: resident launches first (each runs all K iterations
  // of its pairs), then the two-launch path (K iterations of column and row
  // launches), then the checks.  Replayed from a captured graph when the same
  // plan recurs.
  bool any_two = false, any_res = false;
  for (auto& L : launches) {
    any_two |= !L.resident;
    any_res |= L.resident;
  }
  const int fenced = (c->cfg.flags & PD_FLAG_FENCED_EXCHANGE) ? 1 : 0;
  auto enqueue_resident = [&](bool with_events) -> hipError_t {
    for (auto& L : launches) {
      if (!L.resident) continue;
      if (L.multi) {
        // team counters, then the per-XCD tickets and the grid arrival counter
        const int ticket_base = (L.nteams + kXcds - 1) / kXcds * kXcds;
        hipError_t r = launch_zero(c->d_counters, align_up(counter_bytes((size_t)ticket_base)), c->stream);
        if (r != hipSuccess) return r;
        auto res = [&] {
          return launch_resident_multi(L.quota, c->d_vols, c->d_ranges + L.range_off, c->d_ctl, c->d_counters,
                                       c->d_abort, ticket_base, fenced, c->spin_limit, c->stream);
        };
        r = with_events ? timed(6, L.multi_pts * K, res) : res();
        if (r != hipSuccess) return r;
        continue;
      }
      // team counters of every team slot of the launch (rounds of 8 teams),
      // then the per-XCD tickets and the grid arrival counter
      const size_t slots_ = (size_t)((L.npairs + kXcds - 1) / kXcds) * kXcds;
      hipError_t r = launch_zero(c->d_counters, align_up(counter_bytes(slots_)), c->stream);
      if (r != hipSuccess) return r;
      const Range* rr = c->d_ranges + L.range_off;
      double pts = (double)L.npairs * L.nx * L.ny * K;
      auto res = [&] {
        return L.rv->launch(L.npairs, c->d_vols, rr, L.nranges, c->d_ctl, c->d_counters, c->d_abort, fenced,
                            c->spin_limit, c->stream);
      };
      r = with_events ? timed(L.tv ? 7 : 2, pts, res) : res();
      if (r != hipSuccess) return r;
    }
    return hipSuccess;
  };
  auto enqueue_rest = [&](bool with_events) -> hipError_t {
    hipError_t r = enqueue_resident(with_events);
    if (r != hipSuccess) return r;
    if (any_two) {
      for (int it = 0; it < K; ++it) {
        for (auto& L : launches) {
          if (L.resident) continue;
          const Range* rrow = c->d_ranges + L.row_off;
          const Range* rcol = c->d_ranges + L.col_off;
          double pts = (double)L.npairs * L.nx * L.ny;
          auto col = [&] {
            return launch_col_p(L.py, COL_ITER, L.cols, L.ncolp * L.cg, L.cg, c->d_vols, rcol, L.nranges, c->d_ctl,
                                it, c->precision, L.ec, L.plany, c->stream);
          };
          auto row = [&] {
            return launch_row_p(L.px, ROW_ITER, L.rows, L.npairs * L.rg, L.rg, c->d_vols, rrow, L.nranges, c->d_ctl,
                                it, c->precision, L.er, L.planx, c->stream);
          };
          if (L.tv && L.z3) {
            // TV model in three dimensions, per half iteration: F_y per plane,
            // (F_z, D / (nx ny nz), F_z^-1) on the z view, F_y^-1 per plane,
            // then the dual or primal row kernel over the pairs
            const Range* rz = c->d_ranges + L.z_off;
            auto cfwd = [&] {
              return launch_col(L.py, COL_FWD, L.cols, L.ncolp * L.cg, L.cg, c->d_vols, rcol, L.nranges, c->d_ctl,
                                it, c->precision, L.ec, c->stream);
            };
            auto zk = [&] {
              return launch_col(L.pz, COL_TV, L.zc, L.nzr * L.zg, L.zg, c->d_vols + c->zoff, rz, L.nzr, c->d_ctl, it,
                                c->precision, L.ez, c->stream);
            };
            auto cinv = [&] {
              return launch_col(L.py, COL_INV, L.cols, L.ncolp * L.cg, L.cg, c->d_vols, rcol, L.nranges, c->d_ctl,
                                it, c->precision, L.ec, c->stream);
            };
            for (int half = 0; half < 2; ++half) {
              r = with_events ? timed(3, pts, cfwd) : cfwd();
              if (r != hipSuccess) return r;
              r = with_events ? timed(5, pts, zk) : zk();
              if (r != hipSuccess) return r;
              r = with_events ? timed(3, pts, cinv) : cinv();
              if (r != hipSuccess) return r;
              const int mode = half == 0 ? ROW_TV3_DUAL : ROW_TV3_PRIMAL;
              auto rk = [&] {
                return launch_row(L.px, mode, L.rows, L.npairs * L.rg, L.rg, c->d_vols, rrow, L.nranges, c->d_ctl,
                                  it, c->precision, L.er, c->stream);
              };
              r = with_events ? timed(4, pts, rk) : rk();
              if (r != hipSuccess) return r;
            }
            continue;
          }
          if (L.z3) {   // 3-D kernel: F_y, (F_z, dual prox, F_z^-1) on the z view, F_y^-1, row kernel
            const Range* rz = c->d_ranges + L.z_off;
            auto cfwd = [&] {
              return launch_col(L.py, COL_FWD, L.cols, L.ncolp * L.cg, L.cg, c->d_vols, rcol, L.nranges, c->d_ctl,
                                it, c->precision, L.ec, c->stream);
            };
            auto zk = [&] {
              return launch_col(L.pz, COL_ITER, L.zc, L.nzr * L.zg, L.zg, c->d_vols + c->zoff, rz, L.nzr, c->d_ctl, it,
                                c->precision, L.ez, c->stream);
            };
            auto cinv = [&] {
              return launch_col(L.py, COL_INV, L.cols, L.ncolp * L.cg, L.cg, c->d_vols, rcol, L.nranges, c->d_ctl,
                                it, c->precision, L.ec, c->stream);
            };
            r = with_events ? timed(0, pts, cfwd) : cfwd();
            if (r != hipSuccess) return r;
            r = with_events ? timed(5, pts, zk) : zk();
            if (r != hipSuccess) return r;
            r = with_events ? timed(0, pts, cinv) : cinv();
            if (r != hipSuccess) return r;
            r = with_events ? timed(1, pts, row) : row();
            if (r != hipSuccess) return r;
            continue;
          }
          if (L.tv) {
            auto col_tv = [&] {
              return launch_col(L.py, COL_TV, L.cols, L.ncolp * L.cg, L.cg, c->d_vols, rcol, L.nranges, c->d_ctl,
                                it, c->precision, L.ec, c->stream);
            };
            auto row_tv = [&](int mode) {
              return [&, mode] {
                return launch_row(L.px, mode, L.rows, L.npairs * L.rg, L.rg, c->d_vols, rrow, L.nranges, c->d_ctl,
                                  it, c->precision, L.er, c->stream);
              };
            };
            for (int half = 0; half < 2; ++half) {
              r = with_events ? timed(3, pts, col_tv) : col_tv();
              if (r != hipSuccess) return r;
              auto rk = row_tv(half == 0 ? ROW_TV_DUAL : ROW_TV_PRIMAL);
              r = with_events ? timed(4, pts, rk) : rk();
              if (r != hipSuccess) return r;
            }
            continue;
          }
          r = with_events ? timed(0, pts, col) : col();
          if (r != hipSuccess) return r;
          r = with_events ? timed(1, pts, row) : row();
          if (r != hipSuccess) return r;
        }
      }
      if (any_check) {
        for (auto& L : launches) {
          if (L.resident || L.tv) continue;
          const Range* rcol = c->d_ranges + L.col_off;
          if (L.z3) {   // F_y of the check buffer in place, then F_z and the partials on the z view
            r = launch_col(L.py, COL_FWD_CHK, L.cols, L.ncolp * L.cg, L.cg, c->d_vols, rcol, L.nranges, c->d_ctl,
                           K - 1, c->precision, L.ec, c->stream);
            if (r != hipSuccess) return r;
            r = launch_col(L.pz, COL_CHECK, L.zc, L.nzr * L.zg, L.zg, c->d_vols + c->zoff, c->d_ranges + L.z_off,
                           L.nzr, c->d_ctl, K - 1, c->precision, L.ez, c->stream);
            if (r != hipSuccess) return r;
            continue;
          }
          r = launch_col_p(L.py, COL_CHECK, L.cols, L.ncolp * L.cg, L.cg, c->d_vols, rcol, L.nranges, c->d_ctl,
                           K - 1, c->precision, L.ec, L.plany, c->stream);
          if (r != hipSuccess) return r;
        }
      }
    }
    if (any_check) {
      // check-only volumes have iters == 1: their reduction runs at it == 0 == K - 1
      r = launch_reduce(nslot_list, c->d_vols, c->d_slots, c->d_ctl, K - 1, c->precision, c->stream);
      if (r != hipSuccess) return r;
    }
    return r;
  };
  bool use_graph = (any_two || any_res) && !c->time_kernels && !(c->cfg.flags & PD_FLAG_NO_GRAPHS);
  if (use_graph) {
    std::string sig = std::to_string(K) + (any_check ? "c" : "n") + std::to_string(nslot_list) + ":" +
                      std::to_string(c->precision);
    for (auto& L : launches) {
      if (L.multi) {
        sig += "|m" + std::to_string(L.quota) + "," + std::to_string(L.nteams) + "," + std::to_string(L.range_off);
        continue;
      }
      if (L.resident) {
        // the variant (its kernel: shape, team, block size and FFT plan) and its arguments
        sig += "|r" + std::string(L.tv ? "tv" : "") + std::to_string(L.nx) + "," + std::to_string(L.rv->team()) + "," +
               std::to_string(L.rv->threads()) + "," + std::to_string(L.rv->plan()) + "," +
               std::to_string(L.npairs) + "," + std::to_string(L.range_off) + "," + std::to_string(L.nranges);
        continue;
      }
      sig += "|" + std::string(L.tv ? "tv" : "l1") + (L.z3 ? "z" + std::to_string(L.pz) + "," + std::to_string(L.zg) + "," +
                                                                std::to_string(L.z_off) + "," + std::to_string(L.nzr) + "," + std::to_string(L.zc)
                                                          : std::string()) +
             std::to_string(L.nx) + "," + std::to_string(L.ny) + "," + std::to_string(L.rows) + "," +
             std::to_string(L.cols) + "," + std::to_string(L.npairs) + "," + std::to_string(L.nranges) + "," +
             std::to_string(L.row_off) + "," + std::to_string(L.col_off) + "," + std::to_string(L.planx) + "," +
             std::to_string(L.plany) + "," + std::to_string(L.ncolp);
    }
    auto& G = c->graphs[sig];
    G.last_use = ++c->graph_clock;
    if (!G.exec && ++G.seen >= 2) {
      // a plan seen before: capture it once, replay it from now on
      hipGraph_t g = nullptr;
      e = hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal);
      if (e != hipSuccess) return e;
      hipError_t ecap = enqueue_rest(false);
      e = hipStreamEndCapture(c->stream, &g);
      if (ecap != hipSuccess) e = ecap;
      if (e == hipSuccess) e = hipGraphInstantiate(&G.exec, g, nullptr, nullptr, 0);
      if (g) (void)hipGraphDestroy(g);
      if (e != hipSuccess) return e;
      c->graph_captures++;
      if (c->graphs.size() > (size_t)kMaxGraphs) {   // evict the least recently used plan
        auto victim = c->graphs.end();
        for (auto it2 = c->graphs.begin(); it2 != c->graphs.end(); ++it2)
          if (it2->second.exec && &it2->second != &G &&
              (victim == c->graphs.end() || it2->second.last_use < victim->second.last_use))
            victim = it2;
        if (victim != c->graphs.end()) {
          (void)hipGraphExecDestroy(victim->second.exec);
          c->graphs.erase(victim);
        }
      }
    }
    if (G.exec) {
      if ((e = step_err("graph launch", hipGraphLaunch(G.exec, c->stream))) != hipSuccess) return e;
      c->graph_replays++;
    } else if ((e = step_err("step kernels", enqueue_rest(false))) != hipSuccess) {
      return e;
    }
  } else if ((e = step_err("step kernels", enqueue_rest(c->time_kernels))) != hipSuccess) {
    return e;
  }
  return hipSuccess;
}

// One scheduling round: steps enqueued back to back (run-ahead, while no
// request waits for admission), then one read-back of every volume's control
// block and one wait.  Returns with run_iters = iterations enqueued per job.
hipError_t run_step(pd_ctx* c, std::vector<std::shared_ptr<Job>>& act, bool queued, bool* aborted) {
  *aborted = false;
  for (auto& j : act) {
    j->run_iters = 0;
    j->in_resident = false;
    j->chi_stored = false;
  }
  StepEvents tev;
  hipError_t e = hipSuccess;
  int total = 0;
  for (int s = 0; s < kRunAhead; ++s) {
    int K = 0;
    bool last = false;
    if ((e = enqueue_step(c, act, queued, c->h_stage[s], tev, K, last)) != hipSuccess) break;
    total += K;
    if (last || queued || total >= kRunAheadIters) break;
  }
  // A job whose last iteration is in this round ends in it, whatever its
  // checks decide on the way (a volume stopped earlier keeps its chi), so
  // its result store goes into the round too, before the one wait: the
  // retirement then needs no second round trip.  (Should the round abort, the
  // restarted request stores its result again when it really ends.)
  for (auto& j : act) {
    if (e != hipSuccess) break;
    if (j->req.max_iter > 0 && j->done_iters + j->run_iters >= j->req.max_iter) {
      e = launch_store_chi(c->d_vols, j->slot, (size_t)j->L.P * j->req.nx * j->req.ny, c->precision, c->stream);
      j->chi_stored = e == hipSuccess;
    }
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(c->h_ctl, c->d_ctl, c->off_abort + sizeof(int), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (!tev.evs.empty()) {
    std::lock_guard<std::mutex> lk(c->tmu);
    for (size_t i = 0; i < tev.evs.size(); ++i) {
      auto& x = tev.evs[i];
      float ms = 0.f;
      if (e == hipSuccess && hipEventElapsedTime(&ms, x.second.first, x.second.second) == hipSuccess) {
        c->t_launches[x.first]++;
        c->t_ms[x.first] += ms;
        c->t_points[x.first] += tev.points[i];
      }
      c->ev_pool.push_back(x.second.first);
      c->ev_pool.push_back(x.second.second);
    }
  }
  if (step_err("round", e) != hipSuccess) return e;
  *aborted = *c->h_abort != 0;   // a team barrier gave up
  return hipSuccess;
}

// Recovery from a resident launch whose team barrier gave up (its
// workgroups were not all co-resident, e.g. while other work held CUs).
// Every resident launch of the round from that one on did nothing, and the
// state of the requests they cover is no longer one consistent iterate, so
// each of those requests restarts from chi_0 = 0 (set-up again from its
// field map, which stays valid until its ticket completes) and its shape
// runs on the two-launch path, which needs no co-residency, from now on.
// The other requests of the round are unaffected.  Caller holds exec_mu.
hipError_t recover_round(pd_ctx* c, std::vector<std::shared_ptr<Job>>& act,
                         std::vector<std::shared_ptr<Job>>& restarted) {
  std::vector<Job*> js;
  for (auto& j : act) {
    if (!j->in_resident) continue;
    c->no_resident.insert({j->req.nx, j->req.ny});
    j->done_iters = 0;
    j->run_iters = 0;
    restarted.push_back(j);
    js.push_back(j.get());
  }
  c->aborted_rounds++;
  c->restarted_requests += (int64_t)js.size();
  if (std::getenv("PD_DEBUG"))
    std::fprintf(stderr, "pd: a resident team barrier gave up; %zu request(s) restart on the two-launch path\n",
                 js.size());
  *c->h_abort = 0;
  hipError_t e = launch_zero(c->d_abort, sizeof(int), c->stream);
  for (Job* j : js)
    if (e == hipSuccess) e = setup_job(c, *j);
  if (e == hipSuccess && !js.empty()) e = launch_setup(c, js);
  return e;
}

void finish_job(pd_ctx* c, Job& j, pd_status st) {
  j.res.status = st;
  j.res.t_submit = j.t_submit;
  j.res.t_start = j.t_start;
  j.res.t_done = now_s();
  j.finished = true;
}

void worker_main(pd_ctx* c) {
  (void)hipSetDevice(c->device);
  std::unique_lock<std::mutex> lk(c->mu);
  while (true) {
    auto has_work = [&] { return c->stopping || !c->queue.empty() || !c->active.empty(); };
    if (!has_work()) {
      // idle: poll the queue length for a short while before sleeping, so a
      // request that arrives soon starts without a thread wake-up
      lk.unlock();
      const double t_idle = now_s();
      while (c->n_queued.load(std::memory_order_acquire) == 0 && now_s() - t_idle < kIdleSpin)
        std::this_thread::yield();
      lk.lock();
      c->cv_work.wait(lk, has_work);
    }
    if (c->stopping) break;
    if (c->poisoned != PD_OK) {
      for (auto& j : c->queue) finish_job(c, *j, c->poisoned);
      for (auto& j : c->active) finish_job(c, *j, c->poisoned);
      c->queue.clear();
      c->n_queued.store(0, std::memory_order_relaxed);
      c->active.clear();
      c->cv_done.notify_all();
      continue;
    }
    // admission, FIFO
    std::vector<std::shared_ptr<Job>> admitted;
    while (!c->queue.empty()) {
      auto j = c->queue.front();
      if (!reserve(c, *j)) break;
      c->queue.pop_front();
      c->n_queued.fetch_sub(1, std::memory_order_relaxed);
      admitted.push_back(j);
    }
    std::vector<std::pair<TableKey, Table>> uploads;
    for (auto& j : admitted) {
      Table& t = c->tables.at(j->key);
      if (!t.uploaded) {
        t.uploaded = true;
        uploads.push_back({j->key, t});
      }
    }
    lk.unlock();

    bool ok = true;
    {
      std::lock_guard<std::mutex> ex(c->exec_mu);
      for (auto& u : uploads) {
        hipError_t e = c->precision == PD_FP64 ? upload_table<double>(c, u.first, u.second)
                                               : upload_table<float>(c, u.first, u.second);
        if (!hip_ok(c, e)) ok = false;
      }
      std::vector<Job*> js;
      for (auto& j : admitted) {
        j->t_start = now_s();
        if (ok && !hip_ok(c, setup_job(c, *j))) ok = false;
        js.push_back(j.get());
      }
      if (ok && !js.empty() && !hip_ok(c, launch_setup(c, js))) ok = false;
    }
    lk.lock();
    for (auto& j : admitted) c->active.push_back(j);
    if (!ok) continue;   // poisoned: next loop turn fails everything
    if (c->active.empty()) continue;
    std::vector<std::shared_ptr<Job>> act = c->active;
    const bool queued = !c->queue.empty();
    lk.unlock();

    hipError_t e;
    std::vector<std::shared_ptr<Job>> retired, restarted;
    {
      std::lock_guard<std::mutex> ex(c->exec_mu);
      bool aborted = false;
      e = run_step(c, act, queued, &aborted);
      if (e == hipSuccess && aborted) e = recover_round(c, act, restarted);
      bool need_sync = false;   // a store launched after the round's wait
      if (e == hipSuccess) {
        for (auto& j : act) {
          if (std::find(restarted.begin(), restarted.end(), j) != restarted.end()) continue;
          const Ctl& C = c->h_ctl[j->slot];
          // the final check always stops a volume; the cap test only guards
          // against a step that could not run it
          if (C.stop || ((j->req.max_iter > 0 || j->L.tv) && j->done_iters + j->run_iters >= j->req.max_iter)) {
            j->res.iterations = C.stop ? C.stop_iter : j->done_iters + j->run_iters;
            if (j->L.tv) {   // no duality gap is defined for the TV model
              j->res.primal = j->res.dual = j->res.rel_gap = std::nan("");
            } else {
              j->res.primal = C.primal;
              j->res.dual = C.dual;
              j->res.rel_gap = C.rel_gap;
            }
            j->done_iters = j->res.iterations;
            retired.push_back(j);
            if (j->req.max_iter == 0) {
              e = hipMemsetAsync(j->req.chi, 0,
                                 (size_t)j->req.nx * j->req.ny * j->req.nz * (c->precision == PD_FP64 ? 8 : 4),
                                 c->stream);
              need_sync = true;
            } else if (!j->chi_stored) {   // stopped by a check before its last iteration
              e = launch_store_chi(c->d_vols, j->slot, (size_t)j->L.P * j->req.nx * j->req.ny, c->precision,
                                   c->stream);
              need_sync = true;
            }
            if (e != hipSuccess) break;
          } else {
            j->done_iters += j->run_iters;
          }
        }
        if (e == hipSuccess && need_sync) e = hipStreamSynchronize(c->stream);
      }
    }
    lk.lock();
    if (!hip_ok(c, e)) continue;
    for (auto& j : retired) {
      const Ctl& C = c->h_ctl[j->slot];
      finish_job(c, *j, C.status == 2 ? PD_ERR_STEP : C.status ? PD_ERR_NONFINITE : PD_OK);
      unreserve(c, *j);
      c->active.erase(std::find(c->active.begin(), c->active.end(), j));
    }
    if (!retired.empty()) c->cv_done.notify_all();
  }
}

// The checks pd_tune_set applies to one choice.
pd_status tune_choice_check(const pd_ctx* c, int nx, int ny, int variant, int rows, int cols, int plan_x,
                            int plan_y) {
  if (!axis_ok(nx) || !axis_ok(ny)) return PD_ERR_SIZE;
  if (variant >= 0 && !(nx == ny && variant < resident_variant_count(nx))) return PD_ERR_ARG;
  if (rows > 0 && !rows_valid(rows, nx, ny, c->precision)) return PD_ERR_ARG;
  if (cols > 0 && !cols_valid(cols, nx, ny, c->precision)) return PD_ERR_ARG;
  // alternative plans exist for FP32 direct lengths only
  const int px_max = (c->precision == PD_FP32 && !axis_blue(nx)) ? plan_count(nx) : 1;
  const int py_max = (c->precision == PD_FP32 && !axis_blue(ny)) ? plan_count(ny) : 1;
  if (plan_x >= px_max || plan_y >= py_max) return PD_ERR_ARG;
  return PD_OK;
}

// Autotuner choices on disk: one "nx ny variant rows cols" line per shape.
// Reading skips lines that do not parse or that pd_tune_set would reject;
// writing goes through a temporary file renamed over the old one, so a
// reader never sees half a file.  Caller holds c->mu (save) or is pd_create.
void load_tune_cache(pd_ctx* c) {
  FILE* f = c->tune_cache.empty() ? nullptr : std::fopen(c->tune_cache.c_str(), "r");
  if (!f) return;
  char line[256];
  while (std::fgets(line, sizeof line, f)) {
    int nx, ny, v, r, cl, px = 0, py = 0;
    const int got = std::sscanf(line, "%d %d %d %d %d %d %d", &nx, &ny, &v, &r, &cl, &px, &py);
    if (got != 5 && got != 7) continue;   // five fields: a file written before pass plans were tuned
    if (tune_choice_check(c, nx, ny, v, r, cl, px < 0 ? 0 : px, py < 0 ? 0 : py) != PD_OK) continue;
    pd_ctx::Tuned tn;
    tn.res_variant = v >= 0 ? v : 0;
    tn.rows = r > 0 ? r : 0;
    tn.cols = cl > 0 ? cl : 0;
    tn.plan_x = px > 0 ? px : 0;
    tn.plan_y = py > 0 ? py : 0;
    c->tuned[{nx, ny}] = tn;
  }
  std::fclose(f);
}

void save_tune_cache(const pd_ctx* c) {
  if (c->tune_cache.empty()) return;
  const std::string tmp = c->tune_cache + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "w");
  if (!f) return;
  bool ok = true;
  for (auto& kv : c->tuned) {
    const int nx = kv.first.first, ny = kv.first.second;
    // as pd_tune_get reports it: no resident variant for other shapes
    const int v = (nx == ny && resident_variant_count(nx) > 0) ? kv.second.res_variant : -1;
    ok &= std::fprintf(f, "%d %d %d %d %d %d %d\n", nx, ny, v, kv.second.rows, kv.second.cols, kv.second.plan_x,
                       kv.second.plan_y) > 0;
  }
  ok &= std::fclose(f) == 0;
  if (ok) std::rename(tmp.c_str(), c->tune_cache.c_str());
  else std::remove(tmp.c_str());
}

// The forward operator out = A in (pd_apply_kernel).  Only the exchange
// buffer is used: every state pointer of the descriptor aliases it.  With
// `noalloc` the buffer and the kernel tables live in the library's static
// scratch (pd_scratch.hip) instead of the arena, the tables are uploaded on
// every call (another context may have used the scratch since), and the
// per-device scratch lock serialises such calls across contexts.
pd_status apply_kernel(pd_ctx* c, const pd_request* r, bool noalloc) {
  if (!c || !r) return PD_ERR_ARG;
  CallGuard guard(c);
  if (!guard.ok) return PD_ERR_CANCELLED;
  if (!axis_ok(r->nx) || !axis_ok(r->ny) || r->nz < 1) return PD_ERR_SIZE;
  pd_status ks = kernel_args(r);
  if (ks != PD_OK) return ks;
  if (!r->delta || !r->chi || r->delta == r->chi) return PD_ERR_ARG;

  Job j;
  j.req = *r;
  j.req.gap_tol = 0.0;
  j.req.model = PD_MODEL_L1;         // the operator alone: no model state
  j.L = layout_of(j.req, c->precision);
  j.L.off_chi = j.L.off_yhat = j.L.off_dhat = j.L.off_ex = j.L.off_ex2 = 0;
  j.L.off_prow = j.L.off_pcol = 0;
  j.L.total = j.L.field;
  j.key = key_of(j.req);
  j.slot = c->nslots;                // the reserved descriptor slot
  bool fresh = false;
  std::unique_lock<std::mutex> scratch_lk;
  char* sbase = nullptr;             // noalloc: the field, after the tables
  if (noalloc) {
    const size_t tb = align_up(table_bytes(r->nx, r->ny, nz3_of(*r), c->precision));
    if (!c->scratch) return PD_ERR_HIP;
    if (tb + j.L.field > (size_t)PD_STATIC_SCRATCH_BYTES) return PD_ERR_SCRATCH;
    {
      std::lock_guard<std::mutex> lk(c->mu);
      if (c->poisoned != PD_OK) return c->poisoned;
    }
    scratch_lk = std::unique_lock<std::mutex>(static_scratch_lock(c->device));
    table_ptrs(j.tab, (char*)c->scratch, j.key, c->precision);
    sbase = (char*)c->scratch + tb;
    fresh = true;
  } else {
    std::lock_guard<std::mutex> lk(c->mu);
    if (c->poisoned != PD_OK) return c->poisoned;
    size_t off;
    if (!arena_alloc(c, j.L.total, &off)) return PD_ERR_BUDGET;
    Table* t = acquire_table(c, j.key, &fresh);
    if (!t) {
      c->arena.release(off, j.L.total);
      return PD_ERR_BUDGET;
    }
    if (fresh) t->uploaded = true;   // uploaded below, before any use
    j.tab = *t;
    j.off = off;
  }
  hipError_t e = hipSuccess;
  {
    std::lock_guard<std::mutex> ex(c->exec_mu);
    (void)hipSetDevice(c->device);
    if (fresh)
      e = c->precision == PD_FP64 ? upload_table<double>(c, j.key, j.tab) : upload_table<float>(c, j.key, j.tab);
    Vol& V = c->h_vols[j.slot];
    fill_vol(c, j, V);
    if (sbase) {
      V.chi = V.yhat = V.dhat = V.ex = V.ex2 = sbase;
      V.part_row = V.part_col = (double*)sbase;
    }
    Range* hr = c->h_ranges + (c->range_cap - 1);
    *hr = Range{j.slot, 0, 0, 0};
    const Range* dr = c->d_ranges + (c->range_cap - 1);
    if (e == hipSuccess)
      e = hipMemcpyAsync(c->d_vols + j.slot, &V, sizeof(Vol), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync((void*)dr, hr, sizeof(Range), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess && j.L.unpacked) {
      Vol& Z = c->h_vols[c->zoff + j.slot];
      fill_zvol(j, V, Z);
      e = hipMemcpyAsync(c->d_vols + c->zoff + j.slot, &Z, sizeof(Vol), hipMemcpyHostToDevice, c->stream);
    }
    const int P = j.L.P;
    if (e == hipSuccess)
      e = launch_row(axis_phys(r->nx), ROW_FWD_PLANAR, j.L.rows, P * j.L.row_groups, j.L.row_groups, c->d_vols, dr,
                     1, c->d_ctl, 0, c->precision, j.L.ext_row, c->stream);
    if (j.L.unpacked) {   // 3-D kernel: F_y, then (F_z, D, F_z^-1) on the z view, then F_y^-1
      if (e == hipSuccess)
        e = launch_col(axis_phys(r->ny), COL_FWD, j.L.cols, P * j.L.col_groups, j.L.col_groups, c->d_vols, dr, 1,
                       c->d_ctl, -1, c->precision, j.L.ext_col, c->stream);
      if (e == hipSuccess)
        e = launch_col(axis_phys(r->nz), COL_APPLY, j.L.zcols, j.L.zgroups, j.L.zgroups, c->d_vols + c->zoff, dr, 1,
                       c->d_ctl, 0, c->precision, j.L.ext_z, c->stream);
      if (e == hipSuccess)
        e = launch_col(axis_phys(r->ny), COL_INV, j.L.cols, P * j.L.col_groups, j.L.col_groups, c->d_vols, dr, 1,
                       c->d_ctl, -1, c->precision, j.L.ext_col, c->stream);
    } else if (e == hipSuccess) {
      e = launch_col(axis_phys(r->ny), COL_APPLY, j.L.cols, P * j.L.col_groups, j.L.col_groups, c->d_vols, dr, 1,
                     c->d_ctl, 0, c->precision, j.L.ext_col, c->stream);
    }
    if (e == hipSuccess)
      e = launch_row(axis_phys(r->nx), ROW_INV_PLANAR, j.L.rows, P * j.L.row_groups, j.L.row_groups, c->d_vols, dr,
                     1, c->d_ctl, 0, c->precision, j.L.ext_row, c->stream);
    hipError_t e2 = hipStreamSynchronize(c->stream);
    if (e == hipSuccess) e = e2;
  }
  std::lock_guard<std::mutex> lk(c->mu);
  if (!noalloc) {
    c->arena.release(j.off, j.L.total);
    release_table(c, j.key);
  }
  if (e != hipSuccess) {
    c->poisoned = PD_ERR_HIP;
    return PD_ERR_HIP;
  }
  return PD_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char* pd_status_string(pd_status s) {
  switch (s) {
    case PD_OK: return "ok";
    case PD_PENDING: return "pending";
    case PD_ERR_ARG: return "invalid argument";
    case PD_ERR_SIZE: return "unsupported size";
    case PD_ERR_STEP: return "step sizes violate tau*sigma*max|D|^2 < 1 or theta outside [0,1]";
    case PD_ERR_BUDGET: return "request larger than the arena";
    case PD_ERR_NONFINITE: return "non-finite duality gap";
    case PD_ERR_HIP: return "HIP runtime error";
    case PD_ERR_CANCELLED: return "cancelled";
    case PD_ERR_TICKET: return "unknown ticket";
    case PD_ERR_NODEVICE: return "no usable GPU";
    case PD_ERR_SCRATCH: return "request larger than the static scratch (PD_STATIC_SCRATCH_BYTES)";
    default: return "unknown status";
  }
}

double pd_now(void) { return now_s(); }

pd_status pd_validate(const pd_request* r, int precision, size_t* state_bytes) {
  pd_status s = validate(r, precision, nullptr, false);
  if (s != PD_OK) return s;
  if (state_bytes) *state_bytes = layout_of(*r, precision).total + table_bytes(r->nx, r->ny, nz3_of(*r), precision);
  return PD_OK;
}

pd_status pd_kernel_norm(const pd_request* r, double* norm) {
  if (!r || !norm) return PD_ERR_ARG;
  if (!axis_ok(r->nx) || !axis_ok(r->ny)) return PD_ERR_SIZE;
  pd_status ks = kernel_args(r);
  if (ks != PD_OK) return ks;
  double L = 0.0;
  if (r->kernel == PD_KERNEL_DIPOLE_3D) {
    dipole_grid3(r->nx, r->ny, r->nz, r->b0, r->voxel, r->voxel_z,
                 [&](size_t, double d) { L = std::max(L, std::fabs(d)); });
  } else {
    std::vector<double> D;
    dipole_grid(r->nx, r->ny, r->b0, r->voxel, r->kernel, D);
    L = grid_norm(D);
  }
  *norm = L;
  return PD_OK;
}

pd_status pd_create(const pd_config* cfg, pd_ctx** out) {
  if (!cfg || !out) return PD_ERR_ARG;
  *out = nullptr;
  if (cfg->precision != PD_FP32 && cfg->precision != PD_FP64) return PD_ERR_ARG;
  if (!cfg->arena || cfg->arena_bytes == 0 || ((uintptr_t)cfg->arena & (kAlign - 1)) != 0) return PD_ERR_ARG;
  if (cfg->max_slots < 0 || cfg->step_iters < 0 || cfg->step_iters > kMaxStep) return PD_ERR_ARG;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return PD_ERR_NODEVICE;
  if (cfg->device < 0 || cfg->device >= ndev) return PD_ERR_ARG;
  if (hipSetDevice(cfg->device) != hipSuccess) return PD_ERR_HIP;
  void* scratch = nullptr;   // looked up once per device, with the device current
  if (static_scratch(cfg->device, &scratch) != hipSuccess) return PD_ERR_HIP;

  std::unique_ptr<pd_ctx> c(new pd_ctx());
  c->scratch = scratch;
  c->multi_cap = multi_max_groups_per_xcd();
  c->cfg = *cfg;
  c->device = cfg->device;
  c->precision = cfg->precision;
  c->nslots = cfg->max_slots > 0 ? cfg->max_slots : kDefaultSlots;
  c->time_kernels = (cfg->flags & PD_FLAG_TIME_KERNELS) != 0;
  if (cfg->flags & PD_FLAG_TEST_BARRIER_GIVEUP) c->spin_limit = 0;
  if (cfg->tune_cache) c->tune_cache = cfg->tune_cache;
  else if (const char* env = std::getenv("PD_TUNE_CACHE")) c->tune_cache = env;
  c->cfg.tune_cache = nullptr;   // the caller's string is not kept
  load_tune_cache(c.get());
  c->arena.init((char*)cfg->arena, cfg->arena_bytes);

  c->range_cap = 4 * (size_t)c->nslots + 4096;
  c->zoff = c->nslots + 1;
  c->off_slots = align_up(sizeof(Vol) * 2 * (c->nslots + 1));
  c->off_ranges = c->off_slots + align_up(sizeof(int) * c->nslots);
  c->off_abort = align_up(sizeof(Ctl) * (c->nslots + 1));
  const size_t step_block = c->off_ranges + sizeof(Range) * c->range_cap;
  c->ctl_bytes = align_up(step_block) + align_up(c->off_abort + sizeof(int)) + align_up(counter_bytes(kMaxTeamSlots));
  if (!c->arena.alloc(c->ctl_bytes, &c->ctl_off)) return PD_ERR_BUDGET;
  char* p = c->arena.ptr(c->ctl_off);
  c->d_vols = (Vol*)p;
  c->d_slots = (int*)(p + c->off_slots);
  c->d_ranges = (Range*)(p + c->off_ranges);
  p += align_up(step_block);
  c->d_ctl = (Ctl*)p;
  c->d_abort = (int*)(p + c->off_abort);
  p += align_up(c->off_abort + sizeof(int));
  c->d_counters = (unsigned*)p;

  if (cfg->stream) {
    c->stream = (hipStream_t)cfg->stream;
  } else {
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) return PD_ERR_HIP;
    c->own_stream = true;
  }
  bool ok = hipHostMalloc((void**)&c->h_vols, sizeof(Vol) * 2 * (c->nslots + 1), hipHostMallocDefault) ==
                hipSuccess &&
            hipHostMalloc((void**)&c->h_ctl, c->off_abort + sizeof(int), hipHostMallocDefault) == hipSuccess &&
            hipHostMalloc((void**)&c->h_ranges, sizeof(Range) * c->range_cap, hipHostMallocDefault) == hipSuccess;
  for (int s = 0; ok && s < kRunAhead; ++s)
    ok = hipHostMalloc((void**)&c->h_stage[s], step_block, hipHostMallocDefault) == hipSuccess;
  if (ok) {
    c->h_abort = (int*)((char*)c->h_ctl + c->off_abort);
    *c->h_abort = 0;
    std::memset(c->h_vols, 0, sizeof(Vol) * 2 * (c->nslots + 1));
    std::memset(c->h_ctl, 0, sizeof(Ctl) * (c->nslots + 1));
    for (int s = 0; s < kRunAhead; ++s) std::memset(c->h_stage[s], 0, step_block);
    for (int s = c->nslots - 1; s >= 0; --s) c->free_slots.push_back(s);
    // all descriptors start idle (iters = 0)
    ok = hipMemcpyAsync(c->d_vols, c->h_vols, sizeof(Vol) * 2 * (c->nslots + 1), hipMemcpyHostToDevice,
                        c->stream) == hipSuccess &&
         launch_zero(c->d_ctl, align_up(c->off_abort + sizeof(int)), c->stream) == hipSuccess &&
         hipStreamSynchronize(c->stream) == hipSuccess;
  }
  if (!ok) {
    free_host(c.get());
    if (c->own_stream) (void)hipStreamDestroy(c->stream);
    return PD_ERR_HIP;
  }
  pd_ctx* raw = c.release();
  raw->worker = std::thread(worker_main, raw);
  *out = raw;
  return PD_OK;
}

pd_status pd_solve_batch(pd_ctx* c, const pd_request* r, int n, uint64_t* tickets) {
  if (!c || (n > 0 && (!r || !tickets)) || n < 0) return PD_ERR_ARG;
  CallGuard guard(c);
  if (!guard.ok) return PD_ERR_CANCELLED;
  std::vector<std::shared_ptr<Job>> js;
  size_t avail = c->arena.size() - align_up(c->ctl_bytes);
  for (int i = 0; i < n; ++i) {
    double knorm = 0.0;
    pd_status s = validate(&r[i], c->precision, &knorm);
    if (s != PD_OK) return s;
    auto j = std::make_shared<Job>();
    j->knorm = knorm;
    j->req = r[i];
    j->L = layout_of(r[i], c->precision);
    j->key = key_of(r[i]);
    // the request and its table must fit in an otherwise empty arena
    size_t need = j->L.total + table_bytes(r[i].nx, r[i].ny, nz3_of(r[i]), c->precision);
    if (need > avail) return PD_ERR_BUDGET;
    js.push_back(j);
  }
  std::lock_guard<std::mutex> lk(c->mu);
  if (c->poisoned != PD_OK) return c->poisoned;
  double t = now_s();
  for (int i = 0; i < n; ++i) {
    js[i]->ticket = c->next_ticket++;
    js[i]->t_submit = t;
    tickets[i] = js[i]->ticket;
    c->jobs[js[i]->ticket] = js[i];
    c->queue.push_back(js[i]);
    c->n_queued.fetch_add(1, std::memory_order_release);
  }
  c->cv_work.notify_all();
  return PD_OK;
}

pd_status pd_poll(pd_ctx* c, uint64_t ticket, pd_result* out, int timeout_ms) {
  if (!c) return PD_ERR_ARG;
  CallGuard guard(c);   // outlives the lock below: released after it
  if (!guard.ok) return PD_ERR_CANCELLED;
  std::unique_lock<std::mutex> lk(c->mu);
  auto it = c->jobs.find(ticket);
  if (it == c->jobs.end()) return PD_ERR_TICKET;
  std::shared_ptr<Job> j = it->second;
  // pd_destroy wakes every waiter: the ticket ends cancelled
  auto done = [&] { return j->finished || c->stopping; };
  if (timeout_ms < 0)
    c->cv_done.wait(lk, done);
  else if (timeout_ms > 0)
    c->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), done);
  if (!j->finished) return c->stopping ? PD_ERR_CANCELLED : PD_PENDING;
  if (out) *out = j->res;
  c->jobs.erase(ticket);
  return j->res.status;
}

pd_status pd_destroy(pd_ctx* c) {
  if (!c) return PD_OK;
  {
    std::lock_guard<std::mutex> lk(c->mu);
    c->stopping = true;
    c->cv_work.notify_all();
    c->cv_done.notify_all();   // pd_poll waiters return PD_ERR_CANCELLED
  }
  if (c->worker.joinable()) c->worker.join();
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  {
    std::lock_guard<std::mutex> lk(c->mu);
    for (auto& j : c->queue) finish_job(c, *j, PD_ERR_CANCELLED);
    for (auto& j : c->active) finish_job(c, *j, PD_ERR_CANCELLED);
    c->cv_done.notify_all();
  }
  {
    // calls already inside the context (a waiting pd_poll, a pd_tune) leave
    // before anything they touch is freed
    std::unique_lock<std::mutex> lk(c->mu);
    c->cv_idle.wait(lk, [&] { return c->calls == 0; });
  }
  for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
  for (auto& g : c->graphs)
    if (g.second.exec) (void)hipGraphExecDestroy(g.second.exec);
  free_host(c);
  if (c->own_stream) (void)hipStreamDestroy(c->stream);
  delete c;
  return PD_OK;
}

pd_status pd_apply_kernel(pd_ctx* c, const pd_request* r) { return apply_kernel(c, r, false); }

pd_status pd_apply_kernel_noalloc(pd_ctx* c, const pd_request* r) { return apply_kernel(c, r, true); }

pd_status pd_kernel_time(pd_ctx* c, int kind, int64_t* launches, double* total_ms, double* point_iters) {
  if (!c || kind < 0 || kind >= pd_ctx::kKinds) return PD_ERR_ARG;
  CallGuard guard(c);
  if (!guard.ok) return PD_ERR_CANCELLED;
  std::lock_guard<std::mutex> lk(c->tmu);
  if (launches) *launches = c->t_launches[kind];
  if (total_ms) *total_ms = c->t_ms[kind];
  if (point_iters) *point_iters = c->t_points[kind];
  return PD_OK;
}

pd_status pd_kernel_time_reset(pd_ctx* c) {
  if (!c) return PD_ERR_ARG;
  CallGuard guard(c);
  if (!guard.ok) return PD_ERR_CANCELLED;
  std::lock_guard<std::mutex> lk(c->tmu);
  for (int k = 0; k < pd_ctx::kKinds; ++k) {
    c->t_launches[k] = 0;
    c->t_ms[k] = 0.0;
    c->t_points[k] = 0.0;
  }
  return PD_OK;
}

pd_status pd_tune(pd_ctx* c, int nx, int ny, int nz, int iters, pd_tune_entry* entries, int max_entries,
                  int* n_entries) {
  if (!c || iters < 1 || nz < 1 || max_entries < 0) return PD_ERR_ARG;
  CallGuard guard(c);
  if (!guard.ok) return PD_ERR_CANCELLED;
  if (!axis_ok(nx) || !axis_ok(ny)) return PD_ERR_SIZE;
  if (n_entries) *n_entries = 0;
  pd_request r{};
  r.nx = nx;
  r.ny = ny;
  r.nz = nz;
  r.b0[1] = 1.0;
  r.voxel[0] = r.voxel[1] = 1.0;
  r.kernel = PD_KERNEL_DIPOLE;
  r.lambda = 1e-3;
  r.tau = r.sigma = 1.4;
  r.theta = 1.0;
  r.max_iter = iters;
  Job j;
  j.req = r;
  j.L = layout_of(r, c->precision);
  j.key = key_of(r);
  bool fresh = false;
  {
    std::lock_guard<std::mutex> lk(c->mu);
    if (c->poisoned != PD_OK) return c->poisoned;
    size_t off;
    if (!arena_alloc(c, j.L.total, &off)) return PD_ERR_BUDGET;
    Table* t = acquire_table(c, j.key, &fresh);
    if (!t) {
      c->arena.release(off, j.L.total);
      return PD_ERR_BUDGET;
    }
    if (fresh) t->uploaded = true;   // uploaded below, before any use
    j.tab = *t;
    j.off = off;
    j.slot = c->nslots;              // the reserved descriptor slot
  }
  std::vector<pd_tune_entry> all;
  hipError_t e = hipSuccess;
  {
    std::lock_guard<std::mutex> ex(c->exec_mu);
    (void)hipSetDevice(c->device);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if ((e = hipEventCreate(&e0)) == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess && fresh)
      e = c->precision == PD_FP64 ? upload_table<double>(c, j.key, j.tab) : upload_table<float>(c, j.key, j.tab);
    // zero state and F delta: every value stays zero, so each configuration
    // runs the same data-independent arithmetic
    if (e == hipSuccess) e = launch_zero(c->arena.ptr(j.off), j.L.total, c->stream);
    if (e == hipSuccess) e = launch_zero(c->d_ctl + j.slot, sizeof(Ctl), c->stream);
    Range* hr = c->h_ranges + (c->range_cap - 1);
    *hr = Range{j.slot, 0, 0, 0};
    const Range* dr = c->d_ranges + (c->range_cap - 1);
    if (e == hipSuccess) e = hipMemcpyAsync((void*)dr, hr, sizeof(Range), hipMemcpyHostToDevice, c->stream);
    Vol& V = c->h_vols[j.slot];
    auto upload_vol = [&](int rg, int cg) -> hipError_t {
      fill_vol(c, j, V);
      V.iters = iters;
      V.done_base = 0;
      V.final_it = -1;
      V.check_last = 0;
      V.row_groups = rg;
      V.col_groups = cg;
      hipError_t r2 = hipMemcpyAsync(c->d_vols + j.slot, &V, sizeof(Vol), hipMemcpyHostToDevice, c->stream);
      if (r2 == hipSuccess) r2 = hipStreamSynchronize(c->stream);   // V is reused by the next candidate
      return r2;
    };
    auto time_it = [&](auto&& launch, double* best) -> hipError_t {
      *best = 1e300;
      for (int rep = 0; rep < 4; ++rep) {
        hipError_t r2 = hipEventRecord(e0, c->stream);
        if (r2 == hipSuccess) r2 = launch();
        if (r2 == hipSuccess) r2 = hipEventRecord(e1, c->stream);
        if (r2 == hipSuccess) r2 = hipEventSynchronize(e1);
        if (r2 != hipSuccess) return r2;
        float ms = 0.f;
        if ((r2 = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) return r2;
        if (rep > 0) *best = std::min(*best, (double)ms);   // first run warms up
      }
      return hipSuccess;
    };
    const int P = j.L.P;
    // resident variants
    if (e == hipSuccess && c->precision == PD_FP32 && nx == ny) {
      for (int v = 0; e == hipSuccess && v < resident_variant_count(nx); ++v) {
        const ResidentVariant* rv = resident_variant(nx, v);
        int maxt = std::min(rv->max_teams(), kMaxTeamSlots);
        if (maxt <= 0) continue;
        int nteams = std::min(P, maxt);
        if ((e = upload_vol(rv->team(), rv->team())) != hipSuccess) break;
        double best = 0;
        e = time_it([&] {
          const size_t slots_ = (size_t)((nteams + kXcds - 1) / kXcds) * kXcds;
          hipError_t r2 = launch_zero(c->d_counters, align_up(counter_bytes(slots_)),
                                      c->stream);
          if (r2 != hipSuccess) return r2;
          return rv->launch(nteams, c->d_vols, dr, 1, c->d_ctl, c->d_counters, c->d_abort,
                            (c->cfg.flags & PD_FLAG_FENCED_EXCHANGE) ? 1 : 0, c->spin_limit, c->stream);
        }, &best);
        if (e == hipSuccess) e = hipMemcpy(c->h_abort, c->d_abort, sizeof(int), hipMemcpyDeviceToHost);
        if (e == hipSuccess && *c->h_abort) {
          // a team barrier gave up: this variant is not a candidate (the
          // context stays usable)
          *c->h_abort = 0;
          e = launch_zero(c->d_abort, sizeof(int), c->stream);
          if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
          continue;
        }
        // time per iteration of all P pairs (nteams pairs per launch)
        pd_tune_entry t{nx, ny, nz, iters, 0, v, rv->team(), rv->threads(), 0, 0, rv->plan(),
                        best * (double)P / nteams};
        all.push_back(t);
      }
    }
    // two-launch path: the column kernel per tile width and pass plan of the
    // column (ny) transforms, the row kernel per tile height and pass plan of
    // the row (nx) transforms, each timed alone (the two choices are
    // independent; an iteration runs one of each)
    const int rg0 = ceil_div(ny, rows_per_wg(nx, ny, c->precision));
    const int cg0 = ceil_div(nx, cols_per_wg(nx, ny, c->precision));
    const int wide = col_group_wide(ny);
    for (int cols : {8, 16, wide > 16 ? wide : 0}) {
      if (e != hipSuccess) break;
      if (!cols_valid(cols, nx, ny, c->precision)) continue;
      const int cg = ceil_div(nx, cols);
      const int ec = axis_ext(ny, nx, cols);
      const int nplans = (c->precision == PD_FP32 && ec == 0) ? plan_count(ny) : 1;
      for (int plan = 0; plan < nplans && e == hipSuccess; ++plan) {
        if ((e = upload_vol(rg0, cg)) != hipSuccess) break;
        double best = 0;
        e = time_it([&] {
          hipError_t r2 = hipSuccess;
          for (int it = 0; it < iters && r2 == hipSuccess; ++it)
            r2 = launch_col_p(axis_phys(ny), COL_ITER, cols, P * cg, cg, c->d_vols, dr, 1, c->d_ctl, it, c->precision,
                              ec, plan, c->stream);
          return r2;
        }, &best);
        pd_tune_entry t{nx, ny, nz, iters, 1, -1, 0, 0, 0, cols, plan, best};
        all.push_back(t);
      }
    }
    for (int rows : {8, row_group_big(nx)}) {
      if (e != hipSuccess) break;
      if (!rows_valid(rows, nx, ny, c->precision)) continue;
      bool dup = false;
      for (auto& t : all) dup |= t.path == 2 && t.rows == rows;
      if (dup) continue;
      const int rg = ceil_div(ny, rows);
      const int er = axis_ext(nx, ny, rows);
      const int nplans = (c->precision == PD_FP32 && er == 0) ? plan_count(nx) : 1;
      for (int plan = 0; plan < nplans && e == hipSuccess; ++plan) {
        if ((e = upload_vol(rg, cg0)) != hipSuccess) break;
        double best = 0;
        e = time_it([&] {
          hipError_t r2 = hipSuccess;
          for (int it = 0; it < iters && r2 == hipSuccess; ++it)
            r2 = launch_row_p(axis_phys(nx), ROW_ITER, rows, P * rg, rg, c->d_vols, dr, 1, c->d_ctl, it,
                              c->precision, er, plan, c->stream);
          return r2;
        }, &best);
        pd_tune_entry t{nx, ny, nz, iters, 2, -1, 0, 0, rows, 0, plan, best};
        all.push_back(t);
      }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    hipError_t e2 = hipStreamSynchronize(c->stream);
    if (e == hipSuccess) e = e2;
  }
  std::lock_guard<std::mutex> lk(c->mu);
  c->arena.release(j.off, j.L.total);
  release_table(c, j.key);
  if (e != hipSuccess) {
    c->poisoned = PD_ERR_HIP;
    return PD_ERR_HIP;
  }
  pd_ctx::Tuned tn = c->tuned.count({nx, ny}) ? c->tuned[{nx, ny}] : pd_ctx::Tuned{};
  double best_res = 1e300, best_col = 1e300, best_row = 1e300;
  for (auto& t : all) {
    if (t.path == 0 && t.ms < best_res) {
      best_res = t.ms;
      tn.res_variant = t.variant;
    }
    if (t.path == 1 && t.ms < best_col) {
      best_col = t.ms;
      tn.cols = t.cols;
      tn.plan_y = t.plan;
    }
    if (t.path == 2 && t.ms < best_row) {
      best_row = t.ms;
      tn.rows = t.rows;
      tn.plan_x = t.plan;
    }
  }
  c->tuned[{nx, ny}] = tn;
  save_tune_cache(c);
  int n = 0;
  for (auto& t : all) {
    if (entries && n < max_entries) entries[n] = t;
    ++n;
  }
  if (n_entries) *n_entries = std::min(n, max_entries);
  return PD_OK;
}

pd_status pd_tune_set(pd_ctx* c, int nx, int ny, int variant, int rows, int cols, int plan_x, int plan_y) {
  if (!c) return PD_ERR_ARG;
  CallGuard guard(c);
  if (!guard.ok) return PD_ERR_CANCELLED;
  pd_status st = tune_choice_check(c, nx, ny, variant, rows, cols, plan_x < 0 ? 0 : plan_x, plan_y < 0 ? 0 : plan_y);
  if (st != PD_OK) return st;
  std::lock_guard<std::mutex> ex(c->exec_mu);   // between scheduling steps
  std::lock_guard<std::mutex> lk(c->mu);
  if (variant >= 0) c->no_resident.erase({nx, ny});   // an explicit resident choice re-enables it
  pd_ctx::Tuned tn;
  tn.res_variant = variant >= 0 ? variant : 0;
  tn.rows = rows > 0 ? rows : 0;
  tn.cols = cols > 0 ? cols : 0;
  tn.plan_x = plan_x > 0 ? plan_x : 0;
  tn.plan_y = plan_y > 0 ? plan_y : 0;
  c->tuned[{nx, ny}] = tn;
  save_tune_cache(c);
  return PD_OK;
}

pd_status pd_tune_get(pd_ctx* c, int nx, int ny, int* variant, int* rows, int* cols, int* plan_x, int* plan_y) {
  if (!c) return PD_ERR_ARG;
  CallGuard guard(c);
  if (!guard.ok) return PD_ERR_CANCELLED;
  std::lock_guard<std::mutex> lk(c->mu);
  pd_ctx::Tuned tn = c->tuned.count({nx, ny}) ? c->tuned[{nx, ny}] : pd_ctx::Tuned{};
  if (variant) *variant = (nx == ny && resident_variant_count(nx) > 0) ? tn.res_variant : -1;
  if (rows) *rows = tn.rows > 0 ? tn.rows : rows_per_wg(nx, ny, c->precision);
  if (cols) *cols = tn.cols > 0 ? tn.cols : cols_per_wg(nx, ny, c->precision);
  if (plan_x) *plan_x = tn.plan_x;
  if (plan_y) *plan_y = tn.plan_y;
  return PD_OK;
}

pd_status pd_graph_stats(pd_ctx* c, int64_t* captures, int64_t* replays) {
  if (!c) return PD_ERR_ARG;
  CallGuard guard(c);
  if (!guard.ok) return PD_ERR_CANCELLED;
  std::lock_guard<std::mutex> ex(c->exec_mu);
  if (captures) *captures = c->graph_captures;
  if (replays) *replays = c->graph_replays;
  return PD_OK;
}

pd_status pd_recovery_stats(pd_ctx* c, int64_t* aborted_rounds, int64_t* restarted_requests) {
  if (!c) return PD_ERR_ARG;
  CallGuard guard(c);
  if (!guard.ok) return PD_ERR_CANCELLED;
  std::lock_guard<std::mutex> ex(c->exec_mu);
  if (aborted_rounds) *aborted_rounds = c->aborted_rounds;
  if (restarted_requests) *restarted_requests = c->restarted_requests;
  return PD_OK;
}

pd_status pd_arena_usage(pd_ctx* c, size_t* used, int* resident, int* queued) {
  if (!c) return PD_ERR_ARG;
  CallGuard guard(c);
  if (!guard.ok) return PD_ERR_CANCELLED;
  std::lock_guard<std::mutex> lk(c->mu);
  if (used) *used = c->arena.used();
  if (resident) *resident = (int)c->active.size();
  if (queued) *queued = (int)c->queue.size();
  return PD_OK;
}

}  // extern "C"
