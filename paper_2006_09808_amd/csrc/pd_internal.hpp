// pd_internal.hpp - structures shared by the host scheduler and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

namespace pdk {

// One resident request (a volume of nz slices), as the kernels see it.
// Slices 2p and 2p+1 of the volume share one complex field ("pair" p):
// slice 2p is the real part, slice 2p+1 the imaginary part.  D is real and
// even, so A acts on the two parts independently.  All state buffers are
// [P][ny][nx] complex, x fastest.
struct Vol {
  void* chi;          // chi_n, pair-interleaved
  void* yhat;         // dual variable, kept in the frequency domain
  void* dhat;         // F(delta), computed once at admission
  void* ex;           // exchange buffer between the column and row kernels
  void* ex2;          // row transform of chi on check iterations (may alias ex)
  const void* dtab;   // D[ky][kx], real, shared by volumes of one kernel shape
  const void* twx;    // exp(-2 pi i m / nx), m < nx
  const void* twy;    // exp(-2 pi i m / ny), m < ny
  double* part_row;   // per row-kernel workgroup: sum|chi|, max|A y|
  double* part_col;   // per check-kernel workgroup: sum|D F chi - F delta|^2,
                      //   sum |yhat|^2, Re sum yhat conj(dhat)
  const void* user_in;   // planar [nz][ny][nx] input (field map / operator input)
  void* user_out;        // planar [nz][ny][nx] output
  // weighted TV model (Eq. (1)); unused by the L1 model.  All image-domain,
  // pair-interleaved [P][ny][nx] complex like chi.
  void* chibar;          // over-relaxed primal
  void* pdual;           // data-term dual p
  void* qx;              // gradient dual, x component
  void* qy;              // gradient dual, y component
  void* qz;              // gradient dual, z component (model in three dimensions)
  void* wgt;             // weights W
  void* msk;             // mask M
  void* dpk;             // field map delta
  const void* user_w;    // caller's planar [nz][ny][nx] W and M
  const void* user_m;
  double tau, sigma, lam, theta;
  double gap_tol;
  double inv_dx, inv_dy; // 1 / voxel size (TV model's gradient)
  double inv_dz;         // 1 / slice thickness (TV model in three dimensions), else 0
  double knorm;          // max |D| (TV model's step check)
  double gap_norm;       // 1 / (points of one transform): 1/(nx ny), or 1/(nx ny nz) for the 3-D kernel
  int nx, ny, nz, P;
  int half_last;      // nz odd: the last pair's imaginary part is padding
  int iters;          // iterations to run in this step (0: idle)
  int done_base;      // iterations completed before this step
  int max_iter;
  int final_it;       // step iteration of the volume's last update, or -1
  int row_groups;     // row-kernel workgroups per pair
  int col_groups;     // column-kernel workgroups per pair
  int check_only;     // max_iter == 0: only the gap of chi_0 = 0 is evaluated
  int check_last;     // gap partials after the step's last iteration
  int model;          // 0: L1 prior on chi, 1: weighted TV (Eq. (1))
  int unpacked;       // 3-D kernel: one slice per complex plane (imaginary part 0), P = nz
  int col_parts;      // column-kernel gap partial entries (P col_groups; the z view's groups in 3-D)
  int tv3;            // TV model in three dimensions: image-domain fields pair-interleaved
                      //   [P][ny][nx], the exchange buffer nz unpacked planes [nz][ny][nx]
};

// Device-side control/result block of one resident request.  16-byte
// aligned: the blocks of all slots form one array that is zero-filled per slot
// with 16-byte stores.
struct alignas(16) Ctl {
  int stop;           // set by the gap reduction; kernels skip stopped volumes
  int stop_iter;      // iterations applied when the last check ran
  int status;         // 0 ok, 1 non-finite, 2 step condition violated
  int checks;
  double primal, dual, rel_gap, max_ay;
  // TV model set-up: bit patterns of max|W| and max|M| (non-negative
  // doubles order like their bits), and a non-finite-input flag
  unsigned long long wmax_bits, mmax_bits;
  int bad_input;
  int pad;
};
static_assert(sizeof(Ctl) % 16 == 0, "Ctl entries must stay 16-byte aligned");

// One volume's share of a launch: workgroups [first, next range's first)
// belong to volume `slot`, `groups` consecutive workgroups per pair,
// starting at pair `pair0`.
struct Range {
  int slot;
  int first;
  int pair0;          // first pair of the volume covered by this range
  int pad;
};

// Pointers read from a descriptor are generic; telling the compiler they
// point to global memory lets it use global instead of flat instructions.
template <typename P>
__device__ __forceinline__ P* gmem(P* p) {
#if defined(__HIP_DEVICE_COMPILE__)
  __builtin_assume(!__builtin_amdgcn_is_shared((const void*)p));
  __builtin_assume(!__builtin_amdgcn_is_private((const void*)p));
#endif
  return p;
}

// Copy a per-length twiddle table into LDS (the butterflies gather from it).
template <typename C>
__device__ __forceinline__ void stage_twiddles(C* dst, const C* src, int n, int tid, int nt) {
  for (int i = tid; i < n; i += nt) dst[i] = src[i];
}

// Workgroup b -> (slot, pair, group) by binary search over the launch's ranges.
__device__ __forceinline__ void find_work_b(const Range* __restrict__ ranges, int nranges, int groups, int b,
                                            int& slot, int& pair, int& g) {
  int lo = 0, hi = nranges - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (ranges[mid].first <= b) lo = mid;
    else hi = mid - 1;
  }
  slot = ranges[lo].slot;
  int local = b - ranges[lo].first;
  int p = local / groups;
  g = local - p * groups;
  pair = ranges[lo].pair0 + p;
}
// The dispatcher hands workgroups to the XCDs round-robin (block b to XCD
// b mod 8), and each XCD has its own L2.  Renumbering them XCD-major gives
// each XCD one contiguous run of logical workgroups, so neighbouring column
// strips, which share the 128-byte lines of every [ny][nx] field, meet in the
// same L2 instead of fetching each line once per XCD.  A bijection on
// [0, G) for any G.
__device__ __forceinline__ int xcd_major(int b, int G) {
  const int per = G / 8, rem = G % 8;
  const int x = b % 8, i = b / 8;
  return x * per + (x < rem ? x : rem) + i;
}
__device__ __forceinline__ void find_work(const Range* __restrict__ ranges, int nranges, int groups,
                                          int& slot, int& pair, int& g) {
  find_work_b(ranges, nranges, groups, xcd_major((int)blockIdx.x, (int)gridDim.x), slot, pair, g);
}

// COL_FWD / COL_INV: the column transform alone (forward / inverse, in place
// in the exchange buffer), the in-plane half of the 3-D kernel's transforms;
// with it < 0 they run unconditionally (set-up, operator), else like
// COL_ITER.  COL_FWD_CHK: forward, in place in the check buffer, on check steps.
enum ColMode { COL_ITER = 0, COL_CHECK = 1, COL_SETUP = 2, COL_APPLY = 3, COL_TV = 4, COL_FWD = 5, COL_INV = 6,
               COL_FWD_CHK = 7 };
enum RowMode { ROW_ITER = 0, ROW_FWD_PLANAR = 1, ROW_INV_PLANAR = 2, ROW_TV_DUAL = 3, ROW_TV_PRIMAL = 4,
               ROW_TV3_DUAL = 5, ROW_TV3_PRIMAL = 6 };

constexpr int kThreads = 256;

// Launchers, one set per transform length (defined in pd_kern_<N>.hip).
// `cols` is the strip width / `rows` the rows per workgroup, `grid` the number
// of workgroups and `groups` the workgroups per pair.

bool size_supported(int n);    // transform lengths with a direct plan
// Length of the transforms that carry a Bluestein DFT of length n (the
// smallest direct length >= 2n - 1), 0 if n is out of range.
int blue_len(int n);

// `n` is the transform length (for ext == 2, the Bluestein length M), `ext`
// the kernel variant: 0 plain, 1 partial last tile, 2 Bluestein.
hipError_t launch_col(int n, int mode, int cols, int grid, int groups, const Vol* vols,
                      const Range* ranges, int nranges, Ctl* ctl, int it, int precision, int ext, hipStream_t st);
hipError_t launch_row(int n, int mode, int rows, int grid, int groups, const Vol* vols,
                      const Range* ranges, int nranges, Ctl* ctl, int it, int precision, int ext, hipStream_t st);
// The same with pass plan `plan` of length n (0 .. plan_count(n) - 1; plans
// other than 0 for FP32 whole-tile transforms only).
hipError_t launch_col_p(int n, int mode, int cols, int grid, int groups, const Vol* vols, const Range* ranges,
                        int nranges, Ctl* ctl, int it, int precision, int ext, int plan, hipStream_t st);
hipError_t launch_row_p(int n, int mode, int rows, int grid, int groups, const Vol* vols, const Range* ranges,
                        int nranges, Ctl* ctl, int it, int precision, int ext, int plan, hipStream_t st);
// Number of pass plans of a direct transform length (1 for any other n).
int plan_count(int n);
hipError_t launch_reduce(int nslots, const Vol* vols, const int* slots, Ctl* ctl, int it,
                         int precision, hipStream_t st);
hipError_t launch_store_chi(const Vol* vols, int slot, size_t npairs_pts, int precision,
                            hipStream_t st);
hipError_t launch_zero(void* p, size_t bytes, hipStream_t st);
// TV model set-up of one volume: pack W, M and delta into the pair layout,
// record max|W|, max|M| and non-finite inputs in ctl[slot], then test the
// step condition and stop the volume (status 1 or 2) if it fails.
hipError_t launch_tv_setup(const Vol* vols, Ctl* ctl, int slot, size_t npair_pts, int precision, hipStream_t st);

// Resident (multi-iteration, all workgroups co-resident) launch for square n x n slices.
// resident_team(n) is the workgroups per pair (0: no resident kernel for n);
// resident_max_teams(n) the teams that can be co-resident on the device.
// Teams are placed one XCD apart (team t on XCD t mod 8), so a launch covers
// a multiple of 8 teams; resident_max_teams is such a multiple.  Each square
// shape has one or more variants (workgroups per pair x block size);
// variant 0 is the default, an autotuner may pick another.
constexpr int kXcds = 8;
// Resident-launch synchronisation counters, one per 256-byte line so that
// teams spinning on their own barrier never share a line: team slot t at
// word t * kCounterStride, then kXcds per-XCD tickets, then the grid arrival
// counter.  kMaxTeamSlots bounds the teams of one launch.
constexpr int kCounterStride = 64;
constexpr int kMaxTeamSlots = 2048;
inline size_t counter_bytes(size_t team_slots) {
  return (team_slots + kXcds + 1) * kCounterStride * sizeof(unsigned);
}
// Polls a resident-launch barrier makes before it gives up and raises the
// launch's abort flag (each poll sleeps about 128 cycles, so the default is
// of the order of a second; a test can pass a handful to force the give-up).
constexpr unsigned kSpinLimit = 1u << 22;
typedef hipError_t (*resident_launch_fn)(int nteams, const Vol* vols, const Range* ranges, int nranges, Ctl* ctl,
                                         unsigned* counters, int* abort_flag, int fenced, unsigned spin_limit,
                                         hipStream_t st);
struct ResidentVariant {
  int n;
  resident_launch_fn launch;
  int (*max_teams)();
  int (*team)();
  int (*threads)();
  int (*plan)();      // FFT pass plan of both axes (variants of one plan give the same bits)
};
// The library's fixed device scratch (pd_scratch.hip): device address of
// `device`'s copy (the device must be current), and the lock that
// serialises its users within the process.
hipError_t static_scratch(int device, void** ptr);
std::mutex& static_scratch_lock(int device);

// The multi-shape resident launch (pd_resident_multi.hip): body index and
// team size of the square n x n shape on FFT plan `plan` in it (-1 / 0: not
// a body), the
// co-resident workgroups one XCD holds, and the launch of quota workgroups
// per XCD over the team table at `table` (kXcds + 1 XCD entries, then the
// teams; see k_resident_multi).
int multi_body(int n, int plan);
int multi_team(int n, int plan);
int multi_max_groups_per_xcd();
hipError_t launch_resident_multi(int quota, const Vol* vols, const Range* table, Ctl* ctl, unsigned* counters,
                                 int* abort_flag, int ticket_base, int fenced, unsigned spin_limit, hipStream_t st);

int resident_variant_count(int n);                      // 0: no resident kernel for n x n
const ResidentVariant* resident_variant(int n, int v);  // nullptr if out of range
// The weighted TV model's resident launch of square n x n slices (one
// variant per shape; nullptr: none for n).  Same arguments and protocol as
// the L1 model's; the volumes' descriptors carry the TV state.
const ResidentVariant* resident_tv_variant(int n);

}  // namespace pdk
