// Host-only tests of the library's scheduler (csrc/pd_host.cpp) against a
// mock executor, built with g++ and the address/undefined or thread
// sanitizer; no GPU.  The HIP runtime is the stand-in of
// tests/cpp/mockhip/hip/hip_runtime.h and the kernels are replaced by mock
// launchers that keep one counter per slice pair:
//   - an iteration launch (row kernel, resident launch) adds the iterations
//     it applies to every pair it covers, skipping stopped volumes exactly
//     as the kernels do;
//   - the gap reduction reports rel_gap = 1 / (n + 1) after n iterations and
//     stops a volume like the real reduction (final iteration, or
//     rel_gap <= gap_tol), after checking that every pair of the volume has
//     received exactly n iterations;
//   - storing chi writes each pair's counter into every voxel of its slices.
// So a finished request must report the iteration count its parameters
// imply and its output must hold that count everywhere, whatever the mix of
// requests, the admission order, the round structure or a recovery.
//
// Usage: sched_mock [test-name]; prints one line per test and "ok <n>" when
// all pass; exit status 1 on the first failure.
#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <functional>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "pd.h"
#include "pd_internal.hpp"

// ---------------------------------------------------------------------------
// mock runtime
// ---------------------------------------------------------------------------
thread_local dim3 blockIdx, threadIdx, gridDim, blockDim;

struct ihipStream_t {
  int unused = 0;
};
struct ihipEvent_t {
  double t = 0.0;
};
struct ihipGraph {
  std::vector<std::function<void()>> ops;
};
struct hipGraphExec {
  std::vector<std::function<void()>> ops;
};

namespace mock {
thread_local std::vector<std::function<void()>>* capture = nullptr;
std::atomic<int> violations{0};
std::atomic<int> step_sleep_us{0};     // each iteration launch sleeps this long (a slow GPU)
std::atomic<int> force_aborts{0};      // resident launches to fail, whatever the spin limit
std::atomic<long> resident_launches{0}, row_launches{0}, multi_launches{0};
std::atomic<int*> abort_word{nullptr};  // the context's abort word, as the resident launches see it
std::mutex log_mu;

void run(std::function<void()> f) {
  if (capture) capture->push_back(std::move(f));
  else f();
}
double now() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}
void violation(const char* what, int a, int b) {
  std::lock_guard<std::mutex> lk(log_mu);
  std::printf("  VIOLATION: %s (%d vs %d)\n", what, a, b);
  violations++;
}
}  // namespace mock

hipError_t hipGetDeviceCount(int* n) {
  *n = 1;
  return hipSuccess;
}
hipError_t hipSetDevice(int d) { return d == 0 ? hipSuccess : hipErrorInvalidValue; }
const char* hipGetErrorName(hipError_t e) { return e == hipSuccess ? "hipSuccess" : "hipError(mock)"; }
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) {
  *s = new ihipStream_t();
  return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) {
  delete s;
  return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipHostMalloc(void** p, size_t bytes, unsigned) {
  *p = std::malloc(bytes ? bytes : 1);
  return *p ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipHostFree(void* p) {
  std::free(p);
  return hipSuccess;
}
hipError_t hipMemcpy(void* dst, const void* src, size_t bytes, hipMemcpyKind) {
  std::memcpy(dst, src, bytes);
  return hipSuccess;
}
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t bytes, hipMemcpyKind, hipStream_t) {
  mock::run([=] { std::memcpy(dst, src, bytes); });
  return hipSuccess;
}
hipError_t hipMemsetAsync(void* dst, int v, size_t bytes, hipStream_t) {
  mock::run([=] { std::memset(dst, v, bytes); });
  return hipSuccess;
}
hipError_t hipEventCreate(hipEvent_t* e) {
  *e = new ihipEvent_t();
  return hipSuccess;
}
hipError_t hipEventDestroy(hipEvent_t e) {
  delete e;
  return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t) {
  mock::run([=] { e->t = mock::now(); });
  return hipSuccess;
}
hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b) {
  *ms = (float)((b->t - a->t) * 1e3);
  return hipSuccess;
}
hipError_t hipStreamBeginCapture(hipStream_t, hipStreamCaptureMode) {
  if (mock::capture) return hipErrorInvalidValue;
  mock::capture = new std::vector<std::function<void()>>();
  return hipSuccess;
}
hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t* g) {
  if (!mock::capture) return hipErrorInvalidValue;
  *g = new ihipGraph{std::move(*mock::capture)};
  delete mock::capture;
  mock::capture = nullptr;
  return hipSuccess;
}
hipError_t hipGraphInstantiate(hipGraphExec_t* x, hipGraph_t g, hipGraphNode_t*, char*, size_t) {
  *x = new hipGraphExec{g->ops};
  return hipSuccess;
}
hipError_t hipGraphDestroy(hipGraph_t g) {
  delete g;
  return hipSuccess;
}
hipError_t hipGraphExecDestroy(hipGraphExec_t x) {
  delete x;
  return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t x, hipStream_t) {
  for (auto& f : x->ops) f();
  return hipSuccess;
}

// ---------------------------------------------------------------------------
// mock kernels
// ---------------------------------------------------------------------------
namespace pdk {

bool size_supported(int n) {
  for (int m : {8, 16, 24, 32, 48, 64, 96, 128, 192, 256, 288, 384, 512, 576, 768})
    if (n == m) return true;
  return false;
}
int blue_len(int n) {
  if (n < 2) return 0;
  for (int m : {8, 16, 24, 32, 48, 64, 96, 128, 192, 256, 288, 384, 512, 576, 768})
    if (m >= 2 * n - 1) return m;
  return 0;
}

namespace {
bool fp64 = false;   // precision of the context under test

size_t plane_of(const Vol& V) { return (size_t)V.nx * V.ny; }
double get_count(const Vol& V, int pair) {
  return fp64 ? ((const double*)V.chi)[2 * pair * plane_of(V)] : ((const float*)V.chi)[2 * pair * plane_of(V)];
}
void add_count(const Vol& V, int pair, double k) {
  if (fp64) ((double*)V.chi)[2 * pair * plane_of(V)] += k;
  else ((float*)V.chi)[2 * pair * plane_of(V)] += (float)k;
}
// every workgroup of a launch maps to an existing pair of its volume
void check_cover(const Vol* vols, const Range* ranges, int nranges, int groups, int grid, const char* what) {
  for (int b = 0; b < grid; ++b) {
    int slot, pair, g;
    find_work_b(ranges, nranges, groups, b, slot, pair, g);
    if (pair < 0 || pair >= vols[slot].P) mock::violation(what, pair, vols[slot].P);
  }
}
void sleep_step() {
  int us = mock::step_sleep_us.load();
  if (us > 0) std::this_thread::sleep_for(std::chrono::microseconds(us));
}
}  // namespace

int plan_count(int n) { return (n == 64 || n == 128) ? 2 : 1; }

hipError_t launch_col_p(int n, int, int, int grid, int groups, const Vol* vols, const Range* ranges, int nranges,
                        Ctl*, int, int precision, int ext, int plan, hipStream_t) {
  if (plan < 0 || plan >= plan_count(n) || (plan && (precision || ext))) return hipErrorInvalidValue;
  mock::run([=] { check_cover(vols, ranges, nranges, groups, grid, "column launch covers a pair out of range"); });
  return hipSuccess;
}

hipError_t launch_row_p(int n, int mode, int, int grid, int groups, const Vol* vols, const Range* ranges,
                        int nranges, Ctl* ctl, int it, int precision, int ext, int plan, hipStream_t) {
  if (plan < 0 || plan >= plan_count(n) || (plan && (precision || ext))) return hipErrorInvalidValue;
  mock::run([=] {
    check_cover(vols, ranges, nranges, groups, grid, "row launch covers a pair out of range");
    if (mode == ROW_ITER) {
      mock::row_launches++;
      sleep_step();
      for (int b = 0; b < grid; b += groups) {
        int slot, pair, g;
        find_work_b(ranges, nranges, groups, b, slot, pair, g);
        const Vol& V = vols[slot];
        if (ctl[slot].stop || it >= V.iters || V.check_only) continue;
        add_count(V, pair, 1.0);
      }
    } else if (mode == ROW_INV_PLANAR) {   // the operator: out = in (the mock's A is the identity)
      for (int b = 0; b < grid; b += groups) {
        int slot, pair, g;
        find_work_b(ranges, nranges, groups, b, slot, pair, g);
        const Vol& V = vols[slot];
        const size_t n = (size_t)V.nx * V.ny * V.nz * (fp64 ? 8 : 4);
        if (pair == 0) std::memcpy(V.user_out, V.user_in, n);
      }
    }
  });
  return hipSuccess;
}

hipError_t launch_col(int n, int mode, int cols, int grid, int groups, const Vol* vols, const Range* ranges,
                      int nranges, Ctl* ctl, int it, int precision, int ext, hipStream_t st) {
  return launch_col_p(n, mode, cols, grid, groups, vols, ranges, nranges, ctl, it, precision, ext, 0, st);
}
hipError_t launch_row(int n, int mode, int rows, int grid, int groups, const Vol* vols, const Range* ranges,
                      int nranges, Ctl* ctl, int it, int precision, int ext, hipStream_t st) {
  return launch_row_p(n, mode, rows, grid, groups, vols, ranges, nranges, ctl, it, precision, ext, 0, st);
}

hipError_t launch_reduce(int nslots, const Vol* vols, const int* slots, Ctl* ctl, int it, int, hipStream_t) {
  mock::run([=] {
    for (int i = 0; i < nslots; ++i) {
      const int slot = slots[i];
      const Vol& V = vols[slot];
      if (ctl[slot].stop || it != V.iters - 1 || !V.check_last) continue;
      const int n = V.done_base + it + 1;   // check-only: done_base = -1, it = 0
      // in a round whose resident launch gave up, the volumes it covered hold
      // no consistent iterate; the host discards their checks and restarts them
      int* ab = mock::abort_word.load();
      if (!(ab && *ab))
        for (int p = 0; p < V.P; ++p)
          if ((int)get_count(V, p) != n) mock::violation("pair iterations at a gap check", (int)get_count(V, p), n);
      const double rel = 1.0 / (n + 1.0);
      Ctl& C = ctl[slot];
      C.primal = 1.0;
      C.dual = 1.0 - rel;
      C.rel_gap = rel;
      C.max_ay = 0.0;
      C.stop_iter = n;
      C.checks += 1;
      if (it == V.final_it || (V.gap_tol > 0.0 && rel <= V.gap_tol)) C.stop = 1;
    }
  });
  return hipSuccess;
}

hipError_t launch_store_chi(const Vol* vols, int slot, size_t, int, hipStream_t) {
  mock::run([=] {
    const Vol& V = vols[slot];
    const size_t plane = plane_of(V);
    for (int z = 0; z < V.nz; ++z) {
      const int pair = V.unpacked ? z : z / 2;
      const double c = get_count(V, pair);
      for (size_t o = 0; o < plane; ++o) {
        if (fp64) ((double*)V.user_out)[z * plane + o] = c;
        else ((float*)V.user_out)[z * plane + o] = (float)c;
      }
    }
  });
  return hipSuccess;
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t) {
  if (bytes == 0) return hipSuccess;
  if (((uintptr_t)p & 15) != 0) return hipErrorInvalidValue;
  mock::run([=] { std::memset(p, 0, bytes); });
  return hipSuccess;
}

hipError_t launch_tv_setup(const Vol*, Ctl*, int, size_t, int, hipStream_t) { return hipSuccess; }

namespace {
constexpr int kTeam = 4;
hipError_t mock_resident(int nteams, const Vol* vols, const Range* ranges, int nranges, Ctl* ctl, unsigned*,
                         int* abort_flag, int, unsigned spin_limit, hipStream_t) {
  mock::run([=] {
    mock::resident_launches++;
    mock::abort_word = abort_flag;
    if (*abort_flag) return;   // an earlier launch of the round gave up
    check_cover(vols, ranges, nranges, kTeam, nteams * kTeam, "resident launch covers a pair out of range");
    int forced = mock::force_aborts.load();
    bool give_up = spin_limit == 0;
    while (!give_up && forced > 0 && !mock::force_aborts.compare_exchange_weak(forced, forced - 1)) {
    }
    give_up |= forced > 0;
    sleep_step();
    for (int t = 0; t < nteams; ++t) {
      int slot, pair, m;
      find_work_b(ranges, nranges, kTeam, t * kTeam, slot, pair, m);
      const Vol& V = vols[slot];
      if (ctl[slot].stop || V.iters <= 0 || V.check_only) continue;
      // a launch that gives up leaves its pairs at no consistent iterate
      add_count(V, pair, give_up ? (t % 2 ? 1000.0 : 0.5) : (double)V.iters);
    }
    if (give_up) *abort_flag = 1;
  });
  return hipSuccess;
}
hipError_t mock_resident_multi(int quota, const Vol* vols, const Range* table, Ctl* ctl, unsigned*, int* abort_flag,
                               int ticket_base, int, unsigned spin_limit, hipStream_t) {
  mock::run([=] {
    mock::resident_launches++;
    mock::multi_launches++;
    mock::abort_word = abort_flag;
    if (*abort_flag) return;
    const int nteams = table[kXcds].first;
    if (ticket_base < nteams) mock::violation("multi launch: ticket base below the team count", ticket_base, nteams);
    const Range* teams = table + kXcds + 1;
    for (int x = 0; x < kXcds; ++x) {   // each XCD's teams: consecutive tickets within the quota
      int ticket = 0;
      for (int t = table[x].first; t < table[x + 1].first; ++t) {
        if (teams[t].first != ticket) mock::violation("multi launch: team ticket", teams[t].first, ticket);
        ticket += kTeam;
      }
      if (ticket > quota) mock::violation("multi launch: XCD over its quota", ticket, quota);
    }
    int forced = mock::force_aborts.load();
    bool give_up = spin_limit == 0;
    while (!give_up && forced > 0 && !mock::force_aborts.compare_exchange_weak(forced, forced - 1)) {
    }
    give_up |= forced > 0;
    sleep_step();
    for (int t = 0; t < nteams; ++t) {
      const Vol& V = vols[teams[t].slot];
      if (teams[t].pair0 < 0 || teams[t].pair0 >= V.P) mock::violation("multi launch: pair", teams[t].pair0, V.P);
      if (ctl[teams[t].slot].stop || V.iters <= 0 || V.check_only) continue;
      add_count(V, teams[t].pair0, give_up ? (t % 2 ? 1000.0 : 0.5) : (double)V.iters);
    }
    if (give_up) *abort_flag = 1;
  });
  return hipSuccess;
}
int mock_max_teams() { return 16; }
int mock_team() { return kTeam; }
int mock_threads() { return 256; }
int mock_plan() { return 0; }
const ResidentVariant kVariants[] = {{64, mock_resident, mock_max_teams, mock_team, mock_threads, mock_plan},
                                     {128, mock_resident, mock_max_teams, mock_team, mock_threads, mock_plan},
                                     {256, mock_resident, mock_max_teams, mock_team, mock_threads, mock_plan}};
}  // namespace

namespace {
alignas(256) unsigned char g_scratch[1 << 20];   // the mock's "static scratch" (sizes are checked on the host)
std::mutex g_scratch_mu;
}  // namespace
hipError_t static_scratch(int, void** ptr) {
  *ptr = g_scratch;
  return hipSuccess;
}
std::mutex& static_scratch_lock(int) { return g_scratch_mu; }

int multi_body(int n, int plan) { return plan != 0 ? -1 : n == 64 ? 0 : n == 128 ? 1 : n == 256 ? 2 : -1; }
int multi_team(int n, int plan) { return multi_body(n, plan) >= 0 ? kTeam : 0; }
int multi_max_groups_per_xcd() { return 8; }
hipError_t launch_resident_multi(int quota, const Vol* vols, const Range* table, Ctl* ctl, unsigned* counters,
                                 int* abort_flag, int ticket_base, int fenced, unsigned spin_limit, hipStream_t st) {
  return mock_resident_multi(quota, vols, table, ctl, counters, abort_flag, ticket_base, fenced, spin_limit, st);
}

int resident_variant_count(int n) {
  int k = 0;
  for (auto& v : kVariants) k += v.n == n;
  return k;
}
const ResidentVariant* resident_variant(int n, int v) {
  for (auto& r : kVariants)
    if (r.n == n && v-- == 0) return &r;
  return nullptr;
}
// the scenarios here submit no TV-model requests
const ResidentVariant* resident_tv_variant(int) { return nullptr; }

}  // namespace pdk

// ---------------------------------------------------------------------------
// tests
// ---------------------------------------------------------------------------
namespace {

int failures = 0;
#define EXPECT(cond, ...)                                  \
  do {                                                     \
    if (!(cond)) {                                         \
      std::printf("  FAIL %s:%d: %s: ", __FILE__, __LINE__, #cond); \
      std::printf(__VA_ARGS__);                            \
      std::printf("\n");                                   \
      ++failures;                                          \
    }                                                      \
  } while (0)

struct Arena {
  void* p = nullptr;
  size_t bytes = 0;
  explicit Arena(size_t b) : bytes(b) { p = std::aligned_alloc(256, b); }
  ~Arena() { std::free(p); }
};

struct Ctx {
  pd_ctx* c = nullptr;
  Arena arena;
  Ctx(size_t arena_bytes, int flags = 0, int max_slots = 0, int step_iters = 0) : arena(arena_bytes) {
    mock::abort_word = nullptr;   // the previous context's word is gone
    pd_config cfg{};
    cfg.device = 0;
    cfg.arena = arena.p;
    cfg.arena_bytes = arena.bytes;
    cfg.max_slots = max_slots;
    cfg.step_iters = step_iters;
    cfg.flags = flags;
    pd_status s = pd_create(&cfg, &c);
    if (s != PD_OK) {
      std::printf("  pd_create failed: %d\n", s);
      std::exit(1);
    }
  }
  ~Ctx() {
    if (c) pd_destroy(c);
  }
};

struct Req {
  pd_request r{};
  std::vector<float> delta, chi;
  int expect = 0;   // iterations the parameters imply
};

// A request whose mock gap check stops it at the first check n (a multiple
// of check_every) with 1/(n+1) <= gap_tol, or at max_iter.
Req make_req(int nx, int ny, int nz, int max_iter, int stop_at = 0, int check_every = 10, int kernel = 0) {
  Req q;
  q.r.nx = nx;
  q.r.ny = ny;
  q.r.nz = nz;
  q.r.b0[1] = 1.0;
  q.r.voxel[0] = q.r.voxel[1] = 1.0;
  q.r.voxel_z = 1.0;
  q.r.kernel = kernel;
  q.r.lambda = 1e-3;
  q.r.tau = q.r.sigma = 0.5;
  q.r.theta = 1.0;
  q.r.max_iter = max_iter;
  q.r.check_every = check_every;
  q.r.gap_tol = stop_at > 0 ? 1.0 / (stop_at + 1.0) : 0.0;
  q.delta.assign((size_t)nx * ny * nz, 0.f);
  q.chi.assign((size_t)nx * ny * nz, -1.f);
  q.r.delta = q.delta.data();
  q.r.chi = q.chi.data();
  if (stop_at > 0) {
    int n = ((stop_at + check_every - 1) / check_every) * check_every;
    q.expect = n < max_iter ? n : max_iter;
  } else {
    q.expect = max_iter;
  }
  return q;
}

bool output_is(const Req& q, float v) {
  for (float x : q.chi)
    if (x != v) return false;
  return true;
}

void check_done(pd_ctx* c, uint64_t t, Req& q, const char* what) {
  pd_result res{};
  pd_status s = pd_poll(c, t, &res, -1);
  EXPECT(s == PD_OK && res.status == PD_OK, "%s: status %d", what, s);
  EXPECT(res.iterations == q.expect, "%s: iterations %d, expected %d", what, res.iterations, q.expect);
  EXPECT(output_is(q, (float)q.expect), "%s: chi does not hold %d everywhere (first %g)", what, q.expect,
         (double)q.chi[0]);
  if (q.r.gap_tol > 0.0 && q.expect < q.r.max_iter)
    EXPECT(res.rel_gap <= q.r.gap_tol, "%s: stopped at rel_gap %g > %g", what, res.rel_gap, q.r.gap_tol);
}

std::vector<uint64_t> submit(pd_ctx* c, std::vector<Req*> qs) {
  std::vector<pd_request> rs;
  for (Req* q : qs) rs.push_back(q->r);
  std::vector<uint64_t> t(qs.size());
  pd_status s = pd_solve_batch(c, rs.data(), (int)rs.size(), t.data());
  EXPECT(s == PD_OK, "pd_solve_batch: %d", s);
  return t;
}

// ---- tests -----------------------------------------------------------------

void t_single() {
  for (int flags : {0, (int)PD_FLAG_NO_GRAPHS, (int)PD_FLAG_NO_RESIDENT}) {
    Ctx x(64 << 20, flags);
    Req a = make_req(64, 64, 3, 1234);           // resident shape, odd nz
    Req b = make_req(96, 64, 5, 777);            // two-launch shape (graphs unless disabled)
    Req c = make_req(8, 8, 1, 0);                // check-only request: chi_0 = 0
    auto t = submit(x.c, {&a, &b, &c});
    check_done(x.c, t[0], a, "64x64x3");
    check_done(x.c, t[1], b, "96x64x5");
    check_done(x.c, t[2], c, "8x8x1 max_iter 0");
    pd_result r{};
    EXPECT(pd_poll(x.c, t[0], &r, 0) == PD_ERR_TICKET, "second poll of a ticket");
  }
}

void t_gap_stops() {
  Ctx x(256 << 20);
  std::vector<Req> qs;
  qs.push_back(make_req(64, 64, 4, 1000, 100, 30));    // stops at 120
  qs.push_back(make_req(64, 64, 2, 1000, 7, 1));       // stops at 7
  qs.push_back(make_req(128, 128, 6, 95, 500, 10));    // cap first: 95
  qs.push_back(make_req(96, 64, 3, 1000, 333, 50));    // two-launch, stops at 350
  qs.push_back(make_req(16, 16, 4, 60, 0, 10, PD_KERNEL_DIPOLE_3D));   // 3-D kernel (z view)
  std::vector<Req*> ps;
  for (auto& q : qs) ps.push_back(&q);
  auto t = submit(x.c, ps);
  for (size_t i = 0; i < qs.size(); ++i) check_done(x.c, t[i], qs[i], "gap-stop mix");
}

void t_staggered_arrivals() {
  // requests arrive while others run: rounds with mid-round stops, admission
  // between rounds, volumes split across resident launches (16 teams of 4)
  mock::step_sleep_us = 50;
  Ctx x(512 << 20);
  std::vector<Req> qs;
  for (int i = 0; i < 24; ++i) {
    int shape = i % 4;
    int nx = shape == 0 ? 64 : shape == 1 ? 128 : shape == 2 ? 96 : 256;
    int ny = shape == 2 ? 64 : nx;
    int nz = 1 + (i * 7) % 40;
    int stop = (i % 3 == 0) ? 40 + 13 * i : 0;
    qs.push_back(make_req(nx, ny, nz, 150 + 37 * i, stop, 10 + i % 3));
  }
  std::vector<uint64_t> t;
  for (auto& q : qs) {
    auto tt = submit(x.c, {&q});
    t.push_back(tt[0]);
    std::this_thread::sleep_for(std::chrono::microseconds(300));
  }
  for (size_t i = 0; i < qs.size(); ++i) check_done(x.c, t[i], qs[i], "staggered");
  mock::step_sleep_us = 0;
}

void t_admission_fifo() {
  // an arena that holds about two of these requests at once
  size_t one = 0;
  Req probe = make_req(128, 128, 16, 300);
  pd_validate(&probe.r, PD_FP32, &one);
  Ctx x(2 * one + (2 << 20));
  std::vector<Req> qs;
  for (int i = 0; i < 7; ++i) qs.push_back(make_req(128, 128, 16, 300 + 10 * i));
  std::vector<Req*> ps;
  for (auto& q : qs) ps.push_back(&q);
  auto t = submit(x.c, ps);
  size_t used = 0;
  int resident = 0, queued = 0;
  pd_arena_usage(x.c, &used, &resident, &queued);
  EXPECT(used <= x.arena.bytes, "arena use %zu > %zu", used, x.arena.bytes);
  double prev = 0.0;
  for (size_t i = 0; i < qs.size(); ++i) {
    pd_result r{};
    pd_status s = pd_poll(x.c, t[i], &r, -1);
    EXPECT(s == PD_OK && r.iterations == qs[i].expect, "admission request %zu", i);
    EXPECT(output_is(qs[i], (float)qs[i].expect), "admission request %zu output", i);
    EXPECT(r.t_start >= prev, "FIFO admission: request %zu started before its predecessor", i);
    prev = r.t_start;
  }
  Req big = make_req(384, 384, 200, 10);
  uint64_t tb;
  EXPECT(pd_solve_batch(x.c, &big.r, 1, &tb) == PD_ERR_BUDGET, "request larger than the arena");
}

void t_destroy_while_polling() {
  // pollers blocked in pd_poll(-1) on requests that cannot finish soon, a
  // submitter and a status reader in flight while pd_destroy runs
  mock::step_sleep_us = 200;
  for (int round = 0; round < 3; ++round) {
    Arena arena(256 << 20);
    mock::abort_word = nullptr;
    pd_config cfg{};
    cfg.arena = arena.p;
    cfg.arena_bytes = arena.bytes;
    pd_ctx* c = nullptr;
    EXPECT(pd_create(&cfg, &c) == PD_OK, "create");
    std::vector<Req> qs;
    for (int i = 0; i < 4; ++i) qs.push_back(make_req(i % 2 ? 64 : 96, 64, 8, 1 << 28));
    std::vector<Req*> ps;
    for (auto& q : qs) ps.push_back(&q);
    auto t = submit(c, ps);
    std::atomic<int> cancelled{0}, other{0};
    std::vector<std::thread> th;
    for (int i = 0; i < 4; ++i)
      th.emplace_back([&, i] {
        pd_result r{};
        pd_status s = pd_poll(c, t[i], &r, -1);
        (s == PD_ERR_CANCELLED ? cancelled : other)++;
      });
    std::atomic<bool> stop{false};
    th.emplace_back([&] {
      while (!stop.load()) {
        size_t u;
        int a, b;
        if (pd_arena_usage(c, &u, &a, &b) == PD_ERR_CANCELLED) break;
        std::this_thread::sleep_for(std::chrono::microseconds(100));
      }
    });
    std::this_thread::sleep_for(std::chrono::milliseconds(20 + 10 * round));
    EXPECT(pd_destroy(c) == PD_OK, "destroy");
    stop = true;
    for (auto& x : th) x.join();
    EXPECT(cancelled == 4 && other == 0, "pollers: %d cancelled, %d otherwise", cancelled.load(), other.load());
  }
  mock::step_sleep_us = 0;
}

void t_recovery_forced_giveup() {
  // every resident launch gives up: the resident shapes restart on the
  // two-launch path; a two-launch shape in the same rounds is unaffected
  Ctx x(256 << 20, PD_FLAG_TEST_BARRIER_GIVEUP);
  Req a = make_req(128, 128, 9, 420, 200, 20);   // stops at 200
  Req b = make_req(96, 64, 3, 333);
  Req c = make_req(256, 256, 40, 150);           // 20 pairs: more than one resident launch
  auto t = submit(x.c, {&a, &b, &c});
  check_done(x.c, t[0], a, "restarted 128x128x9");
  check_done(x.c, t[1], b, "two-launch 96x64x3");
  check_done(x.c, t[2], c, "restarted 256x256x40");
  int64_t ab = 0, rs = 0;
  pd_recovery_stats(x.c, &ab, &rs);
  EXPECT(ab >= 1 && rs >= 2, "recovery stats %lld rounds, %lld requests", (long long)ab, (long long)rs);
  // later requests of those shapes: two-launch from the start
  long before = mock::resident_launches.load();
  Req d = make_req(128, 128, 4, 90);
  auto t2 = submit(x.c, {&d});
  check_done(x.c, t2[0], d, "after recovery");
  EXPECT(mock::resident_launches.load() == before, "resident launches after the shape was demoted");
  int64_t ab2 = 0;
  pd_recovery_stats(x.c, &ab2, nullptr);
  EXPECT(ab2 == ab, "no further give-up");
  // tuner: resident variants give up and are skipped, the context lives on
  pd_tune_entry e[8];
  int n = 0;
  EXPECT(pd_tune(x.c, 64, 64, 4, 5, e, 8, &n) == PD_OK, "tune under give-up");
  for (int i = 0; i < n; ++i) EXPECT(e[i].path != 0, "tuner kept a resident variant that gave up");
  // an explicit resident choice re-enables the shape
  EXPECT(pd_tune_set(x.c, 128, 128, 0, 0, 0, 0, 0) == PD_OK, "tune_set");
  Req f = make_req(128, 128, 2, 50);
  auto t3 = submit(x.c, {&f});
  check_done(x.c, t3[0], f, "re-enabled shape gives up again and recovers");
}

void t_recovery_midway() {
  // one resident launch fails in the middle of a long multi-round solve
  mock::step_sleep_us = 300;
  Ctx x(256 << 20, 0, 0, 50);
  Req a = make_req(64, 64, 6, 700);
  Req b = make_req(64, 64, 2, 480, 300, 30);
  auto t = submit(x.c, {&a, &b});
  std::this_thread::sleep_for(std::chrono::milliseconds(1));
  mock::force_aborts = 1;
  check_done(x.c, t[0], a, "64x64x6 after a mid-solve give-up");
  check_done(x.c, t[1], b, "64x64x2 after a mid-solve give-up");
  int64_t ab = 0;
  pd_recovery_stats(x.c, &ab, nullptr);
  EXPECT(ab == 1, "one aborted round, got %lld", (long long)ab);
  mock::force_aborts = 0;
  mock::step_sleep_us = 0;
}

void t_tuned_plans() {
  // the tuner times every plan of each kernel; a chosen plan reaches the
  // launches (the mock rejects plans a length does not have)
  Ctx x(128 << 20, PD_FLAG_NO_RESIDENT);
  pd_tune_entry e[32];
  int n = 0;
  EXPECT(pd_tune(x.c, 128, 64, 8, 5, e, 32, &n) == PD_OK, "tune");
  int cols_plans = 0, rows_plans = 0;
  for (int i = 0; i < n; ++i) {
    cols_plans += e[i].path == 1 && e[i].plan == 1;
    rows_plans += e[i].path == 2 && e[i].plan == 1;
  }
  EXPECT(cols_plans >= 1 && rows_plans >= 1, "plans timed: %d column, %d row", cols_plans, rows_plans);
  EXPECT(pd_tune_set(x.c, 128, 64, -1, 8, 8, 1, 1) == PD_OK, "set plans");
  int v, r, cl, px, py;
  EXPECT(pd_tune_get(x.c, 128, 64, &v, &r, &cl, &px, &py) == PD_OK && px == 1 && py == 1, "get plans");
  EXPECT(pd_tune_set(x.c, 96, 64, -1, 8, 8, 1, 0) == PD_ERR_ARG, "96 has one plan in the mock");
  Req q = make_req(128, 64, 6, 137, 90, 30);
  auto t = submit(x.c, {&q});
  check_done(x.c, t[0], q, "solve under tuned plans");
}

void t_multi_shape() {
  // resident shapes of one step share multi-shape launches (8 workgroups per
  // XCD in the mock: 16 teams of 4 per launch, so 30 pairs need two)
  Ctx x(512 << 20);
  long before = mock::multi_launches.load();
  Req a = make_req(64, 64, 7, 240, 150, 30);
  Req b = make_req(128, 128, 20, 300);
  Req c = make_req(256, 256, 33, 170, 0, 10);
  Req d = make_req(96, 64, 5, 260);
  auto t = submit(x.c, {&a, &b, &c, &d});
  check_done(x.c, t[0], a, "64x64x7 in a multi-shape launch");
  check_done(x.c, t[1], b, "128x128x20 in a multi-shape launch");
  check_done(x.c, t[2], c, "256x256x33 in a multi-shape launch");
  check_done(x.c, t[3], d, "96x64x5 beside them");
  EXPECT(mock::multi_launches.load() > before, "no multi-shape launch ran");
}

void t_apply_kernel() {
  Ctx x(64 << 20);
  Req q = make_req(48, 32, 5, 0);
  for (size_t i = 0; i < q.delta.size(); ++i) q.delta[i] = (float)i;
  EXPECT(pd_apply_kernel(x.c, &q.r) == PD_OK, "apply");
  EXPECT(q.chi == q.delta, "mock operator output");
  std::fill(q.chi.begin(), q.chi.end(), -1.f);
  EXPECT(pd_apply_kernel_noalloc(x.c, &q.r) == PD_OK, "apply, static scratch");
  EXPECT(q.chi == q.delta, "mock operator output, static scratch");
  Req big = make_req(768, 768, 64, 0);   // 32 pairs of 768^2: 151 MB of field
  EXPECT(pd_apply_kernel_noalloc(x.c, &big.r) == PD_ERR_SCRATCH, "too large for the static scratch");
  size_t used;
  int res, qd;
  pd_arena_usage(x.c, &used, &res, &qd);
  EXPECT(res == 0 && qd == 0, "apply leaves no request resident");
}

struct Test {
  const char* name;
  void (*fn)();
};
const Test kTests[] = {{"single", t_single},
                       {"gap_stops", t_gap_stops},
                       {"staggered", t_staggered_arrivals},
                       {"admission_fifo", t_admission_fifo},
                       {"destroy_while_polling", t_destroy_while_polling},
                       {"recovery_forced_giveup", t_recovery_forced_giveup},
                       {"recovery_midway", t_recovery_midway},
                       {"tuned_plans", t_tuned_plans},
                       {"multi_shape", t_multi_shape},
                       {"apply_kernel", t_apply_kernel}};

}  // namespace

int main(int argc, char** argv) {
  int ran = 0;
  for (const Test& t : kTests) {
    if (argc > 1 && std::strcmp(argv[1], t.name) != 0) continue;
    const int f0 = failures, v0 = mock::violations.load();
    t.fn();
    std::printf("%s %s\n", (failures == f0 && mock::violations.load() == v0) ? "pass" : "FAIL", t.name);
    std::fflush(stdout);
    ++ran;
  }
  if (failures || mock::violations.load()) {
    std::printf("failed: %d expectations, %d violations\n", failures, mock::violations.load());
    return 1;
  }
  std::printf("ok %d\n", ran);
  return 0;
}
