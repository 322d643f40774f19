// pd_solve_file - the solver through its C ABI alone (no Python, no torch):
// reads a field map, solves every slice with the L1 model, writes chi.
//
//   pd_solve_file nx ny nz lambda max_iter delta.f32 chi.f32
//
// delta.f32 / chi.f32: nz*ny*nx float32 values, x fastest.  B0 along y, unit
// voxels, tau = sigma = 1.4, theta = 1, fixed iteration count.  Prints the
// status, iteration count and duality gap of the solve.  The caller-owned
// device memory (arena, field map, result) comes from hipMalloc.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <vector>

#include "pd.h"

static int fail(const char* what, int code) {
  std::fprintf(stderr, "pd_solve_file: %s (%d)\n", what, code);
  return 1;
}

int main(int argc, char** argv) {
  if (argc != 8) {
    std::fprintf(stderr, "usage: %s nx ny nz lambda max_iter delta.f32 chi.f32\n", argv[0]);
    return 2;
  }
  const int nx = std::atoi(argv[1]), ny = std::atoi(argv[2]), nz = std::atoi(argv[3]);
  const double lam = std::atof(argv[4]);
  const int iters = std::atoi(argv[5]);
  if (nx <= 0 || ny <= 0 || nz <= 0) return fail("bad shape", 0);
  const size_t n = (size_t)nx * ny * nz;
  std::vector<float> host(n);
  FILE* f = std::fopen(argv[6], "rb");
  if (!f || std::fread(host.data(), sizeof(float), n, f) != n) return fail("cannot read the field map", 0);
  std::fclose(f);

  pd_request r = {};
  r.nx = nx;
  r.ny = ny;
  r.nz = nz;
  r.b0[1] = 1.0;
  r.voxel[0] = r.voxel[1] = 1.0;
  r.kernel = PD_KERNEL_DIPOLE;
  r.lambda = lam;
  r.tau = r.sigma = 1.4;
  r.theta = 1.0;
  r.max_iter = iters;
  r.gap_tol = 0.0;
  r.check_every = 10;
  r.model = PD_MODEL_L1;
  r.voxel_z = 1.0;
  size_t state = 0;
  pd_status st = pd_validate(&r, PD_FP32, &state);
  if (st != PD_OK) return fail(pd_status_string(st), st);

  if (hipSetDevice(0) != hipSuccess) return fail("no GPU", 0);
  const size_t arena_bytes = state + (64u << 20);     // the request plus control blocks
  void *arena = nullptr, *d_delta = nullptr, *d_chi = nullptr;
  if (hipMalloc(&arena, arena_bytes) != hipSuccess || hipMalloc(&d_delta, n * sizeof(float)) != hipSuccess ||
      hipMalloc(&d_chi, n * sizeof(float)) != hipSuccess)
    return fail("hipMalloc", 0);
  if (hipMemcpy(d_delta, host.data(), n * sizeof(float), hipMemcpyHostToDevice) != hipSuccess)
    return fail("hipMemcpy", 0);

  pd_config cfg = {};
  cfg.device = 0;
  cfg.stream = nullptr;            // the library creates its own stream
  cfg.arena = arena;
  cfg.arena_bytes = arena_bytes;
  cfg.precision = PD_FP32;
  pd_ctx* ctx = nullptr;
  if ((st = pd_create(&cfg, &ctx)) != PD_OK) return fail(pd_status_string(st), st);
  r.delta = d_delta;
  r.chi = d_chi;
  uint64_t ticket = 0;
  if ((st = pd_solve_batch(ctx, &r, 1, &ticket)) != PD_OK) return fail(pd_status_string(st), st);
  pd_result res = {};
  st = pd_poll(ctx, ticket, &res, -1);
  if (st != PD_OK) return fail(pd_status_string(st), st);
  std::printf("status %d iterations %d primal %.9e dual %.9e rel_gap %.9e\n", res.status, res.iterations,
              res.primal, res.dual, res.rel_gap);
  if (hipMemcpy(host.data(), d_chi, n * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess)
    return fail("hipMemcpy", 0);
  pd_destroy(ctx);
  (void)hipFree(d_chi);
  (void)hipFree(d_delta);
  (void)hipFree(arena);
  f = std::fopen(argv[7], "wb");
  if (!f || std::fwrite(host.data(), sizeof(float), n, f) != n) return fail("cannot write chi", 0);
  std::fclose(f);
  return 0;
}
