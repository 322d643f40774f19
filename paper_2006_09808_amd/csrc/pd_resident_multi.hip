// The multi-shape resident launch: teams of 64x64, 128x128, 192x192 and
// 256x256 slice pairs in one launch of 256-thread workgroups at two waves per
// SIMD.  A body is a shape's 256-thread variant on one FFT plan (64, 192 and
// 256: the default; 128: the default and 8 x 4 x 4), so a volume gives the
// same bits here as in its own launch of any variant of that plan.  The
// 192x192 body spills part of its state to scratch here, as the two-wave
// 192x192 variants do in their own launches.
#include "pd_resident.hpp"

namespace pdk {

namespace {
using B64 = Resident<64, 64, 2, 256, 0>;
using B128 = Resident<128, 128, 4, 256, 0>;
using B128p2 = Resident<128, 128, 8, 256, 2>;
using B256 = Resident<256, 256, 16, 256, 0>;
using B192 = Resident<192, 192, 12, 256, 0>;
constexpr int kMultiThreads = 256;
}  // namespace

int multi_body(int n, int plan) {
  if (n == 64 && plan == 0) return 0;
  if (n == 128 && plan == 0) return 1;
  if (n == 128 && plan == 2) return 2;
  if (n == 256 && plan == 0) return 3;
  if (n == 192 && plan == 0) return 4;
  return -1;
}

int multi_team(int n, int plan) {
  switch (multi_body(n, plan)) {
    case 0: return B64::kTeam;
    case 1: return B128::kTeam;
    case 2: return B128p2::kTeam;
    case 3: return B256::kTeam;
    case 4: return B192::kTeam;
    default: return 0;
  }
}

int multi_max_groups_per_xcd() {
  int per_cu = 0, dev = 0, ncu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &per_cu, (const void*)k_resident_multi<kMultiThreads, B64, B128, B128p2, B256, B192>, kMultiThreads, 0) !=
      hipSuccess)
    return 0;
  return per_cu * (ncu / kXcds);
}

hipError_t launch_resident_multi(int quota, const Vol* vols, const Range* table, Ctl* ctl, unsigned* counters,
                                 int* abort_flag, int ticket_base, int fenced, unsigned spin_limit, hipStream_t st) {
  hipLaunchKernelGGL((k_resident_multi<kMultiThreads, B64, B128, B128p2, B256, B192>), dim3(quota * kXcds),
                     dim3(kMultiThreads), 0, st, vols, table, ctl, counters, abort_flag, ticket_base, quota, fenced,
                     spin_limit);
  return hipGetLastError();
}

}  // namespace pdk
