// The TV model's resident variants (pd_resident_tv.hpp) of the square slice
// shapes 64x64, 128x128 and 256x256: teams of 4, 8 and 16 workgroups of 256
// threads (16 rows and 16 columns per member), default FFT plans.  With these
// tiles every row and column transform is the one the two-launch TV kernels
// run at their default tiles.
#include "pd_resident_tv.hpp"

PD_INSTANTIATE_RESIDENT_TV(64, 4, 256, 0)
PD_INSTANTIATE_RESIDENT_TV(128, 8, 256, 0)
PD_INSTANTIATE_RESIDENT_TV(256, 16, 256, 0)

namespace pdk {

#define PD_TV_ENTRY(N) \
  {N, launch_resident_tv_##N, resident_tv_max_teams_##N, resident_tv_team_##N, resident_tv_threads_##N, \
   resident_tv_plan_##N},
static const ResidentVariant kResidentTv[] = {PD_TV_ENTRY(64) PD_TV_ENTRY(128) PD_TV_ENTRY(256)};
#undef PD_TV_ENTRY

const ResidentVariant* resident_tv_variant(int n) {
  for (const auto& r : kResidentTv)
    if (r.n == n) return &r;
  return nullptr;
}

}  // namespace pdk
