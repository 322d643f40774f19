// The TV model's resident variants (pd_resident_tv.hpp) of the square slice
// shapes 64x64, 128x128 and 256x256: teams of 4 and 8 workgroups of 256
// threads (16 rows and 16 columns per member) and of 8 workgroups of 512
// threads (32 rows and columns; 7% faster at 256x256x64 than 16 x 256, while
// 512-thread members were slower at 64x64 and 128x128), default FFT plans.
// Every row and column transform is the one the four-launch TV kernels run
// at the same plan (the rows or columns per workgroup do not change a
// sequence's arithmetic).
#include "pd_resident_tv.hpp"

PD_INSTANTIATE_RESIDENT_TV(64, 4, 256, 0)
PD_INSTANTIATE_RESIDENT_TV(128, 8, 256, 0)
PD_INSTANTIATE_RESIDENT_TV(256, 8, 512, 0)

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
