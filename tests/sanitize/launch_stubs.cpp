// Host-only stand-ins for the kernel launch wrappers of hk_kernels.hip, for a sanitizer build of
// the host library (hk_api.cpp) that runs without a GPU: every launch reports that no device is
// present. Only argument validation and host logic are exercised by this build.
#include "hk_internal.h"

namespace hk {
static hipError_t none() { return hipErrorNoDevice; }
hipError_t launch_validate(const double*, int64_t, unsigned long long*, int*, hipStream_t) { return none(); }
hipError_t launch_keys(const double*, const double*, const double*, const double*, const double*, int64_t, KeyMap,
                       uint32_t*, int32_t*, double*, int*, hipStream_t) { return none(); }
hipError_t launch_radix_pass(const uint32_t*, const int32_t*, uint32_t*, int32_t*, int64_t, int, uint32_t*, uint32_t*,
                             hipStream_t) { return none(); }
hipError_t launch_gather(const int32_t*, int64_t, const double*, double*, double*, double*, double*, double*,
                         hipStream_t) { return none(); }
hipError_t launch_prep(const PrepArgs&, float*, float*, double*, double*, double*, hipStream_t) { return none(); }
hipError_t launch_fill_pairs(const PairDesc*, int, PairDesc*, int*, hipStream_t) { return none(); }
hipError_t launch_worklist(const uint32_t*, int64_t, KeyMap, double, double, const PairDesc*, int, int, int, double,
                           double, int, int32_t*, int32_t*, int32_t*, int4*, int32_t*, int, double, int, double,
                           hipStream_t) { return none(); }
hipError_t launch_item_scan(const int32_t*, int, int32_t*, int*, hipStream_t) { return none(); }
hipError_t launch_gridrec(const double*, int64_t, double, double, int64_t, double, int4*, hipStream_t) { return none(); }
hipError_t launch_span_segments(const uint32_t*, int64_t, KeyMap, double, double, const PairDesc*, const PairDesc*, int,
                                int, int, double, double, const int4*, int, SpanSeg*, int32_t*, int, hipStream_t) {
  return none();
}
hipError_t launch_wing(const VoigtArgs&, int, int, hipStream_t) { return none(); }
hipError_t launch_core(const VoigtArgs&, int, int, hipStream_t) { return none(); }
hipError_t launch_combine(const VoigtArgs&, int, bool, hipStream_t) { return none(); }
hipError_t launch_cut_bounds(const double*, const int32_t*, int64_t, double, double, int64_t, double, int32_t*,
                             int32_t*, hipStream_t) { return none(); }
hipError_t launch_far(const FarArgs&, int, int, hipStream_t) { return none(); }
hipError_t launch_combine_far(const FarArgs&, hipStream_t) { return none(); }
int far_max_blocks_per_cu() { return 1; }
int adj_max_blocks_per_cu() { return 1; }
hipError_t launch_adj_nodes(const float*, int64_t, int, const double*, double*, hipStream_t) { return none(); }
hipError_t launch_adjoint(const AdjArgs&, int, hipStream_t) { return none(); }
hipError_t launch_reduce2(const double*, int64_t, double*, int, double*, hipStream_t) { return none(); }
int wing_max_blocks_per_cu(int) { return 1; }
int core_max_blocks_per_cu(int) { return 1; }
hipError_t upload_weideman(const double*, double) { return none(); }
hipError_t upload_weideman40(const double*, double) { return none(); }
hipError_t launch_gridrec_ex(const GridRecArgs&, hipStream_t) { return none(); }
hipError_t launch_direct(const VoigtArgs&, const float*, int, int, int, hipStream_t) { return none(); }
int direct_max_blocks_per_cu(int) { return 1; }
hipError_t scratch_address(void** p) {
  *p = nullptr;
  return none();
}
hipError_t launch_line_stats(const double*, const double*, int64_t, unsigned long long*, hipStream_t) { return none(); }
hipError_t launch_scatter_grec(const int4*, const float*, const int32_t*, int64_t, int32_t*, int32_t*, float*,
                               hipStream_t) { return none(); }
hipError_t launch_hitran_check(const double*, const double*, int64_t, int*, unsigned long long*, hipStream_t) {
  return none();
}
hipError_t launch_gather2(const int32_t*, int64_t, const double*, const double*, double*, double*, hipStream_t) {
  return none();
}
hipError_t launch_shift_keys(const double*, const double*, int64_t, double, KeyMap, uint32_t*, int32_t*, hipStream_t) {
  return none();
}
hipError_t launch_shift_gather(const ShiftArgs&, hipStream_t) { return none(); }
hipError_t launch_fill0(float*, int64_t, hipStream_t) { return none(); }
hipError_t launch_accumulate(float*, const float*, int64_t, hipStream_t) { return none(); }
}  // namespace hk
