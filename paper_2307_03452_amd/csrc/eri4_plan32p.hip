// eri4_plan32p.hip -- the persistent plan kernel with FP32 transforms, shells read from a bra and a ket list of shell pairs.
#include "eri4_device.h"

namespace eri4 {
hipError_t plan_set_attrs_f32p() { return plan_set_attrs_t<true, true>(); }
hipError_t plan_occupancy_f32p(int lds_bytes, int* per_cu) {
  return plan_occupancy_t<true, true>(lds_bytes, per_cu);
}
hipError_t plan_launch_f32p(dim3 grid, int lds_bytes, hipStream_t s, const Tables& t, const PlanArgs& a) {
  return plan_launch_t<true, true>(grid, lds_bytes, s, t, a);
}
}  // namespace eri4
