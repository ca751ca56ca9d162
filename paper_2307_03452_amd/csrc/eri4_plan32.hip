// eri4_plan32.hip -- the persistent plan kernel with FP32 transforms, shells read from per-quartet arrays.
#include "eri4_device.h"

namespace eri4 {
hipError_t plan_set_attrs_f32() { return plan_set_attrs_t<true, false>(); }
hipError_t plan_occupancy_f32(int lds_bytes, int* per_cu) {
  return plan_occupancy_t<true, false>(lds_bytes, per_cu);
}
hipError_t plan_launch_f32(dim3 grid, int lds_bytes, hipStream_t s, const Tables& t, const PlanArgs& a) {
  return plan_launch_t<true, false>(grid, lds_bytes, s, t, a);
}
}  // namespace eri4
