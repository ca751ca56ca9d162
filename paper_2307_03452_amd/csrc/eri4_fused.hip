// eri4_fused.hip -- the single-class fused kernels (FP64), one instance per
// tile height (16, 32 or, with a box layout, 64 rows) and R layout (box,
// slab, two boxes).
#include "eri4_device.h"

namespace eri4 {

namespace {
template <int RB, int LAY>
hipError_t launch_one(const ClassParams& p, dim3 grid, hipStream_t s, const Tables& t, const double* centers,
                      const double* exps, const double* coefs, const int32_t* nprim, double* out, int64_t q0) {
  hipLaunchKernelGGL((eri4_fused_kernel<RB, LAY>), grid, dim3(kThreads), p.lds_bytes, s, p, t.boys, t.rtab, centers,
                     exps, coefs, nprim, out, q0);
  return hipGetLastError();
}
}  // namespace

hipError_t fused_set_attrs() {
  const void* k[8] = {(const void*)eri4_fused_kernel<1, kLayBox>,  (const void*)eri4_fused_kernel<2, kLayBox>,
                      (const void*)eri4_fused_kernel<4, kLayBox>,  (const void*)eri4_fused_kernel<1, kLaySlab>,
                      (const void*)eri4_fused_kernel<2, kLaySlab>, (const void*)eri4_fused_kernel<1, kLayBox2>,
                      (const void*)eri4_fused_kernel<2, kLayBox2>, (const void*)eri4_fused_kernel<4, kLayBox2>};
  for (const void* f : k) {
    const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLdsBytes);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t fused_launch(const ClassParams& p, dim3 grid, hipStream_t s, const Tables& t, const double* centers,
                        const double* exps, const double* coefs, const int32_t* nprim, double* out, int64_t q0) {
  const bool two = p.rb == 2;
  switch (p.lay) {
    case kLaySlab:
      return two ? launch_one<2, kLaySlab>(p, grid, s, t, centers, exps, coefs, nprim, out, q0)
                 : launch_one<1, kLaySlab>(p, grid, s, t, centers, exps, coefs, nprim, out, q0);
    case kLayBox2:
      if (p.rb == 4) return launch_one<4, kLayBox2>(p, grid, s, t, centers, exps, coefs, nprim, out, q0);
      return two ? launch_one<2, kLayBox2>(p, grid, s, t, centers, exps, coefs, nprim, out, q0)
                 : launch_one<1, kLayBox2>(p, grid, s, t, centers, exps, coefs, nprim, out, q0);
    default:
      if (p.rb == 4) return launch_one<4, kLayBox>(p, grid, s, t, centers, exps, coefs, nprim, out, q0);
      return two ? launch_one<2, kLayBox>(p, grid, s, t, centers, exps, coefs, nprim, out, q0)
                 : launch_one<1, kLayBox>(p, grid, s, t, centers, exps, coefs, nprim, out, q0);
  }
}

#ifdef ERI4_STAGE_TIMERS
// Stage-timer build only: the per-stage cycle sums of the Cartesian fused
// kernels (kStCount counters in the order of the stage enum; the last one
// counts tiles), then zeroed if reset.  Returns 0, or 4 on a HIP error.
extern "C" int eri4_stage_cycles(unsigned long long* out, int reset) {
  hipError_t e = hipDeviceSynchronize();
  if (e == hipSuccess) e = hipMemcpyFromSymbol(out, HIP_SYMBOL(g_stage_cycles), sizeof(unsigned long long) * kStCount);
  if (e == hipSuccess && reset) {
    const unsigned long long z[kStCount] = {0};
    e = hipMemcpyToSymbol(HIP_SYMBOL(g_stage_cycles), z, sizeof z);
  }
  return e == hipSuccess ? 0 : 4;
}
#endif

}  // namespace eri4
