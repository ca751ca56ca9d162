// eri4_launch.h -- host-side entry points to the kernels of liberi4 that are
// compiled in their own translation units (eri4_fused.hip, eri4_plan64.hip,
// eri4_plan32.hip).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "eri4_internal.h"

namespace eri4 {

// Tables every kernel reads (uploaded once per device).
struct Tables {
  const double* boys;
  const uint2* rtab;
};

// The single-class fused kernels (one launch per class and quartet chunk).
hipError_t fused_set_attrs();
hipError_t fused_launch(const ClassParams& p, dim3 grid, hipStream_t s, const Tables& t, const double* centers,
                        const double* exps, const double* coefs, const int32_t* nprim, double* out, int64_t q0);

// The persistent plan kernel, with FP64 or FP32 transforms.
struct PlanArgs {
  const ClassParams* classes;
  const int2* items;
  int nitems;
  const int64_t* qoff;
  const int32_t* nprim;
  int* counter;
  const double* centers;
  const double* exps;
  const double* coefs;
  double* out;
};
hipError_t plan_set_attrs_f64();
hipError_t plan_set_attrs_f32();
hipError_t plan_occupancy_f64(int lds_bytes, int* per_cu);
hipError_t plan_occupancy_f32(int lds_bytes, int* per_cu);
hipError_t plan_launch_f64(dim3 grid, int lds_bytes, hipStream_t s, const Tables& t, const PlanArgs& a);
hipError_t plan_launch_f32(dim3 grid, int lds_bytes, hipStream_t s, const Tables& t, const PlanArgs& a);

}  // namespace eri4
