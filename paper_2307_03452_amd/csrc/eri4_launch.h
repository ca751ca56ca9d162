// eri4_launch.h -- host-side entry points to the kernels of liberi4 that are
// compiled in their own translation units (eri4_fused.hip, eri4_small.hip,
// eri4_solid.hip, eri4_coulomb.hip, eri4_exchange.hip and the four
// eri4_plan*.hip).  Not part
// of the public ABI.
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

// One wave per quartet (eri4_small.hip) for classes whose shells all have
// l <= kSmallLMax: p from small_params (rb = bra row blocks per pass).
hipError_t small_set_attrs();
hipError_t small_launch(const ClassParams& p, int64_t nq, hipStream_t s, const Tables& t, const double* centers,
                        const double* exps, const double* coefs, const int32_t* nprim, double* out, int64_t q0);
hipError_t small4_launch(const ClassParams& p, int64_t nq, hipStream_t s, const Tables& t, const double* centers,
                         const double* exps, const double* coefs, const int32_t* nprim, double* out, int64_t q0);

// Solid-harmonic output (eri4_solid.hip): the H matrices of quartets q0..q0+nq-1
// into hbra / hket (hbs / hks doubles per primitive pair, kmax^2 pair slots
// per quartet), then the integral kernels that read them.  stab: the device
// copy of make_solid_table.
hipError_t solid_set_attrs();
hipError_t solid_h_launch(const ClassParams& p, int64_t nq, hipStream_t s, const double* centers, const double* exps,
                          const double* coefs, const int32_t* nprim, const double* stab, double* hbra, double* hket,
                          int64_t q0, int64_t hbs, int64_t hks);
hipError_t solid_launch(const ClassParams& p, dim3 grid, hipStream_t s, const Tables& t, const double* centers,
                        const double* exps, const double* coefs, const int32_t* nprim, double* out, int64_t q0,
                        const double* hbra, const double* hket, int64_t hbs, int64_t hks);

// Coulomb contraction (eri4_coulomb.hip): dket of every ket primitive pair of
// quartets q0..q0+nq-1 (ds doubles each, kmax^2 slots per quartet), then the
// J-engine kernel (J^ij of every bra primitive pair into part, kmax^2 * nab
// doubles per quartet) and the sum over bra pairs into out.  p from
// jengine_params.
hipError_t coulomb_set_attrs();
hipError_t coulomb_dket_launch(const ClassParams& p, int64_t nq, hipStream_t s, const double* centers,
                               const double* exps, const double* coefs, const int32_t* nprim, const double* dens,
                               double* dket, int64_t q0, int64_t ds);
hipError_t coulomb_launch(const ClassParams& p, int64_t nq, hipStream_t s, const Tables& t, const double* centers,
                          const double* exps, const double* coefs, const int32_t* nprim, double* part, double* out,
                          int64_t q0, const double* dket, int64_t ds);

// Exchange contraction (eri4_exchange.hip): F^b of every ket primitive pair
// and shell-b component of quartets q0..q0+nq-1 (fbs doubles each), the
// integral kernels writing the partial rows y^b into part, and the sum over b
// into out (K [q][Na][Nc]).
hipError_t exchange_set_attrs();
hipError_t exchange_launch(const ClassParams& p, int64_t nq, hipStream_t s, const Tables& t, const double* centers,
                           const double* exps, const double* coefs, const int32_t* nprim, const double* dens,
                           double* fb, int64_t fbs, double* part, double* out, int64_t q0);

// Where the shells of quartet q come from: per-quartet arrays (nket == 0:
// centers [q][4][3], exps/coefs [q][4][kmax]), or a bra and a ket list of
// shell pairs (quartet q = bra pair q / nket with ket pair q % nket; each list
// centers [i][2][3], exps/coefs [i][2][kmax]).
struct Shells {
  const double* centers;  // quartets, or bra pairs
  const double* exps;
  const double* coefs;
  const double* kcenters;  // ket pairs (nket > 0)
  const double* kexps;
  const double* kcoefs;
  int64_t nket;
};

// The persistent plan kernel, with FP64 or FP32 transforms (f64 / f32), shells
// from per-quartet arrays or, with the suffix p, from pair lists.
struct PlanArgs {
  const ClassParams* classes;
  const int2* items;
  int nitems;
  const int64_t* qoff;
  const int32_t* nprim;
  int* counter;
  Shells shells;
  double* out;
};
// Solid-harmonic plans (eri4_solid.hip): H of every list entry (pl, pn: l and
// contraction lengths per entry; bra entries first for pair-list plans, bra
// and ket pair of each quartet alternating for quartet plans; hoff: where each
// entry's H starts in h), then the persistent kernel that reads it.
hipError_t plan_solid_set_attrs();
hipError_t plan_solid_occupancy(bool pairs, int lds_bytes, int* per_cu);
hipError_t plan_solid_launch(bool pairs, dim3 grid, int lds_bytes, hipStream_t s, const Tables& t, const PlanArgs& a,
                             int64_t nbra, const int64_t* hoff, const double* h);
hipError_t plan_coulomb_set_attrs();
hipError_t plan_coulomb_occupancy(int lds_bytes, int* per_cu);
hipError_t plan_coulomb_launch(dim3 grid, int lds_bytes, hipStream_t s, const Tables& t, const PlanArgs& a,
                               int nbra, int kmax, const int32_t* pl, const int32_t* pn, const double* ket_dens,
                               const int64_t* doff, const int64_t* dkoff, const int64_t* joff, double* dket,
                               double* jpart, double* out);
// nbra < 0: the alternating (quartet) form, all entries read from x.centers, ...;
// lds: dynamic LDS bytes, solid_h_lds of the largest entry
hipError_t solid_hpairs_launch(int64_t nbra, int64_t nentries, int kmax, int lds, hipStream_t s, const int32_t* pl,
                               const int32_t* pn, const Shells& x, const int64_t* hoff, const double* stab,
                               double* h);

#define ERI4_PLAN_KERNEL_ENTRIES(sfx)                                                                   \
  hipError_t plan_set_attrs_##sfx();                                                                   \
  hipError_t plan_occupancy_##sfx(int lds_bytes, int* per_cu);                                         \
  hipError_t plan_launch_##sfx(dim3 grid, int lds_bytes, hipStream_t s, const Tables& t, const PlanArgs& a);
ERI4_PLAN_KERNEL_ENTRIES(f64)
ERI4_PLAN_KERNEL_ENTRIES(f32)
ERI4_PLAN_KERNEL_ENTRIES(f64p)
ERI4_PLAN_KERNEL_ENTRIES(f32p)
#undef ERI4_PLAN_KERNEL_ENTRIES

}  // namespace eri4
