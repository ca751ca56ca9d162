// eri4_coulomb.hip -- Coulomb contraction without forming (ab|cd) (FP64,
// Cartesian): J_ab = sum_cd (ab|cd) D_cd per quartet.  The ket density is first
// taken to Hermite space per ket primitive pair, dket^kl_q = sum_cd E_cd^q D_cd
// (sign of eq. (pq) included), then the tile code contracts the first
// transform's [ab|q] with it instead of running the second transform.
#include "eri4_device.h"

namespace eri4 {
namespace {

// One workgroup per (quartet q0 + blockIdx.x, ket pair slot blockIdx.y = k *
// kmax + l): dket of that pair in the column order of the first transform
// (qtab), 16 * cp.nqb doubles at dket + (blockIdx.x * kmax^2 + slot) * ds,
// zero past the cp.nq Hermite functions.
__global__ __launch_bounds__(kThreads, 1) void coulomb_dket_kernel(
    const ClassParams cp, const double* __restrict__ centers, const double* __restrict__ exps,
    const double* __restrict__ coefs, const int32_t* __restrict__ nprim, const double* __restrict__ dens,
    double* __restrict__ dket, int64_t q0, int64_t ds) {
  __shared__ double tabs[kMaxEtab];
  __shared__ double pair[16];
  __shared__ int2 qt[kMaxHerm + 16];
  __shared__ int3 cdx[ncart(kTableLMax) * ncart(kTableLMax)];  // E-table rows of each (c, d)
  const int tid = threadIdx.x, lane = tid & 63;
  const int64_t iq = blockIdx.x;
  const int64_t q = q0 + iq;
  const int slot = blockIdx.y, kmax = cp.kmax;
  const int k = slot / kmax, l = slot - (slot / kmax) * kmax;
  const int Kc = nprim[q * 4 + 2], Kd = nprim[q * 4 + 3];
  if (Kc < 1 || Kc > kmax || Kd < 1 || Kd > kmax || k >= Kc || l >= Kd) return;
  const int lc = cp.lc, ld = cp.ld;
  if (tid == 0) {
    const double* c = centers + q * 12 + 6;
    const double* e = exps + (q * 4 + 2) * kmax;
    const double* w = coefs + (q * 4 + 2) * kmax;
    make_pair(pair, e[k], e[kmax + l], w[k], w[kmax + l], c, c + 3);
  }
  build_htab(qt, cp.Lk, cp.nq, 16 * cp.nqb, 0, 0, false, tid);
  for (int cd = tid; cd < cp.ncd; cd += kThreads) {
    const int ic = cd / cp.nd, id = cd - (cd / cp.nd) * cp.nd;
    int cx, cy, cz, dx, dy, dz;
    cart_of(lc, ic, cx, cy, cz);
    cart_of(ld, id, dx, dy, dz);
    cdx[cd] = make_int3((cx * (ld + 1) + dx) * cp.tkrow, cp.tkaxis + (cy * (ld + 1) + dy) * cp.tkrow,
                        2 * cp.tkaxis + (cz * (ld + 1) + dz) * cp.tkrow);
  }
  __syncthreads();
  if (tid < 64) build_etab(tabs, lc, ld, cp.tkrow, cp.tkaxis, 0.5 / pair[0], pair + 5, pair + 8, true, lane);
  __syncthreads();
  const double* D = dens + q * cp.ncd;
  double* out = dket + (iq * kmax * kmax + slot) * ds;
  for (int kq = tid; kq < 16 * cp.nqb; kq += kThreads) {
    double v = 0.0;
    if (kq < cp.nq) {
      const int hx = qt[kq].x;
      const int t = hx & 0xff, u = (hx >> 8) & 0xff, w = (hx >> 16) & 0xff;
#pragma unroll 4
      for (int cd = 0; cd < cp.ncd; ++cd) {
        const int3 o = cdx[cd];
        v += D[cd] * tabs[o.x + t] * tabs[o.y + u] * tabs[o.z + w];
      }
    }
    out[kq] = v;
  }
}

// One workgroup = one quartet x one tile of RB*16 bra rows (eri4_fused_kernel
// with the Coulomb contraction); out: J [nq][Na][Nb].
template <int RB, int LAY>
__global__ __launch_bounds__(kThreads, 1) void eri4_coulomb_kernel(
    const ClassParams cp, const double* __restrict__ boys_tab, const uint2* __restrict__ rtab,
    const double* __restrict__ centers, const double* __restrict__ exps, const double* __restrict__ coefs,
    const int32_t* __restrict__ nprim, double* __restrict__ out, int64_t q0, const double* __restrict__ dket,
    int64_t ds) {
  extern __shared__ __align__(16) unsigned char lds[];
  __shared__ double jt[kCoulLds];  // J rows of the tile and the waves' partial rows
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t i = blockIdx.x / cp.nrt;
  const int64_t q = q0 + i;
  const int rt = blockIdx.x % cp.nrt;
  const int64_t kk2 = (int64_t)cp.kmax * cp.kmax;
  process_tile<RB, LAY, false, false, false, true>(cp, lds, boys_tab, rtab + cp.rtab_off, centers, exps, coefs, nprim,
                                                   out + q * (int64_t)cp.nab, q, rt, tid, wave, lane, nullptr,
                                                   nullptr, nullptr, 0, nullptr, dket + i * kk2 * ds, 0, ds, jt);
}

template <int RB, int LAY>
hipError_t coulomb_launch_t(const ClassParams& p, dim3 grid, hipStream_t s, const Tables& t, const double* centers,
                            const double* exps, const double* coefs, const int32_t* nprim, double* out, int64_t q0,
                            const double* dket, int64_t ds) {
  hipLaunchKernelGGL((eri4_coulomb_kernel<RB, LAY>), grid, dim3(kThreads), p.lds_bytes, s, p, t.boys, t.rtab, centers,
                     exps, coefs, nprim, out, q0, dket, ds);
  return hipGetLastError();
}

}  // namespace

hipError_t coulomb_set_attrs() {
  const void* k[8] = {(const void*)eri4_coulomb_kernel<1, kLayBox>,  (const void*)eri4_coulomb_kernel<2, kLayBox>,
                      (const void*)eri4_coulomb_kernel<4, kLayBox>,  (const void*)eri4_coulomb_kernel<1, kLaySlab>,
                      (const void*)eri4_coulomb_kernel<2, kLaySlab>, (const void*)eri4_coulomb_kernel<1, kLayBox2>,
                      (const void*)eri4_coulomb_kernel<2, kLayBox2>, (const void*)eri4_coulomb_kernel<4, kLayBox2>};
  for (const void* f : k) {
    const hipError_t e =
        hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLdsBytes - kCoulLds * 8 - 512);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t coulomb_dket_launch(const ClassParams& p, int64_t nq, hipStream_t s, const double* centers,
                               const double* exps, const double* coefs, const int32_t* nprim, const double* dens,
                               double* dket, int64_t q0, int64_t ds) {
  const dim3 grid((unsigned)nq, (unsigned)(p.kmax * p.kmax));
  hipLaunchKernelGGL(coulomb_dket_kernel, grid, dim3(kThreads), 0, s, p, centers, exps, coefs, nprim, dens, dket, q0,
                     ds);
  return hipGetLastError();
}

hipError_t coulomb_launch(const ClassParams& p, dim3 grid, hipStream_t s, const Tables& t, const double* centers,
                          const double* exps, const double* coefs, const int32_t* nprim, double* out, int64_t q0,
                          const double* dket, int64_t ds) {
  const bool two = p.rb == 2;
#define L(RB, LAY) coulomb_launch_t<RB, LAY>(p, grid, s, t, centers, exps, coefs, nprim, out, q0, dket, ds)
  switch (p.lay) {
    case kLaySlab:
      return two ? L(2, kLaySlab) : L(1, kLaySlab);
    case kLayBox2:
      if (p.rb == 4) return L(4, kLayBox2);
      return two ? L(2, kLayBox2) : L(1, kLayBox2);
    default:
      if (p.rb == 4) return L(4, kLayBox);
      return two ? L(2, kLayBox) : L(1, kLayBox);
  }
#undef L
}

}  // namespace eri4
