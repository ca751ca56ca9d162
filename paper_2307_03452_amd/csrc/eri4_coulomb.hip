// eri4_coulomb.hip -- Coulomb contraction without forming (ab|cd) (FP64,
// Cartesian): J_ab = sum_cd (ab|cd) D_cd per quartet.  The ket density is first
// taken to Hermite space per ket primitive pair, dket^kl_q = sum_cd E_cd^q D_cd
// (sign of eq. (pq) included), then the tile code contracts the first
// transform's [ab|q] with it instead of running the second transform.
#include "eri4_device.h"

namespace eri4 {
namespace {

// dket of ket primitives (z1, w1) of shell lc and (z2, w2) of shell ld at
// centres c[0..5], for the density block D[Nc][Nd], in the column order of the
// first transform (16 * nqb doubles at out, zero past the nq Hermite
// functions).  Called by all threads of a workgroup.
__device__ __forceinline__ void build_dket(int lc, int ld, const double* __restrict__ c, double z1, double z2,
                                           double w1, double w2, const double* __restrict__ D,
                                           double* __restrict__ out, int tid) {
  __shared__ double tabs[kMaxEtab];
  __shared__ double pair[16];
  __shared__ int2 qt[kMaxHerm + 16];
  __shared__ int3 cdx[ncart(kTableLMax) * ncart(kTableLMax)];  // E-table rows of each (c, d)
  const int lane = tid & 63;
  const int Lk = lc + ld, nq = nherm(Lk), nqb = (nq + 15) / 16;
  const int tkrow = odd_row(Lk + 2), tkaxis = ((lc + 1) * (ld + 1) + 1) * tkrow;
  const int nd = ncart(ld), ncd = ncart(lc) * nd;
  if (tid == 0) make_pair(pair, z1, z2, w1, w2, c, c + 3);
  build_htab(qt, Lk, nq, 16 * nqb, 0, 0, false, tid);
  for (int cd = tid; cd < ncd; cd += kThreads) {
    const int ic = cd / nd, id = cd - (cd / nd) * nd;
    int cx, cy, cz, dx, dy, dz;
    cart_of(lc, ic, cx, cy, cz);
    cart_of(ld, id, dx, dy, dz);
    cdx[cd] = make_int3((cx * (ld + 1) + dx) * tkrow, tkaxis + (cy * (ld + 1) + dy) * tkrow,
                        2 * tkaxis + (cz * (ld + 1) + dz) * tkrow);
  }
  __syncthreads();
  if (tid < 64) build_etab(tabs, lc, ld, tkrow, tkaxis, 0.5 / pair[0], pair + 5, pair + 8, true, lane);
  __syncthreads();
  for (int kq = tid; kq < 16 * nqb; kq += kThreads) {
    double v = 0.0;
    if (kq < nq) {
      const int hx = qt[kq].x;
      const int t = hx & 0xff, u = (hx >> 8) & 0xff, w = (hx >> 16) & 0xff;
#pragma unroll 4
      for (int cd = 0; cd < ncd; ++cd) {
        const int3 o = cdx[cd];
        v += D[cd] * tabs[o.x + t] * tabs[o.y + u] * tabs[o.z + w];
      }
    }
    out[kq] = v;
  }
}

// Batch form: one workgroup per (quartet q0 + blockIdx.x, ket pair slot
// blockIdx.y = k * kmax + l), dket at dket + (blockIdx.x * kmax^2 + slot) * ds.
__global__ __launch_bounds__(kThreads, 1) void coulomb_dket_kernel(
    const ClassParams cp, const double* __restrict__ centers, const double* __restrict__ exps,
    const double* __restrict__ coefs, const int32_t* __restrict__ nprim, const double* __restrict__ dens,
    double* __restrict__ dket, int64_t q0, int64_t ds) {
  const int tid = threadIdx.x;
  const int64_t iq = blockIdx.x;
  const int64_t q = q0 + iq;
  const int slot = blockIdx.y, kmax = cp.kmax;
  const int k = slot / kmax, l = slot - (slot / kmax) * kmax;
  const int Kc = nprim[q * 4 + 2], Kd = nprim[q * 4 + 3];
  if (Kc < 1 || Kc > kmax || Kd < 1 || Kd > kmax || k >= Kc || l >= Kd) return;
  const double* e = exps + (q * 4 + 2) * kmax;
  const double* w = coefs + (q * 4 + 2) * kmax;
  build_dket(cp.lc, cp.ld, centers + q * 12 + 6, e[k], e[kmax + l], w[k], w[kmax + l], dens + q * cp.ncd,
             dket + (iq * kmax * kmax + slot) * ds, tid);
}

// List form: one workgroup per (ket list entry blockIdx.x, slot blockIdx.y);
// pl / pn hold (lc, ld) and the contraction lengths per entry, its density
// block starts at dens + doff[entry], its dket slots at dket + dkoff[entry]
// (16 * nqb doubles each).
__global__ __launch_bounds__(kThreads, 1) void coulomb_dket_pairs_kernel(
    int kmax, const int32_t* __restrict__ pl, const int32_t* __restrict__ pn, const double* __restrict__ kcenters,
    const double* __restrict__ kexps, const double* __restrict__ kcoefs, const double* __restrict__ dens,
    const int64_t* __restrict__ doff, const int64_t* __restrict__ dkoff, double* __restrict__ dket) {
  const int tid = threadIdx.x;
  const int64_t jk = blockIdx.x;
  const int slot = blockIdx.y;
  const int k = slot / kmax, l = slot - (slot / kmax) * kmax;
  const int Kc = pn[2 * jk], Kd = pn[2 * jk + 1];
  if (Kc < 1 || Kc > kmax || Kd < 1 || Kd > kmax || k >= Kc || l >= Kd) return;
  const int lc = pl[2 * jk], ld = pl[2 * jk + 1];
  const int ds = 16 * ((nherm(lc + ld) + 15) / 16);
  const double* e = kexps + jk * 2 * kmax;
  const double* w = kcoefs + jk * 2 * kmax;
  build_dket(lc, ld, kcenters + jk * 6, e[k], e[kmax + l], w[k], w[kmax + l], dens + doff[jk],
             dket + dkoff[jk] + (int64_t)slot * ds, tid);
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

// Persistent kernel of a Coulomb pair-list plan: the work loop of
// eri4_plan_kernel (shells from the lists), each tile contracting [ab|q] with
// the dket of the quartet's ket entry (dket + dkoff[q % nket]) and writing its
// J rows to jpart + qoff[q].
__global__ __launch_bounds__(kThreads, 1) void eri4_plan_coulomb_kernel(
    const ClassParams* __restrict__ classes, const int2* __restrict__ items, int nitems,
    const int64_t* __restrict__ qoff, const int32_t* __restrict__ nprim, int* __restrict__ counter,
    const double* __restrict__ boys_tab, const uint2* __restrict__ rtab, const double* __restrict__ centers,
    const double* __restrict__ exps, const double* __restrict__ coefs, double* __restrict__ jpart,
    const double* __restrict__ kcenters, const double* __restrict__ kexps, const double* __restrict__ kcoefs,
    int64_t nket, const int64_t* __restrict__ dkoff, const double* __restrict__ dket) {
  extern __shared__ __align__(16) unsigned char lds[];
  __shared__ double jt[kCoulLds];
  __shared__ int next_item;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  for (;;) {
    if (tid == 0) next_item = atomicAdd(counter, 1);
    __syncthreads();
    const int it = __builtin_amdgcn_readfirstlane(next_item);
    __syncthreads();
    if (it >= nitems) break;
    const int2 w = items[it];
    const int q = __builtin_amdgcn_readfirstlane(w.x);
    const int rc = __builtin_amdgcn_readfirstlane(w.y);
    const ClassParams cp = classes[rc >> 16];
    const int rt = rc & 0xffff;
    const uint2* rt_L = rtab + cp.rtab_off;
    double* oq = jpart + qoff[q];
    const int64_t ik = q - (q / nket) * nket;
    const double* hk = dket + dkoff[ik];
    const int64_t hks = 16 * (int64_t)cp.nqb;
#define T(RB, LAY)                                                                                                   \
  process_tile<RB, LAY, false, true, false, true>(cp, lds, boys_tab, rt_L, centers, exps, coefs, nprim, oq, q, rt, tid, \
                                                  wave, lane, kcenters, kexps, kcoefs, nket, nullptr, hk, 0, hks, jt)
    const int lay = cp.lay;
    if (lay == kLaySlab) {
      if (cp.rb == 2) T(2, kLaySlab); else T(1, kLaySlab);
    } else if (lay == kLayBox2) {
      if (cp.rb == 4) T(4, kLayBox2); else if (cp.rb == 2) T(2, kLayBox2); else T(1, kLayBox2);
    } else {
      if (cp.rb == 4) T(4, kLayBox); else if (cp.rb == 2) T(2, kLayBox); else T(1, kLayBox);
    }
#undef T
  }
}

// J of bra entry blockIdx.x: the sum over ket entries j = 0..nket-1, in that
// order, of the J rows of quartet (i, j) (jpart + qoff[i * nket + j]), into
// out + joff[i]; nab rows from the entry's (la, lb) in pl.
__global__ void coulomb_reduce_kernel(int64_t nket, const int32_t* __restrict__ pl, const int64_t* __restrict__ qoff,
                                      const double* __restrict__ jpart, const int64_t* __restrict__ joff,
                                      double* __restrict__ out) {
  const int64_t i = blockIdx.x;
  const int nab = ncart(pl[2 * i]) * ncart(pl[2 * i + 1]);
  for (int ab = threadIdx.x; ab < nab; ab += blockDim.x) {
    double a = 0.0;
    for (int64_t j = 0; j < nket; ++j) a += jpart[qoff[i * nket + j] + ab];
    out[joff[i] + ab] = a;
  }
}

}  // namespace

hipError_t plan_coulomb_set_attrs() {
  return hipFuncSetAttribute((const void*)eri4_plan_coulomb_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                             kMaxLdsBytes - kCoulLds * 8 - 512);
}

hipError_t plan_coulomb_occupancy(int lds_bytes, int* per_cu) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, (const void*)eri4_plan_coulomb_kernel, kThreads,
                                                      lds_bytes);
}

// The three steps of a Coulomb pair-list plan (after the caller reset the work
// counter): dket of every ket entry, the persistent kernel, the reduction.
hipError_t plan_coulomb_launch(dim3 grid, int lds_bytes, hipStream_t s, const Tables& t, const PlanArgs& a,
                               int nbra, int kmax, const int32_t* pl, const int32_t* pn, const double* ket_dens,
                               const int64_t* doff, const int64_t* dkoff, const int64_t* joff, double* dket,
                               double* jpart, double* out) {
  const Shells& x = a.shells;
  hipLaunchKernelGGL(coulomb_dket_pairs_kernel, dim3((unsigned)x.nket, (unsigned)(kmax * kmax)), dim3(kThreads), 0, s,
                     kmax, pl + 2 * nbra, pn + 2 * nbra, x.kcenters, x.kexps, x.kcoefs, ket_dens, doff, dkoff, dket);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(eri4_plan_coulomb_kernel, grid, dim3(kThreads), lds_bytes, s, a.classes, a.items, a.nitems,
                     a.qoff, a.nprim, a.counter, t.boys, t.rtab, x.centers, x.exps, x.coefs, jpart, x.kcenters,
                     x.kexps, x.kcoefs, x.nket, dkoff, dket);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(coulomb_reduce_kernel, dim3((unsigned)nbra), dim3(256), 0, s, x.nket, pl, a.qoff, jpart, joff,
                     out);
  return hipGetLastError();
}

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
