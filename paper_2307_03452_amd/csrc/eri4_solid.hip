// eri4_solid.hip -- solid-harmonic output (FP64): the kernel that builds the H
// matrices of every primitive pair, and the single-class integral kernels that
// read them, one instance per tile height and R layout.
#include <algorithm>

#include "eri4_device.h"

namespace eri4 {
namespace {

// H = (C_1 x C_2) E for one primitive pair (Sec. 2, the contraction of E with
// the Cartesian-to-solid coefficients), written in the operand order of the
// transform that reads it (see gemm1_h): one workgroup per (quartet q0 +
// blockIdx.x, side = blockIdx.y & 1, pair slot).  Side 0 is the bra (shells a,
// b; cp.nrt * cp.rb units of 16 rows, cp.np4 k), side 1 the ket (shells c, d,
// sign (-1)^|q| of eq. (pq); cp.ncdb units of 16 columns, cp.nq4 k).  Elements
// past the solid functions or the Hermite functions are 0.  Pairs beyond the
// quartet's contraction lengths are skipped (the integral kernel does not read
// them).
//
// Both sums run on the FP64 matrix cores, per chunk of 16 Hermite indices k:
//   P[m1][b][k]  = sum_a C_1[m1][a] E_ab^k   (16 x 4 steps over a, one 16-wide
//                                             block of k per shell-2 component b)
//   H[m1 m2][k] = sum_b C_2[m2][b] P[m1][b][k]
// with the coefficients as the A operands (dense, from the sparse table, in
// registers) and E_ab^k formed once per (a, b, k) from the three 1-d tables as
// the B operand of the first product; P goes through LDS.
constexpr int kHNc = ncart(kTableLMax);  // Cartesian components per shell, at most
constexpr int kHSteps = (kHNc + 3) / 4;  // MFMA k steps over them
constexpr int kSolidHLdsMax = solid_h_lds(kTableLMax, kTableLMax, kMaxHerm);

// H of primitives (z1, w1) of shell l1 and (z2, w2) of shell l2 at centres
// c[0..2], c[3..5], into H (this pair slot's nunits units of 16 rows by nk4 k).
// Called by all threads of a workgroup; dyn is LDS for solid_h_lds(l1, l2,
// nk4) bytes: P, then the 1-d tables, then the Hermite index table.
__device__ __forceinline__ void build_h(int l1, int l2, bool ket, const double* __restrict__ c, double z1, double z2,
                                        double w1, double w2, const double* __restrict__ stab, double* __restrict__ H,
                                        int nunits, int nk4, unsigned char* dyn, int tid) {
  __shared__ double pair[16];
  __shared__ double cd[2][16][kHNc];  // dense C_1, C_2 (rows m, columns Cartesian index), zero-padded
  __shared__ int cart[2][kHNc];       // table-row offsets (x, y, z packed) of each Cartesian component
  const int lane = tid & 63, g = lane >> 4, n = lane & 15;
  const int wave = tid >> 6;
  const int Lh = l1 + l2;
  const int nh = nherm(Lh);
  const int trow = odd_row(Lh + 2), taxis = ((l1 + 1) * (l2 + 1) + 1) * trow;
  const int s1 = 2 * l1 + 1, s2 = 2 * l2 + 1, n1c = ncart(l1), n2c = ncart(l2);
  double* P = (double*)dyn;        // [s1][n2c][16]
  double* tabs = P + s1 * n2c * 16;  // 3 * taxis
  int2* htab = (int2*)(tabs + 3 * taxis);
  if (tid == 0) make_pair(pair, z1, z2, w1, w2, c, c + 3);
  build_htab(htab, Lh, nh, nk4, 0, 0, false, tid);
  for (int e = tid; e < 2 * 16 * kHNc; e += kThreads) (&cd[0][0][0])[e] = 0.0;
  for (int e = tid; e < 2 * kHNc; e += kThreads) {
    const int sh = e / kHNc, k = e - sh * kHNc, l = sh ? l2 : l1;
    int x = 0, y = 0, z = 0;
    if (k < ncart(l)) cart_of(l, k, x, y, z);
    cart[sh][k] = x | (y << 8) | (z << 16);
  }
  __syncthreads();
  // the two shells' solid functions, scattered into dense rows
  for (int e = tid; e < 2 * kSolidRows * kSolidTerms; e += kThreads) {
    const int sh = e / (kSolidRows * kSolidTerms), rem = e - sh * (kSolidRows * kSolidTerms);
    const int m = rem / kSolidTerms, jt = rem - m * kSolidTerms;
    const int l = sh ? l2 : l1;
    if (m < 2 * l + 1) {
      const double* ent = stab + (l * kSolidRows + m) * kSolidEntry;
      if (jt < (int)ent[0]) cd[sh][m][(int)ent[1 + 2 * jt]] = ent[2 + 2 * jt];
    }
  }
  if (tid < 64) build_etab(tabs, l1, l2, trow, taxis, 0.5 / pair[0], pair + 5, pair + 8, ket, lane);
  __syncthreads();
  const int per = nk4 * 16;  // doubles per unit of 16 rows
  // element (row r, k) of H in operand order
  auto at = [&](int r, int k) { return (r >> 4) * per + (k >> 2) * 64 + (k & 3) * 16 + (r & 15); };
  const int nrow = s1 * s2;
  for (int e = tid; e < (nunits * 16 - nrow) * nk4; e += kThreads) {
    const int r = nrow + e / nk4, k = e - (e / nk4) * nk4;
    H[at(r, k)] = 0.0;
  }
  // A operands: lane (n, g) holds C[n][4 s + g] for the k steps s
  const int ks1 = (n1c + 3) >> 2, ks2 = (n2c + 3) >> 2;
  double a1[kHSteps], a2[kHSteps];
  int ra[kHSteps];  // 1-d table rows of shell-1 component 4 s + g (the last one past n1c)
#pragma unroll
  for (int st = 0; st < kHSteps; ++st) {
    a1[st] = cd[0][n][4 * st + g];
    a2[st] = cd[1][n][4 * st + g];
    ra[st] = cart[0][min(4 * st + g, n1c - 1)];
  }
  for (int c0 = 0; c0 < nk4; c0 += 16) {
    // this lane's Hermite index k = c0 + n (past nk4: the zero entry Lh + 1)
    const int kk = c0 + n;
    const int hx = kk < nk4 ? htab[kk].x : Lh + 1;
    const int t = hx & 0xff, u = (hx >> 8) & 0xff, w = (hx >> 16) & 0xff;
    // P[m1][b][k] = sum_a C_1[m1][a] E_ab^k, one 16 x 16 block per b
    for (int b = wave; b < n2c; b += kWaves) {
      const int cb = cart[1][b];
      const int bx = cb & 0xff, by = (cb >> 8) & 0xff, bz = (cb >> 16) & 0xff;
      d4 acc = acc_zero<false>();
#pragma unroll
      for (int st = 0; st < kHSteps; ++st) {
        if (st < ks1) {
          const int axp = ra[st];
          const int ax = axp & 0xff, ay = (axp >> 8) & 0xff, az = (axp >> 16) & 0xff;
          const double e = tabs[(ax * (l2 + 1) + bx) * trow + t] * tabs[taxis + (ay * (l2 + 1) + by) * trow + u] *
                           tabs[2 * taxis + (az * (l2 + 1) + bz) * trow + w];
          acc = mfma16<false>(a1[st], e, acc);
        }
      }
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) {
        const int m1 = acc_row<false>(jj, g);
        if (m1 < s1) P[(m1 * n2c + b) * 16 + n] = acc[jj];
      }
    }
    __syncthreads();
    // H[m1 s2 + m2][k] = sum_b C_2[m2][b] P[m1][b][k]
    for (int m1 = wave; m1 < s1; m1 += kWaves) {
      d4 acc = acc_zero<false>();
#pragma unroll
      for (int st = 0; st < kHSteps; ++st) {
        if (st < ks2) acc = mfma16<false>(a2[st], P[(m1 * n2c + min(4 * st + g, n2c - 1)) * 16 + n], acc);
      }
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) {
        const int m2 = acc_row<false>(jj, g);
        if (m2 < s2 && kk < nk4) H[at(m1 * s2 + m2, kk)] = acc[jj];
      }
    }
    __syncthreads();
  }
}

// Batch form: one workgroup per (quartet q0 + blockIdx.x, side = blockIdx.y & 1,
// primitive pair (i, j) = divmod(blockIdx.y >> 1, kmax)); side 0 is the bra
// (shells a, b; cp.nrt * cp.rb units, cp.np4 k), side 1 the ket (shells c, d;
// cp.ncdb units, cp.nq4 k).  Quartet q0 + x reserves kmax^2 slots per side and
// fills the first K1 * K2: pair (i, j) at slot i * K2 + j, i.e. at hbra +
// (x * kmax^2 + i * K2 + j) * hbs (bra) or the same in hket with hks (ket).
__global__ __launch_bounds__(kThreads, 1) void solid_h_kernel(
    const ClassParams cp, const double* __restrict__ centers, const double* __restrict__ exps,
    const double* __restrict__ coefs, const int32_t* __restrict__ nprim, const double* __restrict__ stab,
    double* __restrict__ hbra, double* __restrict__ hket, int64_t q0, int64_t hbs, int64_t hks) {
  extern __shared__ __align__(16) unsigned char dyn[];
  const int tid = threadIdx.x;
  const int64_t iq = blockIdx.x;
  const int64_t q = q0 + iq;
  const int side = blockIdx.y & 1, slot = blockIdx.y >> 1;
  const int kmax = cp.kmax;
  const int i = slot / kmax, j = slot - (slot / kmax) * kmax;
  const int K1 = nprim[q * 4 + 2 * side], K2 = nprim[q * 4 + 2 * side + 1];
  if (K1 < 1 || K1 > kmax || K2 < 1 || K2 > kmax || i >= K1 || j >= K2) return;
  const double* e = exps + (q * 4 + 2 * side) * kmax;
  const double* w = coefs + (q * 4 + 2 * side) * kmax;
  const int64_t at = iq * kmax * kmax + i * K2 + j;
  double* H = side ? hket + at * hks : hbra + at * hbs;
  build_h(side ? cp.lc : cp.la, side ? cp.ld : cp.lb, side == 1, centers + q * 12 + 6 * side, e[i], e[kmax + j], w[i],
          w[kmax + j], stab, H, side ? cp.ncdb : cp.nrt * cp.rb, side ? cp.nq4 : cp.np4, dyn, tid);
}

// List form: one workgroup per (list entry e0 + blockIdx.x, primitive pair (i, j) =
// divmod(blockIdx.y, kmax)).  With nbra >= 0, entries 0..nbra-1 are the bra
// list (shells from bcenters, ...) and the rest the ket list (kcenters, ...);
// with nbra < 0 the entries alternate, 2q the bra pair and 2q + 1 the ket pair
// of quartet q, all read from bcenters, ... at the entry's own index (the
// quartet layout seen as a list of pairs).  An entry with K1 * K2 primitive
// pairs holds K1 * K2 slots from h + hoff[entry], pair (i, j) at slot i * K2 +
// j, each solid_pair_units(...) * 16 * nk4 doubles; bra rows are padded to 64
// so that every tile height can read them.
__global__ __launch_bounds__(kThreads, 1) void solid_hpairs_kernel(
    int64_t e0, int64_t nbra, int kmax, const int32_t* __restrict__ pl, const int32_t* __restrict__ pn,
    const double* __restrict__ bcenters, const double* __restrict__ bexps, const double* __restrict__ bcoefs,
    const double* __restrict__ kcenters, const double* __restrict__ kexps, const double* __restrict__ kcoefs,
    const int64_t* __restrict__ hoff, const double* __restrict__ stab, double* __restrict__ h) {
  extern __shared__ __align__(16) unsigned char dyn[];
  const int tid = threadIdx.x;
  const int64_t p = e0 + blockIdx.x;
  const int slot = blockIdx.y;
  const int i = slot / kmax, j = slot - (slot / kmax) * kmax;
  const int K1 = pn[2 * p], K2 = pn[2 * p + 1];
  if (K1 < 1 || K1 > kmax || K2 < 1 || K2 > kmax || i >= K1 || j >= K2) return;
  const bool alt = nbra < 0;
  const bool ket = alt ? (p & 1) != 0 : p >= nbra;
  const bool klist = ket && !alt;
  const int64_t ip = klist ? p - nbra : p;
  const int l1 = pl[2 * p], l2 = pl[2 * p + 1];
  const double* e = (klist ? kexps : bexps) + ip * 2 * kmax;
  const double* w = (klist ? kcoefs : bcoefs) + ip * 2 * kmax;
  const int nk4 = (nherm(l1 + l2) + 3) & ~3;
  const int nunits = solid_pair_units(l1, l2, ket);
  build_h(l1, l2, ket, (klist ? kcenters : bcenters) + ip * 6, e[i], e[kmax + j], w[i], w[kmax + j], stab,
          h + hoff[p] + (int64_t)(i * K2 + j) * nunits * 16 * nk4, nunits, nk4, dyn, tid);
}

// Persistent kernel of a solid-harmonic plan: the work loop of
// eri4_plan_kernel, both transforms reading the H matrices built by
// solid_hpairs_kernel.  PAIRS: shells from the bra and ket lists, H of the
// quartet's bra entry at h + hoff[q / nket] and of its ket entry at h +
// hoff[nbra + q % nket]; otherwise shells from the quartet arrays and H at h +
// hoff[2q] (bra) and h + hoff[2q + 1] (ket).
template <bool PAIRS>
__global__ __launch_bounds__(kThreads, 1) void eri4_plan_solid_kernel(
    const ClassParams* __restrict__ classes, const int2* __restrict__ items, int nitems,
    const int64_t* __restrict__ qoff, const int32_t* __restrict__ nprim, int* __restrict__ counter,
    const double* __restrict__ boys_tab, const uint2* __restrict__ rtab, const double* __restrict__ centers,
    const double* __restrict__ exps, const double* __restrict__ coefs, double* __restrict__ out,
    const double* __restrict__ kcenters, const double* __restrict__ kexps, const double* __restrict__ kcoefs,
    int64_t nket, int64_t nbra, const int64_t* __restrict__ hoff, const double* __restrict__ h) {
  extern __shared__ __align__(16) unsigned char lds[];
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
    double* oq = out + qoff[q];
    const double* hb;
    const double* hk;
    if constexpr (PAIRS) {
      const int64_t ib = q / nket, ik = q - ib * nket;
      hb = h + hoff[ib];
      hk = h + hoff[nbra + ik];
    } else {
      hb = h + hoff[2 * (int64_t)q];
      hk = h + hoff[2 * (int64_t)q + 1];
    }
    const int64_t hbs = (int64_t)solid_pair_units(cp.la, cp.lb, false) * 16 * cp.np4;
    const int64_t hks = (int64_t)cp.ncdb * 16 * cp.nq4;
#define T(RB, LAY)                                                                                                   \
  process_tile<RB, LAY, false, PAIRS, true>(cp, lds, boys_tab, rt_L, centers, exps, coefs, nprim, oq, q, rt, tid, wave, \
                                           lane, kcenters, kexps, kcoefs, nket, hb, hk, hbs, hks)
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

}  // namespace

hipError_t plan_solid_set_attrs() {
  hipError_t e = hipFuncSetAttribute((const void*)eri4_plan_solid_kernel<true>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLdsBytes - 64);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)eri4_plan_solid_kernel<false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             kMaxLdsBytes - 64);
}

hipError_t plan_solid_occupancy(bool pairs, int lds_bytes, int* per_cu) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(
      per_cu, pairs ? (const void*)eri4_plan_solid_kernel<true> : (const void*)eri4_plan_solid_kernel<false>, kThreads,
      lds_bytes);
}

hipError_t plan_solid_launch(bool pairs, dim3 grid, int lds_bytes, hipStream_t s, const Tables& t, const PlanArgs& a,
                             int64_t nbra, const int64_t* hoff, const double* h) {
  const Shells& x = a.shells;
  if (pairs)
    hipLaunchKernelGGL(eri4_plan_solid_kernel<true>, grid, dim3(kThreads), lds_bytes, s, a.classes, a.items, a.nitems,
                       a.qoff, a.nprim, a.counter, t.boys, t.rtab, x.centers, x.exps, x.coefs, a.out, x.kcenters,
                       x.kexps, x.kcoefs, x.nket, nbra, hoff, h);
  else
    hipLaunchKernelGGL(eri4_plan_solid_kernel<false>, grid, dim3(kThreads), lds_bytes, s, a.classes, a.items,
                       a.nitems, a.qoff, a.nprim, a.counter, t.boys, t.rtab, x.centers, x.exps, x.coefs, a.out,
                       nullptr, nullptr, nullptr, (int64_t)0, (int64_t)0, hoff, h);
  return hipGetLastError();
}

hipError_t solid_hpairs_launch(int64_t nbra, int64_t nentries, int kmax, int lds, hipStream_t s, const int32_t* pl,
                               const int32_t* pn, const Shells& x, const int64_t* hoff, const double* stab,
                               double* h) {
  // entries per launch: the grid's x extent in work-items stays below 2^32
  constexpr int64_t kChunk = (int64_t)1 << 22;
  for (int64_t e0 = 0; e0 < nentries; e0 += kChunk) {
    const dim3 grid((unsigned)std::min(kChunk, nentries - e0), (unsigned)(kmax * kmax));
    hipLaunchKernelGGL(solid_hpairs_kernel, grid, dim3(kThreads), lds, s, e0, nbra, kmax, pl, pn, x.centers,
                       x.exps, x.coefs, x.kcenters, x.kexps, x.kcoefs, hoff, stab, h);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t solid_set_attrs() {
  const void* k[8] = {(const void*)eri4_solid_kernel<1, kLayBox>,  (const void*)eri4_solid_kernel<2, kLayBox>,
                      (const void*)eri4_solid_kernel<4, kLayBox>,  (const void*)eri4_solid_kernel<1, kLaySlab>,
                      (const void*)eri4_solid_kernel<2, kLaySlab>, (const void*)eri4_solid_kernel<1, kLayBox2>,
                      (const void*)eri4_solid_kernel<2, kLayBox2>, (const void*)eri4_solid_kernel<4, kLayBox2>};
  for (const void* f : k) {
    const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLdsBytes);
    if (e != hipSuccess) return e;
  }
  const hipError_t e = hipFuncSetAttribute((const void*)solid_h_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           kSolidHLdsMax);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)solid_hpairs_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                             kSolidHLdsMax);
}

hipError_t solid_h_launch(const ClassParams& p, int64_t nq, hipStream_t s, const double* centers, const double* exps,
                          const double* coefs, const int32_t* nprim, const double* stab, double* hbra, double* hket,
                          int64_t q0, int64_t hbs, int64_t hks) {
  const dim3 grid((unsigned)nq, (unsigned)(2 * p.kmax * p.kmax));
  const int lds = std::max(solid_h_lds(p.la, p.lb, p.np4), solid_h_lds(p.lc, p.ld, p.nq4));
  hipLaunchKernelGGL(solid_h_kernel, grid, dim3(kThreads), lds, s, p, centers, exps, coefs, nprim, stab, hbra,
                     hket, q0, hbs, hks);
  return hipGetLastError();
}

hipError_t solid_launch(const ClassParams& p, dim3 grid, hipStream_t s, const Tables& t, const double* centers,
                        const double* exps, const double* coefs, const int32_t* nprim, double* out, int64_t q0,
                        const double* hbra, const double* hket, int64_t hbs, int64_t hks) {
  const bool two = p.rb == 2;
#define L(RB, LAY) solid_launch_t<RB, LAY>(p, grid, s, t, centers, exps, coefs, nprim, out, q0, hbra, hket, hbs, hks)
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
