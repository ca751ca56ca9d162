// eri4_solid.hip -- solid-harmonic output (FP64): the kernel that builds the H
// matrices of every primitive pair, and the single-class integral kernels that
// read them, one instance per tile height and R layout.
#include "eri4_device.h"

namespace eri4 {
namespace {

// H = (C_1 x C_2) E for one primitive pair (Sec. 2, the contraction of E with
// the Cartesian-to-solid coefficients), written in the operand order of the
// transform that reads it (see gemm1_h): one workgroup per (quartet q0 +
// blockIdx.x, side = blockIdx.y & 1, pair slot blockIdx.y >> 1 = i * kmax + j).
// Side 0 is the bra (shells a, b; units of 16 rows, cp.nrt * cp.rb of them,
// cp.np4 k), side 1 the ket (shells c, d, sign (-1)^|q| of eq. (pq); cp.ncdb
// units of 16 columns, cp.nq4 k).  Elements past the solid functions or the
// Hermite functions are 0.  Pairs beyond the quartet's contraction lengths are
// skipped (the integral kernel does not read them).
__global__ __launch_bounds__(kThreads, 1) void solid_h_kernel(
    const ClassParams cp, const double* __restrict__ centers, const double* __restrict__ exps,
    const double* __restrict__ coefs, const int32_t* __restrict__ nprim, const double* __restrict__ stab,
    double* __restrict__ hbra, double* __restrict__ hket, int64_t q0, int64_t hbs, int64_t hks) {
  __shared__ double tabs[kMaxEtab];
  __shared__ double pair[16];
  __shared__ int2 htab[kMaxHerm];
  __shared__ int4 terms[2][kSolidRows][kSolidTerms];  // (table offsets x, y, z | Cartesian index) per term
  __shared__ double tcoef[2][kSolidRows][kSolidTerms];
  __shared__ int tcount[2][kSolidRows];
  const int tid = threadIdx.x, lane = tid & 63;
  const int64_t iq = blockIdx.x;
  const int64_t q = q0 + iq;
  const int side = blockIdx.y & 1, slot = blockIdx.y >> 1;
  const int kmax = cp.kmax;
  const int i = slot / kmax, j = slot - (slot / kmax) * kmax;
  const int K1 = nprim[q * 4 + 2 * side], K2 = nprim[q * 4 + 2 * side + 1];
  if (K1 < 1 || K1 > kmax || K2 < 1 || K2 > kmax || i >= K1 || j >= K2) return;
  const int l1 = side ? cp.lc : cp.la, l2 = side ? cp.ld : cp.lb;
  const int Lh = l1 + l2;
  const int nh = nherm(Lh), nk4 = side ? cp.nq4 : cp.np4;
  const int trow = side ? cp.tkrow : cp.tbrow, taxis = side ? cp.tkaxis : cp.tbaxis;
  const int s1 = 2 * l1 + 1, s2 = 2 * l2 + 1;
  if (tid == 0) {
    const double* c = centers + q * 12 + 6 * side;
    const double* e = exps + (q * 4 + 2 * side) * kmax;
    const double* w = coefs + (q * 4 + 2 * side) * kmax;
    make_pair(pair, e[i], e[kmax + j], w[i], w[kmax + j], c, c + 3);
  }
  build_htab(htab, Lh, nh, nk4, 0, 0, false, tid);
  // the two shells' solid functions as lists of (E-table offsets, coefficient)
  for (int e = tid; e < 2 * kSolidRows * kSolidTerms; e += kThreads) {
    const int sh = e / (kSolidRows * kSolidTerms), rem = e - sh * (kSolidRows * kSolidTerms);
    const int m = rem / kSolidTerms, jt = rem - m * kSolidTerms;
    const int l = sh ? l2 : l1;
    if (m < 2 * l + 1) {
      const double* ent = stab + (l * kSolidRows + m) * kSolidEntry;
      const int n = (int)ent[0];
      if (jt == 0) tcount[sh][m] = n;
      if (jt < n) {
        int x, y, z;
        cart_of(l, (int)ent[1 + 2 * jt], x, y, z);
        terms[sh][m][jt] = make_int4(x, y, z, 0);
        tcoef[sh][m][jt] = ent[2 + 2 * jt];
      }
    }
  }
  __syncthreads();
  if (tid < 64)
    build_etab(tabs, l1, l2, trow, taxis, 0.5 / pair[0], pair + 5, pair + 8, side == 1, lane);
  __syncthreads();
  const int nunits = side ? cp.ncdb : cp.nrt * cp.rb;
  const int64_t per = (int64_t)nk4 * 16;
  double* H = (side ? hket + (iq * kmax * kmax + slot) * hks : hbra + (iq * kmax * kmax + slot) * hbs);
  for (int64_t e = tid; e < nunits * per; e += kThreads) {
    const int u = (int)(e / per);
    const int rem = (int)(e - u * per);
    const int ln = rem & 63, k = 4 * (rem >> 6) + (ln >> 4);
    const int r = u * 16 + (ln & 15);
    double v = 0.0;
    if (r < s1 * s2 && k < nh) {
      const int m1 = r / s2, m2 = r - (r / s2) * s2;
      const int hx = htab[k].x;
      const int t = hx & 0xff, uu = (hx >> 8) & 0xff, w = (hx >> 16) & 0xff;
      const int n1 = tcount[0][m1], n2 = tcount[1][m2];
      for (int a = 0; a < n1; ++a) {
        const int4 ta = terms[0][m1][a];
        double sb = 0.0;
        for (int b = 0; b < n2; ++b) {
          const int4 tb = terms[1][m2][b];
          sb += tcoef[1][m2][b] * tabs[(ta.x * (l2 + 1) + tb.x) * trow + t] *
                tabs[taxis + (ta.y * (l2 + 1) + tb.y) * trow + uu] *
                tabs[2 * taxis + (ta.z * (l2 + 1) + tb.z) * trow + w];
        }
        v += tcoef[0][m1][a] * sb;
      }
    }
    H[e] = v;
  }
}

}  // namespace

hipError_t solid_set_attrs() {
  const void* k[8] = {(const void*)eri4_solid_kernel<1, kLayBox>,  (const void*)eri4_solid_kernel<2, kLayBox>,
                      (const void*)eri4_solid_kernel<4, kLayBox>,  (const void*)eri4_solid_kernel<1, kLaySlab>,
                      (const void*)eri4_solid_kernel<2, kLaySlab>, (const void*)eri4_solid_kernel<1, kLayBox2>,
                      (const void*)eri4_solid_kernel<2, kLayBox2>, (const void*)eri4_solid_kernel<4, kLayBox2>};
  for (const void* f : k) {
    const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLdsBytes);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t solid_h_launch(const ClassParams& p, int64_t nq, hipStream_t s, const double* centers, const double* exps,
                          const double* coefs, const int32_t* nprim, const double* stab, double* hbra, double* hket,
                          int64_t q0, int64_t hbs, int64_t hks) {
  const dim3 grid((unsigned)nq, (unsigned)(2 * p.kmax * p.kmax));
  hipLaunchKernelGGL(solid_h_kernel, grid, dim3(kThreads), 0, s, p, centers, exps, coefs, nprim, stab, hbra, hket, q0,
                     hbs, hks);
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
