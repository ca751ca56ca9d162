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
//
// The sum is taken in two steps per chunk of kHChunk Hermite indices k and
// per solid function m1 of the first shell:
//   P[b][k]     = sum_a C_1[m1][a] E_ab^k      (b over Cartesians of shell 2)
//   H[m1 m2][k] = sum_b C_2[m2][b] P[b][k]
// with the lanes of a wave on consecutive k (the same coefficient lists); H is
// stored straight into operand order.  Rows past the solid functions are
// zero-filled first.
constexpr int kHChunk = 64;
constexpr int kSolidHLds = ncart(kTableLMax) * kHChunk * 8;

__global__ __launch_bounds__(kThreads, 1) void solid_h_kernel(
    const ClassParams cp, const double* __restrict__ centers, const double* __restrict__ exps,
    const double* __restrict__ coefs, const int32_t* __restrict__ nprim, const double* __restrict__ stab,
    double* __restrict__ hbra, double* __restrict__ hket, int64_t q0, int64_t hbs, int64_t hks) {
  extern __shared__ __align__(16) unsigned char dyn[];
  double* P = (double*)dyn;  // [ncart(l2)][kHChunk]
  __shared__ double tabs[kMaxEtab];
  __shared__ double pair[16];
  __shared__ int2 htab[kMaxHerm];
  __shared__ int4 terms[2][kSolidRows][kSolidTerms];  // (a_x, a_y, a_z, Cartesian index) per term
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
  const int s1 = 2 * l1 + 1, s2 = 2 * l2 + 1, n2c = ncart(l2);
  const int nunits = side ? cp.ncdb : cp.nrt * cp.rb;
  if (tid == 0) {
    const double* c = centers + q * 12 + 6 * side;
    const double* e = exps + (q * 4 + 2 * side) * kmax;
    const double* w = coefs + (q * 4 + 2 * side) * kmax;
    make_pair(pair, e[i], e[kmax + j], w[i], w[kmax + j], c, c + 3);
  }
  build_htab(htab, Lh, nh, nk4, 0, 0, false, tid);
  // the two shells' solid functions as lists of (exponents, Cartesian index, coefficient)
  for (int e = tid; e < 2 * kSolidRows * kSolidTerms; e += kThreads) {
    const int sh = e / (kSolidRows * kSolidTerms), rem = e - sh * (kSolidRows * kSolidTerms);
    const int m = rem / kSolidTerms, jt = rem - m * kSolidTerms;
    const int l = sh ? l2 : l1;
    if (m < 2 * l + 1) {
      const double* ent = stab + (l * kSolidRows + m) * kSolidEntry;
      const int n = (int)ent[0];
      if (jt == 0) tcount[sh][m] = n;
      if (jt < n) {
        const int k = (int)ent[1 + 2 * jt];
        int x, y, z;
        cart_of(l, k, x, y, z);
        terms[sh][m][jt] = make_int4(x, y, z, k);
        tcoef[sh][m][jt] = ent[2 + 2 * jt];
      }
    }
  }
  __syncthreads();
  if (tid < 64)
    build_etab(tabs, l1, l2, trow, taxis, 0.5 / pair[0], pair + 5, pair + 8, side == 1, lane);
  __syncthreads();
  double* H = side ? hket + (iq * kmax * kmax + slot) * hks : hbra + (iq * kmax * kmax + slot) * hbs;
  const int per = nk4 * 16;  // doubles per unit of 16 rows
  // element (row r, k) of H in operand order
  auto at = [&](int r, int k) { return (r >> 4) * per + (k >> 2) * 64 + (k & 3) * 16 + (r & 15); };
  const int nrow = s1 * s2;
  for (int e = tid; e < (nunits * 16 - nrow) * nk4; e += kThreads) {
    const int r = nrow + e / nk4, k = e - (e / nk4) * nk4;
    H[at(r, k)] = 0.0;
  }
  for (int c0 = 0; c0 < nk4; c0 += kHChunk) {
    for (int m1 = 0; m1 < s1; ++m1) {
      const int n1 = tcount[0][m1];
      for (int e = tid; e < n2c * kHChunk; e += kThreads) {
        const int b = e / kHChunk, kc = e - b * kHChunk, k = c0 + kc;
        double v = 0.0;
        if (k < nh) {
          int bx, by, bz;
          cart_of(l2, b, bx, by, bz);
          const int hx = htab[k].x;
          const int t = hx & 0xff, u = (hx >> 8) & 0xff, w = (hx >> 16) & 0xff;
#pragma unroll 4
          for (int a = 0; a < n1; ++a) {
            const int4 ta = terms[0][m1][a];
            v += tcoef[0][m1][a] * tabs[(ta.x * (l2 + 1) + bx) * trow + t] *
                 tabs[taxis + (ta.y * (l2 + 1) + by) * trow + u] * tabs[2 * taxis + (ta.z * (l2 + 1) + bz) * trow + w];
          }
        }
        P[e] = v;
      }
      __syncthreads();
      for (int e = tid; e < s2 * kHChunk; e += kThreads) {
        const int m2 = e / kHChunk, kc = e - m2 * kHChunk, k = c0 + kc;
        const int n2 = tcount[1][m2];
        double v = 0.0;
#pragma unroll 4
        for (int b = 0; b < n2; ++b) v += tcoef[1][m2][b] * P[terms[1][m2][b].w * kHChunk + kc];
        if (k < nk4) H[at(m1 * s2 + m2, k)] = v;
      }
      __syncthreads();
    }
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
  return hipFuncSetAttribute((const void*)solid_h_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, kSolidHLds);
}

hipError_t solid_h_launch(const ClassParams& p, int64_t nq, hipStream_t s, const double* centers, const double* exps,
                          const double* coefs, const int32_t* nprim, const double* stab, double* hbra, double* hket,
                          int64_t q0, int64_t hbs, int64_t hks) {
  const dim3 grid((unsigned)nq, (unsigned)(2 * p.kmax * p.kmax));
  hipLaunchKernelGGL(solid_h_kernel, grid, dim3(kThreads), kSolidHLds, s, p, centers, exps, coefs, nprim, stab, hbra,
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
