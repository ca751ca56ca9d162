// eri4_small.hip -- (ab|cd) for classes whose four shells all have l <= 3
// ((dd|dd), (ff|ff) and the classes between), one or four waves per quartet.
//
// Their matrices are small (at most 100 x 84 for the first transform of
// (ff|ff)), so the 8-wave tile of the fused kernel spends most of its time in
// barriers and per-tile set-up.  Here one 64-lane workgroup computes a whole
// quartet with the same steps (Sec. 2: Boys function, eq. (md1) in LDS, the
// first transform (eq. (ab_to_hermite)) accumulated over the bra primitive
// pairs on the matrix cores, the second transform (eq. (cd_to_hermite)) into
// the output, accumulated over the ket primitive pairs), RG bra row blocks at
// a time, and many such waves share a compute unit, so that one quartet's
// recursion runs while another's products occupy the matrix cores.
#include "eri4_device.h"

namespace eri4 {
namespace {

constexpr int kSmallThreads = 64;
// Hermite recursion entries per lane: nherm(12) = 455 <= 8 * 64
constexpr int kSmallRE = 8;

// eq. (md1) for decreasing m in the box layout, by one wave (entries
// e = lane + 64 k of the recursion table for total order L, read from the
// copy in LDS: held in registers they cost 16 VGPRs for the whole kernel).
__device__ void hermite_r_wave(double* R, const double* baseM, int L, const double* PQ,
                               const uint2* __restrict__ entl, int lane) {
  if (lane == 0) R[0] = baseM[L];
  __syncthreads();
  const double px = PQ[0], py = PQ[1], pz = PQ[2];
  for (int m = L - 1; m >= 0; --m) {
    const int nact = nherm(L - m);
    double nv[kSmallRE];
    uint2 en[kSmallRE];
#pragma unroll
    for (int k = 0; k < kSmallRE; ++k) {
      const int e = lane + k * kSmallThreads;
      en[k] = e < nact ? entl[e] : make_uint2(0u, 0u);
    }
#pragma unroll
    for (int k = 0; k < kSmallRE; ++k) {
      const int e = lane + k * kSmallThreads;
      if (e < nact) {
        const int o1 = (int)(en[k].x >> 16);
        const int o2 = (int)(en[k].y & 0xffffu);
        const int dir = (int)((en[k].y >> 16) & 3u);
        const int ri = (int)(en[k].y >> 18);
        const double c1 = dir == 0 ? px : (dir == 1 ? py : pz);
        nv[k] = c1 * R[o1] + (double)max(ri - 1, 0) * R[o2];
      }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kSmallRE; ++k) {
      const int e = lane + k * kSmallThreads;
      if (e < nact && e > 0) R[en[k].x & 0xffffu] = nv[k];
    }
    if (lane == 0) R[0] = baseM[m];
    __syncthreads();
  }
}

// Second transform of the RG row blocks in X, in column groups of up to 3
// output column blocks, written (kl == 0) or added to the output.  (Groups of
// 4 hold 96 accumulator registers for RG = 3, which keeps the kernel from
// running two waves per SIMD.)
template <int RG>
__device__ __forceinline__ void small_gemm2(const ClassParams& cp, const double* __restrict__ X,
                                            const double* __restrict__ kete, const int2* __restrict__ qtab,
                                            int row0, double* __restrict__ outq, bool first, int lane) {
  for (int cb0 = 0; cb0 < cp.ncdb; cb0 += 3) {
    switch (min(3, cp.ncdb - cb0)) {
      case 3: gemm2_group<RG, 3, false, 1>(cp, X, kete, qtab, cb0, row0, outq, first, 1.0, lane); break;
      case 2: gemm2_group<RG, 2, false, 1>(cp, X, kete, qtab, cb0, row0, outq, first, 1.0, lane); break;
      default: gemm2_group<RG, 1, false, 1>(cp, X, kete, qtab, cb0, row0, outq, first, 1.0, lane); break;
    }
  }
}

// Waves per SIMD the one-wave kernel is compiled for: two (at most 256
// registers) wherever that costs at most a register or two of spills, one
// (the compiler may use all 512) for 3 row blocks x 4 column blocks, whose 96
// first-transform accumulators leave too little for the rest.  Measured on
// 4096 quartets: two waves per SIMD made (dd|dd) 1.5-1.6x and (pp|pp) 1.8x
// faster; (3, 4) on two waves spills 132 bytes per lane and was 11% slower.
template <int RG, int NCQ>
constexpr int small_waves() { return RG * NCQ >= 12 ? 1 : 2; }

// One quartet (q0 + blockIdx.x) per 64-lane workgroup.  RG: bra row blocks
// held in the first transform's accumulators at a time (the X region of cp
// holds RG * 16 rows); NCQ: 16-wide column blocks of [ab|q] (cp.nqb, at most
// 4).  Box layout of R (cp.lay == kLayBox, L <= 12).  The last
// align16(8 nherm(L)) bytes of the dynamic LDS hold the recursion entries.
template <int RG, int NCQ>
__global__ __launch_bounds__(kSmallThreads) __attribute__((amdgpu_waves_per_eu(small_waves<RG, NCQ>()))) void eri4_small_kernel(
    const ClassParams cp, const double* __restrict__ boys_tab, const uint2* __restrict__ rtab,
    const double* __restrict__ centers, const double* __restrict__ exps, const double* __restrict__ coefs,
    const int32_t* __restrict__ nprim, double* __restrict__ out, int64_t q0) {
  extern __shared__ __align__(16) unsigned char lds[];
  const int lane = threadIdx.x;
  const int64_t q = q0 + blockIdx.x;
  const int kmax = cp.kmax;
  double* sh = (double*)(lds + cp.o_shell);
  double* baseM = (double*)(lds + cp.o_base);
  double* kpair = baseM + 32;
  double* bpair = kpair + 16;
  double* pqv = bpair + 16;
  int2* ptab = (int2*)(lds + cp.o_ptab);
  int2* qtab = (int2*)(lds + cp.o_qtab);
  double* R = (double*)(lds + cp.o_union);
  double* brae = (double*)(lds + cp.o_brae);
  double* X = (double*)(lds + cp.o_union);
  double* kete = (double*)(lds + cp.o_kete);
  int* shn = (int*)(sh + 12 + 8 * kmax);
  double* outq = out + q * (int64_t)cp.nab * cp.ncd;

  for (int i = lane; i < 12 + 8 * kmax; i += kSmallThreads) {
    const int j = i - 12;
    sh[i] = i < 12 ? centers[q * 12 + i] : (j < 4 * kmax ? exps[q * 4 * kmax + j] : coefs[q * 4 * kmax + (j - 4 * kmax)]);
  }
  if (lane < 4) shn[lane] = nprim[q * 4 + lane];
  build_htab<kSmallThreads>(ptab, cp.Lb, cp.np, cp.np4, cp.S1, cp.S2, false, lane);
  build_htab<kSmallThreads>(qtab, cp.Lk, cp.nq, 16 * cp.nqb, cp.S1, cp.S2, false, lane);
  uint2* entl = (uint2*)(lds + cp.lds_bytes - ((8 * nherm(cp.L) + 15) & ~15));
  {
    const uint2* rt = rtab + cp.rtab_off;
    for (int e = lane; e < nherm(cp.L); e += kSmallThreads) entl[e] = rt[e];
  }
  __syncthreads();
  const int Ka = shn[0], Kb = shn[1], Kc = shn[2], Kd = shn[3];
  if (Ka < 1 || Ka > kmax || Kb < 1 || Kb > kmax || Kc < 1 || Kc > kmax || Kd < 1 || Kd > kmax) {
    for (int i = lane; i < cp.nab * cp.ncd; i += kSmallThreads) outq[i] = __builtin_nan("");
    return;
  }
  const double* A = sh;
  const double* B = sh + 3;
  const double* C = sh + 6;
  const double* D = sh + 9;
  const double* ex = sh + 12;
  const double* co = sh + 12 + 4 * kmax;
  const double pref = 2.0 * pow(M_PI, 2.5);
  // columns q of this lane in each block (B operand of the first transform)
  int offq[NCQ], tq[NCQ];
#pragma unroll
  for (int c = 0; c < NCQ; ++c) {
    const int2 e = qtab[c * 16 + (lane & 15)];
    offq[c] = e.y;
    tq[c] = 0;
  }

  for (int row0 = 0; row0 < cp.nab; row0 += RG * 16) {
    int rowx[RG], rowy[RG], rowz[RG];
#pragma unroll
    for (int r = 0; r < RG; ++r) {
      const int ab = row0 + r * 16 + (lane & 15);
      if (ab < cp.nab) {
        const int ia = ab / cp.nb, ib = ab - ia * cp.nb;
        int ax, ay, az, bx, by, bz;
        cart_of(cp.la, ia, ax, ay, az);
        cart_of(cp.lb, ib, bx, by, bz);
        rowx[r] = (ax * (cp.lb + 1) + bx) * cp.tbrow;
        rowy[r] = cp.tbaxis + (ay * (cp.lb + 1) + by) * cp.tbrow;
        rowz[r] = 2 * cp.tbaxis + (az * (cp.lb + 1) + bz) * cp.tbrow;
      } else {
        const int zr = (cp.la + 1) * (cp.lb + 1) * cp.tbrow;
        rowx[r] = zr;
        rowy[r] = cp.tbaxis + zr;
        rowz[r] = 2 * cp.tbaxis + zr;
      }
    }
    for (int kl = 0; kl < Kc * Kd; ++kl) {
      if (lane == 0) {
        const int k = kl / Kd, l = kl - (kl / Kd) * Kd;
        make_pair(kpair, ex[2 * kmax + k], ex[3 * kmax + l], co[2 * kmax + k], co[3 * kmax + l], C, D);
      }
      d4 acc1[RG][NCQ];
#pragma unroll
      for (int r = 0; r < RG; ++r)
#pragma unroll
        for (int c = 0; c < NCQ; ++c) acc1[r][c] = acc_zero<false>();
      for (int ij = 0; ij < Ka * Kb; ++ij) {
        if (lane == 0) {
          const int i = ij / Kb, j = ij - (ij / Kb) * Kb;
          make_pair(bpair, ex[i], ex[kmax + j], co[i], co[kmax + j], A, B);
        }
        __syncthreads();
        if (lane < 3) pqv[lane] = bpair[2 + lane] - kpair[2 + lane];
        if (lane <= cp.L) {
          const double zp = bpair[0], zq = kpair[0];
          const double zs = zp + zq;
          const double rho = zp * zq / zs;
          double r2 = 0.0;
#pragma unroll
          for (int x = 0; x < 3; ++x) {
            const double dd = bpair[2 + x] - kpair[2 + x];
            r2 += dd * dd;
          }
          const double F = boys_fm(lane, rho * r2, boys_tab);
          double pw = 1.0;
          for (int mm = 0; mm < lane; ++mm) pw *= -2.0 * rho;
          baseM[lane] = pw * (pref / (zp * zq * sqrt(zs))) * (bpair[1] * kpair[1]) * F;
        }
        build_etab<2 * kSmallLMax + 2>(brae, cp.la, cp.lb, cp.tbrow, cp.tbaxis, 0.5 / bpair[0], bpair + 5, bpair + 8, false, lane);
        __syncthreads();
        hermite_r_wave(R, baseM, cp.L, pqv, entl, lane);
        gemm1_range<RG, NCQ, false, false>(acc1, brae, R, ptab, rowx, rowy, rowz, offq, tq, 0, cp.np4, cp.L, cp.S1,
                                           lane);
        __syncthreads();
      }
      // [ab|q] of the RG row blocks -> LDS (over the R box), ket tables
      // (only the nq4 columns the second transform reads: rows are cp.xs long)
#pragma unroll
      for (int r = 0; r < RG; ++r)
#pragma unroll
        for (int c = 0; c < NCQ; ++c)
          if (c * 16 + (lane & 15) < cp.nq4) {
#pragma unroll
            for (int jj = 0; jj < 4; ++jj)
              X[(r * 16 + acc_row<false>(jj, lane >> 4)) * cp.xs + c * 16 + (lane & 15)] = acc1[r][c][jj];
          }
      build_etab<2 * kSmallLMax + 2>(kete, cp.lc, cp.ld, cp.tkrow, cp.tkaxis, 0.5 / kpair[0], kpair + 5, kpair + 8, true, lane);
      __syncthreads();
      small_gemm2<RG>(cp, X, kete, qtab, row0, outq, kl == 0, lane);
      __syncthreads();
    }
  }
}

// The same quartet on four waves (256 threads), for kets of more than four
// [ab|q] column blocks, whose one-wave form needs more than 256 registers:
// the recursion over 256 threads, the first transform's blocks dealt to the
// waves (column block c to wave c % 4, NCW at most per wave; or evenly over
// rows and columns, below), the second transform's output column blocks to
// wave c % 4.  Capped at four waves per SIMD (128 registers, some spilled),
// which measured faster than two, three or five.
constexpr int kSmall4Threads = 256;
constexpr int kSmall4RE = (nherm(4 * kSmallLMax) + kSmall4Threads - 1) / kSmall4Threads;

__device__ void hermite_r_4w(double* R, const double* baseM, int L, const double* PQ,
                             const uint2 (&ent)[kSmall4RE], int tid) {
  if (tid == 0) R[0] = baseM[L];
  __syncthreads();
  const double px = PQ[0], py = PQ[1], pz = PQ[2];
  for (int m = L - 1; m >= 0; --m) {
    const int nact = nherm(L - m);
    double nv[kSmall4RE];
#pragma unroll
    for (int k = 0; k < kSmall4RE; ++k) {
      const int e = tid + k * kSmall4Threads;
      if (e < nact) {
        const int o1 = (int)(ent[k].x >> 16);
        const int o2 = (int)(ent[k].y & 0xffffu);
        const int dir = (int)((ent[k].y >> 16) & 3u);
        const int ri = (int)(ent[k].y >> 18);
        const double c1 = dir == 0 ? px : (dir == 1 ? py : pz);
        nv[k] = c1 * R[o1] + (double)max(ri - 1, 0) * R[o2];
      }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kSmall4RE; ++k) {
      const int e = tid + k * kSmall4Threads;
      if (e < nact && e > 0) R[ent[k].x & 0xffffu] = nv[k];
    }
    if (tid == 0) R[0] = baseM[m];
    __syncthreads();
  }
}

// One quartet (q0 + blockIdx.x) per 256-thread workgroup; RG as in
// eri4_small_kernel, NCW: first-transform column blocks per wave (at most).
// With RG = 2 and six [ab|q] column blocks ((ff)-type kets), the first
// transform's 2 x 6 blocks are split evenly instead: wave w takes row block
// w / 2 and column blocks 3 (w % 2) .. 3 (w % 2) + 2, three MFMAs per k step
// where two row blocks x two column blocks (one of them a repeat on waves 2
// and 3) took four.
#ifndef ERI4_SMALL4_SPLIT
#define ERI4_SMALL4_SPLIT 1
#endif
template <int RG, int NCW>
__global__ __launch_bounds__(kSmall4Threads) __attribute__((amdgpu_waves_per_eu(4))) void eri4_small4_kernel(
    const ClassParams cp, const double* __restrict__ boys_tab, const uint2* __restrict__ rtab,
    const double* __restrict__ centers, const double* __restrict__ exps, const double* __restrict__ coefs,
    const int32_t* __restrict__ nprim, double* __restrict__ out, int64_t q0) {
  extern __shared__ __align__(16) unsigned char lds[];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t q = q0 + blockIdx.x;
  const int kmax = cp.kmax;
  double* sh = (double*)(lds + cp.o_shell);
  double* baseM = (double*)(lds + cp.o_base);
  double* kpair = baseM + 32;
  double* bpair = kpair + 16;
  double* pqv = bpair + 16;
  int2* ptab = (int2*)(lds + cp.o_ptab);
  int2* qtab = (int2*)(lds + cp.o_qtab);
  double* R = (double*)(lds + cp.o_union);
  double* brae = (double*)(lds + cp.o_brae);
  double* X = (double*)(lds + cp.o_union);
  double* kete = (double*)(lds + cp.o_kete);
  int* shn = (int*)(sh + 12 + 8 * kmax);
  double* outq = out + q * (int64_t)cp.nab * cp.ncd;

  for (int i = tid; i < 12 + 8 * kmax; i += kSmall4Threads) {
    const int j = i - 12;
    sh[i] = i < 12 ? centers[q * 12 + i] : (j < 4 * kmax ? exps[q * 4 * kmax + j] : coefs[q * 4 * kmax + (j - 4 * kmax)]);
  }
  if (tid < 4) shn[tid] = nprim[q * 4 + tid];
  build_htab<kSmall4Threads>(ptab, cp.Lb, cp.np, cp.np4, cp.S1, cp.S2, false, tid);
  build_htab<kSmall4Threads>(qtab, cp.Lk, cp.nq, 16 * cp.nqb, cp.S1, cp.S2, false, tid);
  uint2 ent[kSmall4RE];
  {
    const uint2* rt = rtab + cp.rtab_off;
    const int n = nherm(cp.L);
#pragma unroll
    for (int k = 0; k < kSmall4RE; ++k) {
      const int e = tid + k * kSmall4Threads;
      ent[k] = e < n ? rt[e] : make_uint2(0u, 0u);
    }
  }
  __syncthreads();
  const int Ka = shn[0], Kb = shn[1], Kc = shn[2], Kd = shn[3];
  if (Ka < 1 || Ka > kmax || Kb < 1 || Kb > kmax || Kc < 1 || Kc > kmax || Kd < 1 || Kd > kmax) {
    for (int i = tid; i < cp.nab * cp.ncd; i += kSmall4Threads) outq[i] = __builtin_nan("");
    return;
  }
  const double* A = sh;
  const double* B = sh + 3;
  const double* C = sh + 6;
  const double* D = sh + 9;
  const double* ex = sh + 12;
  const double* co = sh + 12 + 4 * kmax;
  const double pref = 2.0 * pow(M_PI, 2.5);
  // this wave's [ab|q] column blocks wave, wave + 4, ... (B operand of the first transform)
  constexpr bool SPLIT = ERI4_SMALL4_SPLIT && RG == 2 && NCW == 2;
  constexpr int NR1 = SPLIT ? 1 : RG;    // first-transform row blocks of this wave
  constexpr int NC1 = SPLIT ? 3 : NCW;   // and column blocks
  const int rw = SPLIT ? wave >> 1 : 0;  // its row block (SPLIT)
  // column block c of this wave, and whether it is one (not a repeat)
  auto col_block = [&](int c) { return SPLIT ? 3 * (wave & 1) + c : wave + 4 * c; };
  int offq[NC1], tq[NC1];
#pragma unroll
  for (int c = 0; c < NC1; ++c) {
    const int cb = min(col_block(c), cp.nqb - 1);
    offq[c] = qtab[cb * 16 + (lane & 15)].y;
    tq[c] = 0;
  }

  for (int row0 = 0; row0 < cp.nab; row0 += RG * 16) {
    int rowx[NR1], rowy[NR1], rowz[NR1];
#pragma unroll
    for (int r = 0; r < NR1; ++r) {
      const int ab = row0 + (rw + r) * 16 + (lane & 15);
      if (ab < cp.nab) {
        const int ia = ab / cp.nb, ib = ab - ia * cp.nb;
        int ax, ay, az, bx, by, bz;
        cart_of(cp.la, ia, ax, ay, az);
        cart_of(cp.lb, ib, bx, by, bz);
        rowx[r] = (ax * (cp.lb + 1) + bx) * cp.tbrow;
        rowy[r] = cp.tbaxis + (ay * (cp.lb + 1) + by) * cp.tbrow;
        rowz[r] = 2 * cp.tbaxis + (az * (cp.lb + 1) + bz) * cp.tbrow;
      } else {
        const int zr = (cp.la + 1) * (cp.lb + 1) * cp.tbrow;
        rowx[r] = zr;
        rowy[r] = cp.tbaxis + zr;
        rowz[r] = 2 * cp.tbaxis + zr;
      }
    }
    for (int kl = 0; kl < Kc * Kd; ++kl) {
      if (tid == 0) {
        const int k = kl / Kd, l = kl - (kl / Kd) * Kd;
        make_pair(kpair, ex[2 * kmax + k], ex[3 * kmax + l], co[2 * kmax + k], co[3 * kmax + l], C, D);
      }
      // accumulators of this wave's column blocks; a wave with fewer than NCW
      // also runs a repeat of the last column block, which it does not store
      // (fewer registers than a second accumulator set: measured faster)
      d4 acc1[NR1][NC1];
#pragma unroll
      for (int r = 0; r < NR1; ++r) {
#pragma unroll
        for (int c = 0; c < NC1; ++c) acc1[r][c] = acc_zero<false>();
      }
      for (int ij = 0; ij < Ka * Kb; ++ij) {
        if (tid == 64) {
          const int i = ij / Kb, j = ij - (ij / Kb) * Kb;
          make_pair(bpair, ex[i], ex[kmax + j], co[i], co[kmax + j], A, B);
        }
        __syncthreads();
        if (wave == 0) {
          if (lane < 3) pqv[lane] = bpair[2 + lane] - kpair[2 + lane];
          if (lane <= cp.L) {
            const double zp = bpair[0], zq = kpair[0];
            const double zs = zp + zq;
            const double rho = zp * zq / zs;
            double r2 = 0.0;
#pragma unroll
            for (int x = 0; x < 3; ++x) {
              const double dd = bpair[2 + x] - kpair[2 + x];
              r2 += dd * dd;
            }
            const double F = boys_fm(lane, rho * r2, boys_tab);
            double pw = 1.0;
            for (int mm = 0; mm < lane; ++mm) pw *= -2.0 * rho;
            baseM[lane] = pw * (pref / (zp * zq * sqrt(zs))) * (bpair[1] * kpair[1]) * F;
          }
        } else if (wave == 1) {
          build_etab<2 * kSmallLMax + 2>(brae, cp.la, cp.lb, cp.tbrow, cp.tbaxis, 0.5 / bpair[0], bpair + 5,
                                         bpair + 8, false, lane);
        }
        __syncthreads();
        hermite_r_4w(R, baseM, cp.L, pqv, ent, tid);
        if (col_block(0) < cp.nqb)
          gemm1_range<NR1, NC1, false, false>(acc1, brae, R, ptab, rowx, rowy, rowz, offq, tq, 0, cp.np4, cp.L, cp.S1,
                                              lane);
        __syncthreads();
      }
      // [ab|q] of this wave's blocks -> LDS (over the R box), ket tables
#pragma unroll
      for (int r = 0; r < NR1; ++r)
#pragma unroll
        for (int c = 0; c < NC1; ++c) {
          const int cb = col_block(c);
          if (cb < cp.nqb && cb * 16 + (lane & 15) < cp.nq4) {  // not a repeat; the nq4 columns read next
            const d4 v = acc1[r][c];
#pragma unroll
            for (int jj = 0; jj < 4; ++jj)
              X[((rw + r) * 16 + acc_row<false>(jj, lane >> 4)) * cp.xs + cb * 16 + (lane & 15)] = v[jj];
          }
        }
      if (wave == 2)
        build_etab<2 * kSmallLMax + 2>(kete, cp.lc, cp.ld, cp.tkrow, cp.tkaxis, 0.5 / kpair[0], kpair + 5, kpair + 8,
                                       true, lane);
      __syncthreads();
      // second transform: output column blocks wave, wave + 4, ...
      for (int cb0 = wave; cb0 < cp.ncdb; cb0 += 4)
        gemm2_group<RG, 1, false, 4>(cp, X, kete, qtab, cb0, row0, outq, kl == 0, 1.0, lane);
      __syncthreads();
    }
  }
}

template <int RG, int NCQ>
hipError_t small_launch_t(const ClassParams& p, int64_t nq, hipStream_t s, const Tables& t, const double* centers,
                          const double* exps, const double* coefs, const int32_t* nprim, double* out, int64_t q0) {
  hipLaunchKernelGGL((eri4_small_kernel<RG, NCQ>), dim3((unsigned)nq), dim3(kSmallThreads), p.lds_bytes, s, p, t.boys,
                     t.rtab, centers, exps, coefs, nprim, out, q0);
  return hipGetLastError();
}

template <int RG>
hipError_t small_launch_rg(const ClassParams& p, int64_t nq, hipStream_t s, const Tables& t, const double* centers,
                           const double* exps, const double* coefs, const int32_t* nprim, double* out, int64_t q0) {
  switch (p.nqb) {
    case 1: return small_launch_t<RG, 1>(p, nq, s, t, centers, exps, coefs, nprim, out, q0);
    case 2: return small_launch_t<RG, 2>(p, nq, s, t, centers, exps, coefs, nprim, out, q0);
    case 3: return small_launch_t<RG, 3>(p, nq, s, t, centers, exps, coefs, nprim, out, q0);
    case 4: return small_launch_t<RG, 4>(p, nq, s, t, centers, exps, coefs, nprim, out, q0);
    default: return hipErrorInvalidValue;  // more column blocks go to the four-wave kernel
  }
}

template <int RG, int NCW>
hipError_t small4_launch_t(const ClassParams& p, int64_t nq, hipStream_t s, const Tables& t, const double* centers,
                           const double* exps, const double* coefs, const int32_t* nprim, double* out, int64_t q0) {
  hipLaunchKernelGGL((eri4_small4_kernel<RG, NCW>), dim3((unsigned)nq), dim3(kSmall4Threads), p.lds_bytes, s, p,
                     t.boys, t.rtab, centers, exps, coefs, nprim, out, q0);
  return hipGetLastError();
}

template <int RG, int NCQ>
hipError_t small_attr_t() {
  return hipFuncSetAttribute((const void*)eri4_small_kernel<RG, NCQ>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             kSmallLdsMax);
}

}  // namespace

hipError_t small_set_attrs() {
  hipError_t e = hipSuccess;
#define A(RG)                                                                                                        \
  if (e == hipSuccess) e = small_attr_t<RG, 1>();                                                                     \
  if (e == hipSuccess) e = small_attr_t<RG, 2>();                                                                     \
  if (e == hipSuccess) e = small_attr_t<RG, 3>();                                                                     \
  if (e == hipSuccess) e = small_attr_t<RG, 4>();
  A(1) A(2) A(3)
#undef A
  const void* k4[6] = {(const void*)eri4_small4_kernel<1, 1>, (const void*)eri4_small4_kernel<1, 2>,
                       (const void*)eri4_small4_kernel<2, 1>, (const void*)eri4_small4_kernel<2, 2>,
                       (const void*)eri4_small4_kernel<3, 1>, (const void*)eri4_small4_kernel<3, 2>};
  for (const void* f : k4)
    if (e == hipSuccess) e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, kSmallLdsMax);
  return e;
}

hipError_t small4_launch(const ClassParams& p, int64_t nq, hipStream_t s, const Tables& t, const double* centers,
                         const double* exps, const double* coefs, const int32_t* nprim, double* out, int64_t q0) {
  const bool two = p.nqb > 4;
#define L(RG) (two ? small4_launch_t<RG, 2>(p, nq, s, t, centers, exps, coefs, nprim, out, q0) \
                   : small4_launch_t<RG, 1>(p, nq, s, t, centers, exps, coefs, nprim, out, q0))
  switch (p.rb) {
    case 3: return L(3);
    case 2: return L(2);
    default: return L(1);
  }
#undef L
}

hipError_t small_launch(const ClassParams& p, int64_t nq, hipStream_t s, const Tables& t, const double* centers,
                        const double* exps, const double* coefs, const int32_t* nprim, double* out, int64_t q0) {
  switch (p.rb) {
    case 3: return small_launch_rg<3>(p, nq, s, t, centers, exps, coefs, nprim, out, q0);
    case 2: return small_launch_rg<2>(p, nq, s, t, centers, exps, coefs, nprim, out, q0);
    default: return small_launch_rg<1>(p, nq, s, t, centers, exps, coefs, nprim, out, q0);
  }
}

}  // namespace eri4
