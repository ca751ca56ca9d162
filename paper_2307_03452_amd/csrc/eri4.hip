// eri4.hip -- gfx950 kernels and the C ABI of liberi4.
//
// (ab|cd) over contracted Cartesian Gaussians by the matrix form of the
// McMurchie-Davidson scheme (Asadchev & Valeev, Sec. 2 and Sec. 3):
//
//   [0]^(m) = (-2 rho)^m 2 pi^(5/2) / (zp zq sqrt(zp+zq)) F_m(rho |P-Q|^2)
//   [r + 1_i]^(m) = r_i [r - 1_i]^(m+1) + (P_i - Q_i) [r]^(m+1)      eq. (md1)
//   [p|q] = (-1)^|q| [p+q]^(0)                                       eq. (pq)
//   [ab|q] = sum_p E_ab^p [p|q]                                      eq. (ab_to_hermite)
//   (ab|cd) = sum_q E_cd^q [ab|q]                                    eq. (cd_to_hermite)
//
// One workgroup (8 waves) owns one quartet and a tile of RB*16 bra rows ab.
// For each ket primitive pair kl it accumulates, over the bra primitive pairs
// ij, the first transform [ab_tile|q] in FP64 MFMA registers (the contraction
// is folded into the product dimension, Sec. 3), moves that tile to LDS and
// applies the second transform straight into the output.  [p|q] is never
// stored: its entries are gathered from the R box in LDS, whose linear layout
// turns the index p+q into an address sum.  E entries are products of three
// 1-d tables in LDS.  The sign (-1)^|q| is folded into the ket tables and the
// Gaussian-product prefactors and contraction coefficients into [0]^(m).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <mutex>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "eri4.h"
#include "eri4_internal.h"

namespace eri4 {
void make_boys_table(std::vector<double>& tab);
void make_rtabs(std::vector<uint32_t>& tab, std::vector<int>& start);

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kMaxLdsBytes = 160 * 1024;

// ---------------------------------------------------------------------------
// device helpers
// ---------------------------------------------------------------------------

// D[16x16] += A[16x4] B[4x16] on the matrix cores, in FP64 or (F32 = true)
// with both operands rounded to FP32 and an FP32 accumulator.  Lane l holds
// A[l%16][l/16] and B[l/16][l%16]; element j of its accumulator is column l%16
// of row acc_row<F32>(j, l/16).
template <bool F32>
struct Acc {
  using type = d4;
};
template <>
struct Acc<true> {
  using type = f4;
};

template <bool F32>
__device__ __forceinline__ typename Acc<F32>::type mfma16(double a, double b, typename Acc<F32>::type c) {
  if constexpr (F32)
    return __builtin_amdgcn_mfma_f32_16x16x4f32((float)a, (float)b, c, 0, 0, 0);
  else
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <bool F32>
__device__ __forceinline__ int acc_row(int j, int g) {
  return F32 ? 4 * g + j : 4 * j + g;
}

template <bool F32>
__device__ __forceinline__ typename Acc<F32>::type acc_zero() {
  return typename Acc<F32>::type{0, 0, 0, 0};
}

// F_m(T), eq. (boys): Taylor expansion on the grid below kBoysTMax, asymptotic
// form above.  Negative T gives NaN.
__device__ double boys_fm(int m, double T, const double* __restrict__ tab) {
  if (T >= 0.0 && T < kBoysTMax) {
    const int i = (int)(T * kBoysInvH + 0.5);
    const double x = (double)i * kBoysH - T;  // -(T - T_i), exact
    const double* r = tab + (size_t)i * kBoysCols + m;
    double s = r[kBoysJ];
#pragma unroll
    for (int j = kBoysJ - 1; j >= 0; --j) s = fma(s * x, 1.0 / (double)(j + 1), r[j]);
    return s;
  }
  if (!(T >= 0.0)) return __builtin_nan("");
  // F_m(T) = Gamma(m+1/2) / (2 T^(m+1/2)); the neglected incomplete-gamma part
  // is below 1e-20 relative for T >= kBoysTMax and m <= kMaxL.
  return tab[(size_t)kBoysAsymRow * kBoysCols + m] / (pow(T, (double)m) * sqrt(T));
}

// One step of the E recursions that follow eq. (cart2herm-2):
//   E^t <- (1/(2 zp)) E^(t-1) + c E^t + (t+1) E^(t+1),  c = P-A or P-B.
__device__ __forceinline__ void etab_step(double (&e)[16], double h, double c) {
  double prev = 0.0;
#pragma unroll
  for (int t = 0; t < 16; ++t) {
    const double cur = e[t];
    const double nxt = (t + 1 < 16) ? e[t + 1] : 0.0;
    e[t] = h * prev + c * cur + (double)(t + 1) * nxt;
    prev = cur;
  }
}

// Three 1-d tables (x, y, z) of one primitive pair into LDS, one wave:
// row (a,b) of axis i at E + i*taxis + (a*(lb+1)+b)*trow, entries t < trow
// (t > a+b are 0, in particular the last one).  Each axis ends with an all-zero
// row at row index (la+1)*(lb+1), used for padding rows.  alt_sign multiplies
// entry t by (-1)^t (the ket side of eq. (pq)).
__device__ void build_etab(double* E, int la, int lb, int trow, int taxis, double h,
                           const double* PA, const double* PB, bool alt_sign, int lane) {
  const int na = la + 1;
  for (int j = lane; j < 3 * trow; j += 64) {  // the all-zero padding rows
    const int axis = j / trow;
    E[axis * taxis + na * (lb + 1) * trow + (j - axis * trow)] = 0.0;
  }
  if (lane < 3 * na) {
    const int axis = lane / na;
    const int a = lane - axis * na;
    const double pa = PA[axis], pb = PB[axis];
    double e[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) e[t] = (t == 0) ? 1.0 : 0.0;
    for (int s = 0; s < a; ++s) etab_step(e, h, pa);
    double* base = E + axis * taxis + a * (lb + 1) * trow;
    for (int b = 0; b <= lb; ++b) {
      double* row = base + b * trow;
#pragma unroll
      for (int t = 0; t < 16; ++t)
        if (t < trow) row[t] = (alt_sign && (t & 1)) ? -e[t] : e[t];
      for (int t = 16; t < trow; ++t) row[t] = 0.0;  // beyond a+b <= 14
      if (b < lb) etab_step(e, h, pb);
    }
  }
}

// Hermite index table: ordinal -> (t,u,v) in lexicographic order over
// t+u+v <= Lh, packed t | u<<8 | v<<16 | t<<24 together with its part of the R
// offset (box: t*S2 + u*S1 + v; slab: u*S1 + v, the slab of the summed t,
// taken from bits 24.., is added per gather).  Entries n..n_alloc-1 are
// padding: E index (Lh+1, 0, 0), whose value is 0, and R index (0,0,0).
__device__ void build_htab(int2* tab, int Lh, int n, int n_alloc, int S1, int S2, bool slab, int tid) {
  const int ncol = (Lh + 1) * (Lh + 2) / 2;
  for (int c = tid; c < ncol; c += kThreads) {
    int t = 0, rem = c;
    while (rem >= Lh - t + 1) {
      rem -= Lh - t + 1;
      ++t;
    }
    const int u = rem;
    // triples before column (t,u): all with a smaller t, then columns u' < u of this t
    const int first = (nherm(Lh) - nherm(Lh - t)) + u * (2 * (Lh - t) + 3 - u) / 2;
    for (int v = 0; v <= Lh - t - u; ++v)
      tab[first + v] = make_int2(t | (u << 8) | (v << 16) | (t << 24), (slab ? 0 : t * S2) + u * S1 + v);
  }
  for (int i = n + tid; i < n_alloc; i += kThreads) tab[i] = make_int2(Lh + 1, 0);
}

// Cartesian component index -> (x, y, z) for shell l (order ax = l..0, ay = l-ax..0).
__device__ __forceinline__ void cart_of(int l, int i, int& x, int& y, int& z) {
  int n = 0;
  while ((n + 1) * (n + 2) / 2 <= i) ++n;
  z = i - n * (n + 1) / 2;
  y = n - z;
  x = l - n;
}

// [r]^(0) for |r| <= L in LDS (box or slab layout, encoded in the table), by
// eq. (md1) for decreasing m, overwriting [r]^(m+1) with [r]^(m).  Each level
// reads all its operands into registers, then writes after a barrier.
// baseM[m] holds [0]^(m); PQ (3 doubles, LDS) is P - Q.  ent[] holds this
// thread's recursion-table entries; they are made opaque every level so that
// only the packed words stay live, not their decoded form.
template <int NE>
__device__ void hermite_r_lds(double* R, const double* baseM, int L, const double* PQ, const uint2 (&ent_in)[NE],
                              int tid) {
  uint2 ent[NE];
#pragma unroll
  for (int k = 0; k < NE; ++k) ent[k] = ent_in[k];
  if (tid == 0) R[0] = baseM[L];
  __syncthreads();
  const double px = PQ[0], py = PQ[1], pz = PQ[2];
  for (int m = L - 1; m >= 0; --m) {
    const int nact = nherm(L - m);
    const int kact = (nact + kThreads - 1) / kThreads;  // entry slots in use at this level (uniform)
    double nv[NE];
#pragma unroll
    for (int k = 0; k < NE; ++k) {
      if (k < kact) {
        asm volatile("" : "+v"(ent[k].x), "+v"(ent[k].y));
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
    for (int k = 0; k < NE; ++k) {
      if (k < kact) {
        const int e = tid + k * kThreads;
        if (e < nact && e > 0) R[ent[k].x & 0xffffu] = nv[k];
      }
    }
    if (tid == 0) R[0] = baseM[m];
    __syncthreads();
  }
}

template <int NE>
__device__ __forceinline__ void load_rtab(uint2 (&ent)[NE], const uint2* __restrict__ rt, int L, int tid) {
  const int n = nherm(L);
#pragma unroll
  for (int k = 0; k < NE; ++k) {
    const int e = tid + k * kThreads;
    ent[k] = (e < n) ? rt[e] : make_uint2(0u, 0u);
  }
}

// Primitive-pair data, stored in LDS as 11 doubles:
//   [0] z = za + zb, [1] w = ca cb exp(-za zb / z |A-B|^2) (Gaussian product
//   prefactor times the two contraction coefficients), [2..4] P, [5..7] P-A, [8..10] P-B.
// The ket pair's slots [11] and [12] hold the power-of-two scale of [0]^(m)
// and its inverse (1 in FP64).
constexpr int kPairDoubles = 11;

__device__ __forceinline__ void make_pair(double* out, double za, double zb, double ca, double cb,
                                          const double* A, const double* B) {
  const double z = za + zb;
  const double iz = 1.0 / z;
  double ab2 = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    // P - A = zb (B - A) / z and P - B = za (A - B) / z, formed without the
    // cancellation of subtracting two absolute positions
    const double dd = A[i] - B[i];
    out[2 + i] = (za * A[i] + zb * B[i]) * iz;
    out[5 + i] = -zb * iz * dd;
    out[8 + i] = za * iz * dd;
    ab2 += dd * dd;
  }
  out[0] = z;
  out[1] = ca * cb * exp(-za * zb * iz * ab2);
}

// First transform over one bra primitive pair for NR row blocks x NC column
// blocks of this wave (both fixed per wave):
//   acc[r][c] += sum_p E_ab[row block r][p] * box[off(p) + off(q in block c)]
// E_ab is the product of three bra-table entries.  All LDS reads of a k step
// are issued before its MFMAs; the next p index is fetched one step ahead.
template <int NR, int NC, bool SLAB, bool F32>
__device__ __forceinline__ void gemm1_pair(typename Acc<F32>::type (&acc)[NR][NC], const double* __restrict__ brae,
                                           const double* __restrict__ R, const int2* __restrict__ ptab,
                                           const int (&rowx)[NR], const int (&rowy)[NR], const int (&rowz)[NR],
                                           const int (&offq)[NC], const int (&tq)[NC], int np4, int L, int S1,
                                           int lane) {
  const int g = lane >> 4;
  int2 pt = ptab[g];
  for (int kk = 0; kk < np4; kk += 4) {
    const int tp = pt.x & 0xff, up = (pt.x >> 8) & 0xff, vp = (pt.x >> 16) & 0xff;
    double ex[NR], ey[NR], ez[NR], b[NC];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      ex[r] = brae[rowx[r] + tp];
      ey[r] = brae[rowy[r] + up];
      ez[r] = brae[rowz[r] + vp];
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      if constexpr (SLAB) {
        const int t = (pt.x >> 24) + tq[c];  // t of p+q selects the slab
        b[c] = R[slab_base(t, L, S1) + pt.y + offq[c]];
      } else {
        b[c] = R[pt.y + offq[c]];
      }
    }
    pt = ptab[min(kk + 4, np4 - 4) + g];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const double a = ex[r] * ey[r] * ez[r];
#pragma unroll
      for (int c = 0; c < NC; ++c) acc[r][c] = mfma16<F32>(a, b[c], acc[r][c]);
    }
  }
}

// Second transform for one group of NC output column blocks (cb0, cb0+8, ...)
// and NR row blocks, then the output write:
//   out[ab][cd] (+)= sum_q X[ab][q] E_cd[cd][q]
// E_cd is the product of three ket-table entries (sign of eq. (pq) folded in).
template <int NR, int NC, bool F32>
__device__ __forceinline__ void gemm2_group(const ClassParams& cp, const double* __restrict__ X,
                                            const double* __restrict__ kete, const int2* __restrict__ qtab,
                                            int cb0, int row0, double* __restrict__ outq, bool first,
                                            double unscale, int lane) {
  const int g = lane >> 4, n = lane & 15;
  int kx[NC], ky[NC], kz[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const int cd = (cb0 + 8 * c) * 16 + n;
    if (cd < cp.ncd) {
      const int ic = cd / cp.nd, id = cd - (cd / cp.nd) * cp.nd;
      int cx, cy, cz, dx, dy, dz;
      cart_of(cp.lc, ic, cx, cy, cz);
      cart_of(cp.ld, id, dx, dy, dz);
      kx[c] = (cx * (cp.ld + 1) + dx) * cp.tkrow;
      ky[c] = cp.tkaxis + (cy * (cp.ld + 1) + dy) * cp.tkrow;
      kz[c] = 2 * cp.tkaxis + (cz * (cp.ld + 1) + dz) * cp.tkrow;
    } else {
      const int zr = (cp.lc + 1) * (cp.ld + 1) * cp.tkrow;
      kx[c] = zr;
      ky[c] = cp.tkaxis + zr;
      kz[c] = 2 * cp.tkaxis + zr;
    }
  }
  typename Acc<F32>::type acc[NR][NC];
#pragma unroll
  for (int r = 0; r < NR; ++r)
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[r][c] = acc_zero<F32>();
  const int xs = cp.xs, nq4 = cp.nq4;
  int pk = qtab[g].x;
  for (int kk = 0; kk < nq4; kk += 4) {
    const int tq = pk & 0xff, uq = (pk >> 8) & 0xff, vq = (pk >> 16) & 0xff;
    double a[NR], fx[NC], fy[NC], fz[NC];
#pragma unroll
    for (int r = 0; r < NR; ++r) a[r] = X[(r * 16 + n) * xs + kk + g];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      fx[c] = kete[kx[c] + tq];
      fy[c] = kete[ky[c] + uq];
      fz[c] = kete[kz[c] + vq];
    }
    pk = qtab[min(kk + 4, nq4 - 4) + g].x;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const double b = fx[c] * fy[c] * fz[c];
#pragma unroll
      for (int r = 0; r < NR; ++r) acc[r][c] = mfma16<F32>(a[r], b, acc[r][c]);
    }
  }
#pragma unroll
  for (int r = 0; r < NR; ++r)
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const int cd = (cb0 + 8 * c) * 16 + n;
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) {
        const int ab = row0 + r * 16 + acc_row<F32>(jj, g);
        if (ab < cp.nab && cd < cp.ncd) {
          double* o = outq + (int64_t)ab * cp.ncd + cd;
          double v = acc[r][c][jj];
          if constexpr (F32) v *= unscale;
          if (first)
            __builtin_nontemporal_store(v, o);
          else
            *o += v;
        }
      }
    }
}

// LDS regions of the fused kernel (see make_params for the layout).
struct Lds {
  double *sh, *baseM, *kpair, *bpair, *pqv, *box, *brae, *X, *kete;
  int2 *ptab, *qtab;
};

constexpr int kGroup = 4;  // output column blocks per second-transform pass

// Everything a workgroup does after its prologue, for NR valid row blocks and
// NC1 first-transform column blocks of this wave.
template <int NR, int NC1, bool SLAB, bool F32>
__device__ __forceinline__ void fused_body(const ClassParams& cp, const Lds& s, const double* __restrict__ boys_tab,
                           const uint2 (&rent)[SLAB ? kRPerThread : kRPerBox], double* __restrict__ outq,
                           int row0, int Ka, int Kb, int Kc, int Kd, int tid, int wave, int lane) {
  const int kmax = cp.kmax;
  const double* A = s.sh;
  const double* B = s.sh + 3;
  const double* C = s.sh + 6;
  const double* D = s.sh + 9;
  const double* ex = s.sh + 12;
  const double* co = s.sh + 12 + 4 * kmax;
  constexpr int NC1A = NC1 > 0 ? NC1 : 1;

  // bra rows of this lane (A operand of the first transform)
  int rowx[NR], rowy[NR], rowz[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) {
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
  // [ab|q] columns of this lane (B operand of the first transform)
  int offq[NC1A], tq[NC1A];
#pragma unroll
  for (int c = 0; c < NC1A; ++c) {
    const int2 e = (c < NC1) ? s.qtab[(wave + 8 * c) * 16 + (lane & 15)] : make_int2(0, 0);
    offq[c] = e.y;
    tq[c] = (int)((unsigned)e.x >> 24);
  }
  const int ncbw = (wave < cp.ncdb) ? (cp.ncdb - wave + 7) / 8 : 0;  // output column blocks of this wave

  const double pref = 2.0 * pow(M_PI, 2.5);

  for (int kl = 0; kl < Kc * Kd; ++kl) {
    if (tid == 0) {
      const int k = kl / Kd, l = kl - (kl / Kd) * Kd;
      make_pair(s.kpair, ex[2 * kmax + k], ex[3 * kmax + l], co[2 * kmax + k], co[3 * kmax + l], C, D);
      if constexpr (F32) {
        // A power of two that brings the largest product of bra and ket pair
        // weights near 1: [0]^(m) is multiplied by it so that the FP32
        // operands of both transforms stay inside FP32's exponent range for
        // quartets with tiny integrals; the output write divides it out.
        double ab2 = 0.0;
        for (int x = 0; x < 3; ++x) ab2 += (A[x] - B[x]) * (A[x] - B[x]);
        double wmax = 0.0;
        for (int ij = 0; ij < Ka * Kb; ++ij) {
          const int i = ij / Kb, j = ij - (ij / Kb) * Kb;
          const double za = ex[i], zb = ex[kmax + j];
          wmax = fmax(wmax, fabs(co[i] * co[kmax + j]) * exp(-za * zb / (za + zb) * ab2));
        }
        const double wq = wmax * fabs(s.kpair[1]);
        const int e = (wq > 0.0 && wq < INFINITY) ? max(-1020, min(1020, ilogb(wq))) : 0;
        s.kpair[11] = ldexp(1.0, -e);
        s.kpair[12] = ldexp(1.0, e);
      } else {
        s.kpair[11] = 1.0;
        s.kpair[12] = 1.0;
      }
    }
    typename Acc<F32>::type acc1[NR][NC1A];
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int c = 0; c < NC1A; ++c) acc1[r][c] = acc_zero<F32>();

    for (int ij = 0; ij < Ka * Kb; ++ij) {
      if (tid == 64) {
        const int i = ij / Kb, j = ij - (ij / Kb) * Kb;
        make_pair(s.bpair, ex[i], ex[kmax + j], co[i], co[kmax + j], A, B);
      }
      __syncthreads();
      if (wave == 0) {
        if (lane < 3) s.pqv[lane] = s.bpair[2 + lane] - s.kpair[2 + lane];
        if (lane <= cp.L) {
          const double zp = s.bpair[0], zq = s.kpair[0];
          const double zs = zp + zq;
          const double rho = zp * zq / zs;
          double r2 = 0.0;
#pragma unroll
          for (int x = 0; x < 3; ++x) {
            const double d = s.bpair[2 + x] - s.kpair[2 + x];
            r2 += d * d;
          }
          const double F = boys_fm(lane, rho * r2, boys_tab);
          double pw = 1.0;
          for (int mm = 0; mm < lane; ++mm) pw *= -2.0 * rho;
          s.baseM[lane] = pw * (pref / (zp * zq * sqrt(zs))) * (s.bpair[1] * (s.kpair[1] * s.kpair[11])) * F;
        }
      } else if (wave == 1) {
        build_etab(s.brae, cp.la, cp.lb, cp.tbrow, cp.tbaxis, 0.5 / s.bpair[0], s.bpair + 5, s.bpair + 8, false,
                   lane);
      }
      __syncthreads();
      hermite_r_lds(s.box, s.baseM, cp.L, s.pqv, rent, tid);
      // first transform, accumulated over ij: [ab|q] += E_ab^p [p|q]
      if constexpr (NC1 > 0)
        gemm1_pair<NR, NC1, SLAB, F32>(acc1, s.brae, s.box, s.ptab, rowx, rowy, rowz, offq, tq, cp.np4, cp.L, cp.S1, lane);
      __syncthreads();
    }

    // [ab_tile|q] -> LDS (aliases the R box); ket tables for kl
    if constexpr (NC1 > 0) {
#pragma unroll
      for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int c = 0; c < NC1; ++c) {
          const int cb = wave + 8 * c;
#pragma unroll
          for (int jj = 0; jj < 4; ++jj)
            s.X[(r * 16 + acc_row<F32>(jj, lane >> 4)) * cp.xs + cb * 16 + (lane & 15)] = acc1[r][c][jj];
        }
    }
    if (wave == 0)
      build_etab(s.kete, cp.lc, cp.ld, cp.tkrow, cp.tkaxis, 0.5 / s.kpair[0], s.kpair + 5, s.kpair + 8, true, lane);
    __syncthreads();

    // second transform, written to HBM (accumulated over kl)
    const double unscale = s.kpair[12];
    for (int g0 = 0; g0 < ncbw; g0 += kGroup) {
      const int ng = min(kGroup, ncbw - g0);
      const int cb0 = wave + 8 * g0;
      const bool first = kl == 0;
      if (ng == 4)
        gemm2_group<NR, 4, F32>(cp, s.X, s.kete, s.qtab, cb0, row0, outq, first, unscale, lane);
      else if (ng == 3)
        gemm2_group<NR, 3, F32>(cp, s.X, s.kete, s.qtab, cb0, row0, outq, first, unscale, lane);
      else if (ng == 2)
        gemm2_group<NR, 2, F32>(cp, s.X, s.kete, s.qtab, cb0, row0, outq, first, unscale, lane);
      else
        gemm2_group<NR, 1, F32>(cp, s.X, s.kete, s.qtab, cb0, row0, outq, first, unscale, lane);
    }
    __syncthreads();
  }
}

// All the work of one tile: quartet q, bra rows rt*RB*16.., whose integrals
// start at outq.  Called by every thread of the workgroup; ends with a barrier.
template <int RB, bool SLAB, bool F32>
__device__ __forceinline__ void process_tile(const ClassParams& cp, unsigned char* lds,
                                             const double* __restrict__ boys_tab,
                                             const uint2* __restrict__ rtab_L,
                                             const double* __restrict__ centers, const double* __restrict__ exps,
                                             const double* __restrict__ coefs, const int32_t* __restrict__ nprim,
                                             double* __restrict__ outq, int64_t q, int rt, int tid, int wave,
                                             int lane) {
  const int kmax = cp.kmax;
  Lds s;
  s.sh = (double*)(lds + cp.o_shell);
  s.baseM = (double*)(lds + cp.o_base);
  s.kpair = s.baseM + 32;
  s.bpair = s.kpair + 16;
  s.pqv = s.bpair + 16;
  s.ptab = (int2*)(lds + cp.o_ptab);
  s.qtab = (int2*)(lds + cp.o_qtab);
  s.box = (double*)(lds + cp.o_union);
  s.brae = (double*)(lds + cp.o_brae);
  s.X = (double*)(lds + cp.o_union);
  s.kete = (double*)(lds + cp.o_kete);
  int* shn = (int*)(s.sh + 12 + 8 * kmax);

  // shell data of this quartet
  if (tid < 12) {
    s.sh[tid] = centers[q * 12 + tid];
  } else if (tid < 12 + 8 * kmax) {
    const int j = tid - 12;
    s.sh[tid] = (j < 4 * kmax) ? exps[q * 4 * kmax + j] : coefs[q * 4 * kmax + (j - 4 * kmax)];
  } else if (tid >= 256 && tid < 260) {
    shn[tid - 256] = nprim[q * 4 + (tid - 256)];
  }
  build_htab(s.ptab, cp.Lb, cp.np, cp.np4, cp.S1, cp.S2, SLAB, tid);
  build_htab(s.qtab, cp.Lk, cp.nq, 16 * cp.nqb, cp.S1, cp.S2, SLAB, tid);
  uint2 rent[SLAB ? kRPerThread : kRPerBox];
  load_rtab(rent, rtab_L, cp.L, tid);
  __syncthreads();

  const int Ka = shn[0], Kb = shn[1], Kc = shn[2], Kd = shn[3];
  const int row0 = rt * RB * 16;
  if (Ka < 1 || Ka > kmax || Kb < 1 || Kb > kmax || Kc < 1 || Kc > kmax || Kd < 1 || Kd > kmax) {
    const int nrows = min(RB * 16, cp.nab - row0);
    double* o = outq + (int64_t)row0 * cp.ncd;
    for (int i = tid; i < nrows * cp.ncd; i += kThreads) o[i] = __builtin_nan("");
    __syncthreads();
    return;
  }
  const int nc1 = (wave < cp.nqb) ? min(kMaxC1, (cp.nqb - wave + 7) / 8) : 0;  // [ab|q] column blocks of this wave
  const int nrv = min(RB, (cp.nab - row0 + 15) / 16);                             // valid row blocks of this tile
#define BODY(NR, NC1) fused_body<NR, NC1, SLAB, F32>(cp, s, boys_tab, rent, outq, row0, Ka, Kb, Kc, Kd, tid, wave, lane)
  constexpr int NR2 = RB >= 2 ? 2 : 1;
  if (nrv == NR2 && NR2 == 2) {
    switch (nc1) {
      case 0: BODY(NR2, 0); break;
      case 1: BODY(NR2, 1); break;
      case 2: BODY(NR2, 2); break;
      case 3: BODY(NR2, 3); break;
      default: BODY(NR2, 4); break;
    }
  } else if constexpr (SLAB) {
    switch (nc1) {
      case 0: BODY(1, 0); break;
      case 1: BODY(1, 1); break;
      case 2: BODY(1, 2); break;
      case 3: BODY(1, 3); break;
      case 4: BODY(1, 4); break;
      case 5: BODY(1, 5); break;
      default: BODY(1, 6); break;
    }
  } else {
    switch (nc1) {
      case 0: BODY(1, 0); break;
      case 1: BODY(1, 1); break;
      case 2: BODY(1, 2); break;
      case 3: BODY(1, 3); break;
      default: BODY(1, 4); break;
    }
  }
#undef BODY
}

// One workgroup = one quartet x one tile of RB*16 bra rows; 8 waves.  Grid:
// quartets q0.. in order, cp.nrt tiles each.
template <int RB, bool SLAB>
__global__ __launch_bounds__(kThreads, 1) void eri4_fused_kernel(
    const ClassParams cp, const double* __restrict__ boys_tab, const uint2* __restrict__ rtab,
    const double* __restrict__ centers, const double* __restrict__ exps,
    const double* __restrict__ coefs, const int32_t* __restrict__ nprim, double* __restrict__ out,
    int64_t q0) {
  extern __shared__ __align__(16) unsigned char lds[];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform (SGPR)
  const int64_t q = q0 + blockIdx.x / cp.nrt;
  const int rt = blockIdx.x % cp.nrt;
  process_tile<RB, SLAB, false>(cp, lds, boys_tab, rtab + cp.rtab_off, centers, exps, coefs, nprim,
                         out + q * (int64_t)cp.nab * cp.ncd, q, rt, tid, wave, lane);
}

// Persistent kernel for a plan: work items {quartet, row tile | class << 16},
// largest first, taken from a device counter until none are left (every
// workgroup exits once the counter passes nitems).  qoff[q] is where quartet
// q's integrals start in out.  Each class brings its own tile height and R
// layout.  F32: both transforms on FP32 matrix cores (eri4_plan_create).
template <bool F32>
__global__ __launch_bounds__(kThreads, 1) void eri4_plan_kernel(
    const ClassParams* __restrict__ classes, const int2* __restrict__ items, int nitems,
    const int64_t* __restrict__ qoff, const int32_t* __restrict__ nprim, int* __restrict__ counter,
    const double* __restrict__ boys_tab, const uint2* __restrict__ rtab,
    const double* __restrict__ centers, const double* __restrict__ exps,
    const double* __restrict__ coefs, double* __restrict__ out) {
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
    if (cp.slab) {
      if (cp.rb == 2)
        process_tile<2, true, F32>(cp, lds, boys_tab, rt_L, centers, exps, coefs, nprim, oq, q, rt, tid, wave, lane);
      else
        process_tile<1, true, F32>(cp, lds, boys_tab, rt_L, centers, exps, coefs, nprim, oq, q, rt, tid, wave, lane);
    } else {
      if (cp.rb == 2)
        process_tile<2, false, F32>(cp, lds, boys_tab, rt_L, centers, exps, coefs, nprim, oq, q, rt, tid, wave, lane);
      else
        process_tile<1, false, F32>(cp, lds, boys_tab, rt_L, centers, exps, coefs, nprim, oq, q, rt, tid, wave, lane);
    }
  }
}

__global__ void reset_counter_kernel(int* counter) {
  if (threadIdx.x == 0) counter[0] = 0;
}

// ---------------------------------------------------------------------------
// stage kernels (same device code as the fused kernel)
// ---------------------------------------------------------------------------

__global__ void boys_kernel(int mmax, int64_t n, const double* __restrict__ T, double* __restrict__ F,
                            const double* __restrict__ tab) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = n * (mmax + 1);
  if (g >= total) return;
  const int64_t i = g / (mmax + 1);
  const int m = (int)(g - i * (mmax + 1));
  F[g] = boys_fm(m, T[i], tab);
}

__global__ __launch_bounds__(kThreads, 1) void hermite_r_kernel(
    int L, bool slab, const double* __restrict__ zp, const double* __restrict__ zq, const double* __restrict__ P,
    const double* __restrict__ Q, double* __restrict__ R, const double* __restrict__ boys_tab,
    const uint2* __restrict__ rtab_L) {
  extern __shared__ __align__(16) unsigned char lds[];
  double* baseM = (double*)lds;
  double* pq = baseM + 32;
  double* box = baseM + 36;
  const int tid = threadIdx.x;
  const int64_t it = blockIdx.x;
  const int n1 = L + 1;
  const double a = zp[it], b = zq[it];
  double PQ[3];
  for (int x = 0; x < 3; ++x) PQ[x] = P[it * 3 + x] - Q[it * 3 + x];
  if (tid < 3) pq[tid] = PQ[tid];
  if (tid <= L) {
    const double rho = a * b / (a + b);
    const double T = rho * (PQ[0] * PQ[0] + PQ[1] * PQ[1] + PQ[2] * PQ[2]);
    double pw = 1.0;
    for (int mm = 0; mm < tid; ++mm) pw *= -2.0 * rho;
    baseM[tid] = pw * (2.0 * pow(M_PI, 2.5) / (a * b * sqrt(a + b))) * boys_fm(tid, T, boys_tab);
  }
  uint2 rent[kRPerThread];
  load_rtab(rent, rtab_L, L, tid);
  __syncthreads();
  hermite_r_lds(box, baseM, L, pq, rent, tid);
  double* o = R + it * (int64_t)n1 * n1 * n1;
  for (int e = tid; e < n1 * n1 * n1; e += kThreads) {
    const int t = e / (n1 * n1), u = (e / n1) % n1, v = e % n1;
    o[e] = (t + u + v <= L) ? box[r_offset(slab, L, t, u, v)] : 0.0;
  }
}

__global__ void hermite_e_kernel(int la, int lb, const double* __restrict__ za, const double* __restrict__ zb,
                                 const double* __restrict__ A, const double* __restrict__ B,
                                 double* __restrict__ E) {
  extern __shared__ __align__(16) unsigned char lds[];
  double* tabs = (double*)lds;
  const int lane = threadIdx.x;
  const int64_t it = blockIdx.x;
  const int trow = odd_row(la + lb + 2);
  const int taxis = ((la + 1) * (lb + 1) + 1) * trow;
  double* pair = tabs + 3 * taxis;
  if (lane == 0) {
    double Av[3], Bv[3];
    for (int x = 0; x < 3; ++x) {
      Av[x] = A[it * 3 + x];
      Bv[x] = B[it * 3 + x];
    }
    make_pair(pair, za[it], zb[it], 1.0, 1.0, Av, Bv);
  }
  __syncthreads();
  build_etab(tabs, la, lb, trow, taxis, 0.5 / pair[0], pair + 5, pair + 8, false, lane);
  __syncthreads();
  const int nt = la + lb + 1;
  const int per_axis = (la + 1) * (lb + 1) * nt;
  double* o = E + it * 3 * per_axis;
  for (int e = lane; e < 3 * per_axis; e += blockDim.x) {
    const int axis = e / per_axis, rem = e - axis * per_axis;
    const int ab = rem / nt, t = rem - ab * nt;
    o[e] = tabs[axis * taxis + ab * trow + t];
  }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

namespace {

thread_local std::string g_err;

eri4_status fail(eri4_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

struct DeviceState {
  bool ready = false;
  double* boys = nullptr;
  uint2* rtab = nullptr;
  int rstart[2 * (kMaxL + 1)] = {0};  // [layout][L], in uint2 entries
};

std::mutex g_mu;
std::vector<DeviceState> g_dev;

#define HIP_TRY(call)                                                                     \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess) return fail(ERI4_ERROR_HIP, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

template <int RB, bool SLAB>
eri4_status set_attr_one() {
  HIP_TRY(hipFuncSetAttribute((const void*)eri4_fused_kernel<RB, SLAB>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLdsBytes));
  return ERI4_SUCCESS;
}

eri4_status set_attrs() {
  eri4_status s;
  if ((s = set_attr_one<1, false>()) != ERI4_SUCCESS) return s;
  if ((s = set_attr_one<2, false>()) != ERI4_SUCCESS) return s;
  if ((s = set_attr_one<1, true>()) != ERI4_SUCCESS) return s;
  if ((s = set_attr_one<2, true>()) != ERI4_SUCCESS) return s;
  HIP_TRY(hipFuncSetAttribute((const void*)eri4_plan_kernel<false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              kMaxLdsBytes - 64));
  HIP_TRY(hipFuncSetAttribute((const void*)eri4_plan_kernel<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              kMaxLdsBytes - 64));
  HIP_TRY(hipFuncSetAttribute((const void*)hermite_r_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                              kMaxLdsBytes));
  return ERI4_SUCCESS;
}

eri4_status ensure_device(DeviceState** st) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_mu);
  if ((int)g_dev.size() <= dev) g_dev.resize(dev + 1);
  DeviceState& d = g_dev[dev];
  if (!d.ready) {
    static std::vector<double> boys;
    static std::vector<uint32_t> rt;
    static std::vector<int> rs;
    if (boys.empty()) {
      make_boys_table(boys);
      make_rtabs(rt, rs);
    }
    if ((int)rt.size() != 2 * 2 * kRtabEntries) return fail(ERI4_ERROR_INTERNAL, "recursion table size mismatch");
    if (hipMalloc(&d.boys, boys.size() * sizeof(double)) != hipSuccess)
      return fail(ERI4_ERROR_OUT_OF_MEMORY, "device allocation of the Boys table failed");
    if (hipMalloc(&d.rtab, rt.size() * sizeof(uint32_t)) != hipSuccess)
      return fail(ERI4_ERROR_OUT_OF_MEMORY, "device allocation of the recursion tables failed");
    HIP_TRY(hipMemcpy(d.boys, boys.data(), boys.size() * sizeof(double), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(d.rtab, rt.data(), rt.size() * sizeof(uint32_t), hipMemcpyHostToDevice));
    for (int i = 0; i < 2 * (kMaxL + 1); ++i) d.rstart[i] = rs[i];
    eri4_status s = set_attrs();
    if (s != ERI4_SUCCESS) return s;
    d.ready = true;
  }
  *st = &d;
  return ERI4_SUCCESS;
}

int align16(int x) { return (x + 15) & ~15; }

// Class parameters and LDS layout for a tile of rb*16 bra rows.
ClassParams make_params(int la, int lb, int lc, int ld, int kmax, int rb, bool slab) {
  ClassParams p{};
  p.rb = rb;
  p.slab = slab ? 1 : 0;
  p.la = la; p.lb = lb; p.lc = lc; p.ld = ld;
  p.na = ncart(la); p.nb = ncart(lb); p.nc = ncart(lc); p.nd = ncart(ld);
  p.nab = p.na * p.nb; p.ncd = p.nc * p.nd;
  p.Lb = la + lb; p.Lk = lc + ld; p.L = p.Lb + p.Lk;
  p.np = nherm(p.Lb); p.nq = nherm(p.Lk);
  p.np4 = (p.np + 3) & ~3; p.nq4 = (p.nq + 3) & ~3;
  p.nqb = (p.nq + 15) / 16;
  p.ncdb = (p.ncd + 15) / 16;
  p.nrt = (p.nab + 16 * rb - 1) / (16 * rb);
  p.S1 = box_s1(p.L); p.S2 = box_s2(p.L);
  p.tbrow = odd_row(p.Lb + 2); p.tkrow = odd_row(p.Lk + 2);
  p.tbaxis = ((la + 1) * (lb + 1) + 1) * p.tbrow;
  p.tkaxis = ((lc + 1) * (ld + 1) + 1) * p.tkrow;
  p.xs = 16 * p.nqb + 2;
  p.kmax = kmax;
  int off = 0;
  p.o_shell = off; off = align16(off + (12 + 8 * kmax) * 8 + 4 * 4);
  p.o_base = off;  off = align16(off + 96 * 8);  // [0]^(m), ket pair, bra pair, P-Q
  p.o_ptab = off;  off = align16(off + p.np4 * 8);
  p.o_qtab = off;  off = align16(off + 16 * p.nqb * 8);
  p.o_union = off;
  const int box_b = r_cells(slab, p.L) * 8;
  const int ph1 = align16(box_b) + 3 * p.tbaxis * 8;
  const int xb = align16(rb * 16 * p.xs * 8);
  const int ph2 = xb + 3 * p.tkaxis * 8;
  p.o_brae = off + align16(box_b);
  p.o_kete = off + xb;
  off = align16(off + (ph1 > ph2 ? ph1 : ph2));
  p.lds_bytes = off;
  return p;
}

// Class parameters: the first of (32-row tiles, box), (16, box), (32, slab),
// (16, slab) that fits in LDS (limit: bytes available for the dynamic area).
bool pick_params(int la, int lb, int lc, int ld, int kmax, const DeviceState* d, int limit, ClassParams* out) {
  const int rbs[4] = {2, 1, 2, 1};
  const bool slabs[4] = {false, false, true, true};
  for (int i = 0; i < 4; ++i) {
    ClassParams p = make_params(la, lb, lc, ld, kmax, rbs[i], slabs[i]);
    if (p.lds_bytes > limit || p.L > kMaxL || (p.nqb + 7) / 8 > (slabs[i] && rbs[i] == 1 ? kMaxC1 : 4)) continue;
    if (!slabs[i] && p.L > kBoxLMax) continue;  // the box recursion holds kRPerBox entries per thread
    p.rtab_off = d->rstart[(slabs[i] ? 1 : 0) * (kMaxL + 1) + p.L];
    *out = p;
    return true;
  }
  return false;
}

template <int RB, bool SLAB>
hipError_t launch_fused(const ClassParams& p, dim3 grid, hipStream_t s, const DeviceState* d,
                        const double* c, const double* e, const double* co, const int32_t* np, double* out,
                        int64_t q0) {
  hipLaunchKernelGGL((eri4_fused_kernel<RB, SLAB>), grid, dim3(kThreads), p.lds_bytes, s, p, d->boys, d->rtab, c,
                     e, co, np, out, q0);
  return hipGetLastError();
}

}  // namespace
}  // namespace eri4

using namespace eri4;

extern "C" {

int eri4_ncart(int l) { return l < 0 ? -1 : ncart(l); }

int64_t eri4_quartet_size(int la, int lb, int lc, int ld) {
  if (la < 0 || lb < 0 || lc < 0 || ld < 0) return -1;
  return (int64_t)ncart(la) * ncart(lb) * ncart(lc) * ncart(ld);
}

const char* eri4_last_error(void) { return g_err.c_str(); }

const char* eri4_version(void) { return "eri4 0.1 (gfx950, FP64 MFMA matrix McMurchie-Davidson)"; }

eri4_status eri4_init(void) {
  g_err.clear();
  DeviceState* d;
  return ensure_device(&d);
}

eri4_status eri4_batch(int la, int lb, int lc, int ld, int64_t nquartets, const double* centers,
                       const double* exponents, const double* coeffs, const int32_t* nprim, int kmax,
                       double* out, hipStream_t stream) {
  g_err.clear();
  if (la < 0 || lb < 0 || lc < 0 || ld < 0)
    return fail(ERI4_ERROR_INVALID_ARGUMENT, "angular momenta must be >= 0 (got %d %d %d %d)", la, lb, lc, ld);
  if (la > ERI4_MAX_L || lb > ERI4_MAX_L || lc > ERI4_MAX_L || ld > ERI4_MAX_L)
    return fail(ERI4_ERROR_UNSUPPORTED, "angular momentum above %d is not supported (got %d %d %d %d)",
                ERI4_MAX_L, la, lb, lc, ld);
  if (nquartets < 0) return fail(ERI4_ERROR_INVALID_ARGUMENT, "nquartets must be >= 0");
  if (kmax < 1 || kmax > ERI4_MAX_K)
    return fail(ERI4_ERROR_INVALID_ARGUMENT, "kmax must be in 1..%d (got %d)", ERI4_MAX_K, kmax);
  if (nquartets == 0) return ERI4_SUCCESS;
  if (!centers || !exponents || !coeffs || !nprim || !out)
    return fail(ERI4_ERROR_INVALID_ARGUMENT, "NULL buffer pointer");
  DeviceState* d;
  eri4_status s = ensure_device(&d);
  if (s != ERI4_SUCCESS) return s;
  ClassParams p;
  if (!pick_params(la, lb, lc, ld, kmax, d, kMaxLdsBytes, &p))
    return fail(ERI4_ERROR_UNSUPPORTED, "class (%d %d|%d %d) does not fit in LDS", la, lb, lc, ld);
  const int64_t max_blocks = (int64_t)1 << 30;
  const int64_t qchunk = max_blocks / p.nrt;
  for (int64_t q0 = 0; q0 < nquartets; q0 += qchunk) {
    const int64_t nq = (nquartets - q0 < qchunk) ? nquartets - q0 : qchunk;
    const dim3 grid((unsigned)(nq * p.nrt));
    hipError_t e;
    if (p.slab)
      e = (p.rb == 2) ? launch_fused<2, true>(p, grid, stream, d, centers, exponents, coeffs, nprim, out, q0)
                      : launch_fused<1, true>(p, grid, stream, d, centers, exponents, coeffs, nprim, out, q0);
    else
      e = (p.rb == 2) ? launch_fused<2, false>(p, grid, stream, d, centers, exponents, coeffs, nprim, out, q0)
                      : launch_fused<1, false>(p, grid, stream, d, centers, exponents, coeffs, nprim, out, q0);
    if (e != hipSuccess) return fail(ERI4_ERROR_HIP, "kernel launch: %s", hipGetErrorString(e));
  }
  return ERI4_SUCCESS;
}


// ---------------------------------------------------------------------------
// plans: many classes and contraction lengths in one persistent launch
// ---------------------------------------------------------------------------

struct eri4_plan_s {
  int device = 0;
  int64_t nq = 0;
  int kmax = 1;
  int nitems = 0;
  int nclasses = 0;
  int lds_bytes = 0;
  int grid = 0;
  bool f32 = false;  // ERI4_PREC_FP32
  int64_t out_size = 0;
  std::vector<int64_t> qoff;
  ClassParams* d_classes = nullptr;
  int2* d_items = nullptr;
  int64_t* d_qoff = nullptr;
  int32_t* d_nprim = nullptr;
  int* d_counter = nullptr;
};

static void plan_free(eri4_plan_s* p) {
  if (!p) return;
  if (p->d_classes) (void)hipFree(p->d_classes);
  if (p->d_items) (void)hipFree(p->d_items);
  if (p->d_qoff) (void)hipFree(p->d_qoff);
  if (p->d_nprim) (void)hipFree(p->d_nprim);
  if (p->d_counter) (void)hipFree(p->d_counter);
  delete p;
}

eri4_status eri4_plan_create(eri4_plan* plan, int64_t nquartets, const int32_t* l, const int32_t* nprim, int kmax,
                             eri4_precision precision) {
  g_err.clear();
  if (!plan) return fail(ERI4_ERROR_INVALID_ARGUMENT, "NULL plan pointer");
  *plan = nullptr;
  if (precision != ERI4_PREC_FP64 && precision != ERI4_PREC_FP32)
    return fail(ERI4_ERROR_INVALID_ARGUMENT, "unknown precision %d", (int)precision);
  if (nquartets < 0 || nquartets > ((int64_t)1 << 31) - 1)
    return fail(ERI4_ERROR_INVALID_ARGUMENT, "nquartets must be in 0..2^31-1");
  if (kmax < 1 || kmax > ERI4_MAX_K)
    return fail(ERI4_ERROR_INVALID_ARGUMENT, "kmax must be in 1..%d (got %d)", ERI4_MAX_K, kmax);
  if (nquartets > 0 && (!l || !nprim)) return fail(ERI4_ERROR_INVALID_ARGUMENT, "NULL host array");
  for (int64_t i = 0; i < 4 * nquartets; ++i) {
    if (l[i] < 0) return fail(ERI4_ERROR_INVALID_ARGUMENT, "negative angular momentum at quartet %lld", (long long)(i / 4));
    if (l[i] > ERI4_MAX_L)
      return fail(ERI4_ERROR_UNSUPPORTED, "angular momentum %d above %d at quartet %lld", l[i], ERI4_MAX_L,
                  (long long)(i / 4));
    if (nprim[i] < 1 || nprim[i] > kmax)
      return fail(ERI4_ERROR_INVALID_ARGUMENT, "contraction length %d outside 1..%d at quartet %lld", nprim[i], kmax,
                  (long long)(i / 4));
  }
  DeviceState* d;
  eri4_status st = ensure_device(&d);
  if (st != ERI4_SUCCESS) return st;
  eri4_plan_s* p = new (std::nothrow) eri4_plan_s();
  if (!p) return fail(ERI4_ERROR_OUT_OF_MEMORY, "host allocation failed");
  HIP_TRY(hipGetDevice(&p->device));
  p->nq = nquartets;
  p->kmax = kmax;
  p->f32 = precision == ERI4_PREC_FP32;

  // classes present, keyed by (la,lb,lc,ld)
  std::vector<int> cls_of_key(8 * 8 * 8 * 8, -1);
  std::vector<int> qcls(nquartets);
  std::vector<std::array<int, 4>> keys;
  for (int64_t q = 0; q < nquartets; ++q) {
    const int key = ((l[4 * q] * 8 + l[4 * q + 1]) * 8 + l[4 * q + 2]) * 8 + l[4 * q + 3];
    if (cls_of_key[key] < 0) {
      cls_of_key[key] = (int)keys.size();
      keys.push_back({l[4 * q], l[4 * q + 1], l[4 * q + 2], l[4 * q + 3]});
    }
    qcls[q] = cls_of_key[key];
  }
  // per class: tile height and R layout (see pick_params)
  std::vector<ClassParams> cps(keys.size());
  for (size_t c = 0; c < keys.size(); ++c) {
    if (!pick_params(keys[c][0], keys[c][1], keys[c][2], keys[c][3], kmax, d, kMaxLdsBytes - 64, &cps[c])) {
      plan_free(p);
      return fail(ERI4_ERROR_UNSUPPORTED, "class (%d %d|%d %d) does not fit in LDS", keys[c][0], keys[c][1],
                  keys[c][2], keys[c][3]);
    }
  }
  p->nclasses = (int)keys.size();
  for (const ClassParams& c : cps) p->lds_bytes = std::max(p->lds_bytes, c.lds_bytes);

  // output offsets in input order, and work items with their cost
  p->qoff.resize(nquartets);
  int64_t off = 0;
  std::vector<int2> items;
  std::vector<double> cost;
  for (int64_t q = 0; q < nquartets; ++q) {
    const ClassParams& c = cps[qcls[q]];
    p->qoff[q] = off;
    off += (int64_t)c.nab * c.ncd;
    const double kb = (double)nprim[4 * q] * nprim[4 * q + 1], kk = (double)nprim[4 * q + 2] * nprim[4 * q + 3];
    for (int rt = 0; rt < c.nrt; ++rt) {
      const int rows = 16 * std::min(c.rb, (c.nab - rt * c.rb * 16 + 15) / 16);
      // MFMA cycles of the two transforms at 128 FLOP/clk per CU, plus a
      // latency-bound estimate for Boys and the recursion per primitive quartet
      const double g1 = 2.0 * rows * c.np4 * 16.0 * c.nqb * kb * kk;
      const double g2 = 2.0 * rows * c.nq4 * 16.0 * c.ncdb * kk;
      cost.push_back((g1 + g2) / 128.0 + kb * kk * (8000.0 + 4.0 * nherm(c.L)) + 4000.0);
      items.push_back(make_int2((int)q, rt | (qcls[q] << 16)));
    }
  }
  p->out_size = off;
  std::vector<int> order(items.size());
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
  std::vector<int2> sorted(items.size());
  for (size_t i = 0; i < order.size(); ++i) sorted[i] = items[order[i]];
  if (sorted.size() > (size_t)INT32_MAX) {
    plan_free(p);
    return fail(ERI4_ERROR_INVALID_ARGUMENT, "too many work items");
  }
  p->nitems = (int)sorted.size();

  int ncu = 0, per_cu = 0;
  HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, p->device));
  const hipError_t oe =
      hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &per_cu, p->f32 ? (const void*)eri4_plan_kernel<true> : (const void*)eri4_plan_kernel<false>, kThreads,
          p->lds_bytes);
  if (oe != hipSuccess || per_cu < 1) per_cu = 1;
  p->grid = (int)std::min<int64_t>(std::max(p->nitems, 1), (int64_t)ncu * per_cu);

  const bool ok = hipMalloc(&p->d_classes, std::max<size_t>(1, cps.size()) * sizeof(ClassParams)) == hipSuccess &&
                  hipMalloc(&p->d_items, std::max<size_t>(1, sorted.size()) * sizeof(int2)) == hipSuccess &&
                  hipMalloc(&p->d_qoff, std::max<int64_t>(1, nquartets) * sizeof(int64_t)) == hipSuccess &&
                  hipMalloc(&p->d_nprim, std::max<int64_t>(1, 4 * nquartets) * sizeof(int32_t)) == hipSuccess &&
                  hipMalloc(&p->d_counter, 64) == hipSuccess;
  if (!ok) {
    plan_free(p);
    return fail(ERI4_ERROR_OUT_OF_MEMORY, "device allocation for the plan failed");
  }
  hipError_t e = hipSuccess;
  if (!cps.empty()) e = hipMemcpy(p->d_classes, cps.data(), cps.size() * sizeof(ClassParams), hipMemcpyHostToDevice);
  if (e == hipSuccess && !sorted.empty())
    e = hipMemcpy(p->d_items, sorted.data(), sorted.size() * sizeof(int2), hipMemcpyHostToDevice);
  if (e == hipSuccess && nquartets > 0)
    e = hipMemcpy(p->d_qoff, p->qoff.data(), nquartets * sizeof(int64_t), hipMemcpyHostToDevice);
  if (e == hipSuccess && nquartets > 0)
    e = hipMemcpy(p->d_nprim, nprim, 4 * nquartets * sizeof(int32_t), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    plan_free(p);
    return fail(ERI4_ERROR_HIP, "plan upload: %s", hipGetErrorString(e));
  }
  *plan = p;
  return ERI4_SUCCESS;
}

int64_t eri4_plan_output_size(eri4_plan plan) { return plan ? plan->out_size : -1; }

eri4_status eri4_plan_output_offsets(eri4_plan plan, int64_t* offsets) {
  g_err.clear();
  if (!plan) return fail(ERI4_ERROR_INVALID_ARGUMENT, "NULL plan");
  if (plan->nq > 0 && !offsets) return fail(ERI4_ERROR_INVALID_ARGUMENT, "NULL offsets array");
  std::copy(plan->qoff.begin(), plan->qoff.end(), offsets);
  return ERI4_SUCCESS;
}

eri4_status eri4_plan_execute(eri4_plan plan, const double* centers, const double* exponents, const double* coeffs,
                              double* out, hipStream_t stream) {
  g_err.clear();
  if (!plan) return fail(ERI4_ERROR_INVALID_ARGUMENT, "NULL plan");
  if (plan->nitems == 0) return ERI4_SUCCESS;
  if (!centers || !exponents || !coeffs || !out) return fail(ERI4_ERROR_INVALID_ARGUMENT, "NULL buffer pointer");
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev != plan->device)
    return fail(ERI4_ERROR_INVALID_ARGUMENT, "plan was made for device %d, current device is %d", plan->device, dev);
  DeviceState* d;
  eri4_status st = ensure_device(&d);
  if (st != ERI4_SUCCESS) return st;
  hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(64), 0, stream, plan->d_counter);
  HIP_TRY(hipGetLastError());
  if (plan->f32)
    hipLaunchKernelGGL(eri4_plan_kernel<true>, dim3(plan->grid), dim3(kThreads), plan->lds_bytes, stream,
                       plan->d_classes, plan->d_items, plan->nitems, plan->d_qoff, plan->d_nprim, plan->d_counter,
                       d->boys, d->rtab, centers, exponents, coeffs, out);
  else
    hipLaunchKernelGGL(eri4_plan_kernel<false>, dim3(plan->grid), dim3(kThreads), plan->lds_bytes, stream,
                       plan->d_classes, plan->d_items, plan->nitems, plan->d_qoff, plan->d_nprim, plan->d_counter,
                       d->boys, d->rtab, centers, exponents, coeffs, out);
  HIP_TRY(hipGetLastError());
  return ERI4_SUCCESS;
}

eri4_status eri4_plan_destroy(eri4_plan plan) {
  g_err.clear();
  plan_free(plan);
  return ERI4_SUCCESS;
}

eri4_status eri4_boys(int mmax, int64_t n, const double* T, double* F, hipStream_t stream) {
  g_err.clear();
  if (mmax < 0 || mmax > ERI4_MAX_BOYS_M)
    return fail(ERI4_ERROR_INVALID_ARGUMENT, "mmax must be in 0..%d", ERI4_MAX_BOYS_M);
  if (n < 0) return fail(ERI4_ERROR_INVALID_ARGUMENT, "n must be >= 0");
  if (n == 0) return ERI4_SUCCESS;
  if (!T || !F) return fail(ERI4_ERROR_INVALID_ARGUMENT, "NULL buffer pointer");
  DeviceState* d;
  eri4_status s = ensure_device(&d);
  if (s != ERI4_SUCCESS) return s;
  const int64_t total = n * (mmax + 1);
  const int64_t nb = (total + 255) / 256;
  if (nb > ((int64_t)1 << 31) - 1) return fail(ERI4_ERROR_INVALID_ARGUMENT, "n too large");
  hipLaunchKernelGGL(boys_kernel, dim3((unsigned)nb), dim3(256), 0, stream, mmax, n, T, F, d->boys);
  HIP_TRY(hipGetLastError());
  return ERI4_SUCCESS;
}

eri4_status eri4_hermite_r(int L, int64_t n, const double* zp, const double* zq, const double* P,
                           const double* Q, double* R, hipStream_t stream) {
  g_err.clear();
  if (L < 0 || L > 4 * ERI4_MAX_L)
    return fail(ERI4_ERROR_INVALID_ARGUMENT, "L must be in 0..%d", 4 * ERI4_MAX_L);
  if (n < 0) return fail(ERI4_ERROR_INVALID_ARGUMENT, "n must be >= 0");
  if (n == 0) return ERI4_SUCCESS;
  if (!zp || !zq || !P || !Q || !R) return fail(ERI4_ERROR_INVALID_ARGUMENT, "NULL buffer pointer");
  if (n > ((int64_t)1 << 31) - 1) return fail(ERI4_ERROR_INVALID_ARGUMENT, "n too large");
  DeviceState* d;
  eri4_status s = ensure_device(&d);
  if (s != ERI4_SUCCESS) return s;
  const bool slab = (36 + r_cells(false, L)) * 8 > kMaxLdsBytes;
  const int lds = (36 + r_cells(slab, L)) * 8;
  hipLaunchKernelGGL(hermite_r_kernel, dim3((unsigned)n), dim3(kThreads), lds, stream, L, slab, zp, zq, P, Q, R,
                     d->boys, d->rtab + d->rstart[(slab ? 1 : 0) * (kMaxL + 1) + L]);
  HIP_TRY(hipGetLastError());
  return ERI4_SUCCESS;
}

eri4_status eri4_hermite_e(int la, int lb, int64_t n, const double* za, const double* zb, const double* A,
                           const double* B, double* E, hipStream_t stream) {
  g_err.clear();
  if (la < 0 || lb < 0 || la > kTableLMax || lb > kTableLMax)
    return fail(ERI4_ERROR_INVALID_ARGUMENT, "la, lb must be in 0..%d", kTableLMax);
  if (n < 0) return fail(ERI4_ERROR_INVALID_ARGUMENT, "n must be >= 0");
  if (n == 0) return ERI4_SUCCESS;
  if (!za || !zb || !A || !B || !E) return fail(ERI4_ERROR_INVALID_ARGUMENT, "NULL buffer pointer");
  if (n > ((int64_t)1 << 31) - 1) return fail(ERI4_ERROR_INVALID_ARGUMENT, "n too large");
  DeviceState* d;
  eri4_status s = ensure_device(&d);
  if (s != ERI4_SUCCESS) return s;
  const int trow = odd_row(la + lb + 2);
  const int lds = (3 * ((la + 1) * (lb + 1) + 1) * trow + 16) * 8;
  hipLaunchKernelGGL(hermite_e_kernel, dim3((unsigned)n), dim3(64), lds, stream, la, lb, za, zb, A, B, E);
  HIP_TRY(hipGetLastError());
  return ERI4_SUCCESS;
}

}  // extern "C"
