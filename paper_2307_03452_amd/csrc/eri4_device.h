// eri4_device.h -- gfx950 device code of liberi4 (kernels and their helpers).
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
//
// Everything here has internal linkage: each translation unit that launches
// one of the kernels compiles its own copy (the fused kernels, the FP64 plan
// kernel and the FP32 plan kernel are built in separate units, in parallel).
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>
#include <stdint.h>

#include "eri4_internal.h"
#include "eri4_launch.h"

namespace eri4 {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

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

// Stage timers (compile-time, ERI4_STAGE_TIMERS): wave 0 of each workgroup of
// the Cartesian kernels reads the shader clock after every barrier that ends a
// stage and adds the cycles since the previous read to that stage; the sums of
// all workgroups go to g_stage_cycles at the end of each tile.  The stages
// follow the paper's per-kernel breakdown (Table 2): pair data, Boys function
// and bra 1-d tables ([0]^(m) of eq. (boys)), the recursion of eq. (md1), the
// first transform (eq. (ab_to_hermite)), the tile move and ket tables, and
// the second transform with the output write (eq. (cd_to_hermite)).
enum { kStPair = 0, kStBoysE, kStR, kStGemm1, kStMove, kStGemm2, kStTiles, kStCount };
#ifdef ERI4_STAGE_TIMERS
__device__ unsigned long long g_stage_cycles[kStCount];
struct StageClock {
  unsigned long long t, acc[kStCount];
  __device__ __forceinline__ void start() {
    t = __builtin_readcyclecounter();
    for (int i = 0; i < kStCount; ++i) acc[i] = 0;
  }
  __device__ __forceinline__ void mark(int st) {
    const unsigned long long n = __builtin_readcyclecounter();
    acc[st] += n - t;
    t = n;
  }
  __device__ __forceinline__ void flush(int tid) {
    if (tid == 0) {
      acc[kStTiles] = 1;
      for (int i = 0; i < kStCount; ++i) atomicAdd(&g_stage_cycles[i], acc[i]);
    }
  }
};
#define ERI4_STAGE(st) clk.mark(st)
#else
struct StageClock {
  __device__ __forceinline__ void start() {}
  __device__ __forceinline__ void flush(int) {}
};
#define ERI4_STAGE(st) ((void)0)
#endif

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
template <int NT>
__device__ __forceinline__ void etab_step(double (&e)[NT], double h, double c) {
  double prev = 0.0;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const double cur = e[t];
    const double nxt = (t + 1 < NT) ? e[t + 1] : 0.0;
    e[t] = h * prev + c * cur + (double)(t + 1) * nxt;
    prev = cur;
  }
}

// Three 1-d tables (x, y, z) of one primitive pair into LDS, one wave:
// row (a,b) of axis i at E + i*taxis + (a*(lb+1)+b)*trow, entries t < trow
// (t > a+b are 0, in particular the last one).  Each axis ends with an all-zero
// row at row index (la+1)*(lb+1), used for padding rows.  alt_sign multiplies
// entry t by (-1)^t (the ket side of eq. (pq)).
// TMAX (at least la+lb+1) entries of each recursion are kept in registers.
template <int TMAX = 16>
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
    double e[TMAX];
#pragma unroll
    for (int t = 0; t < TMAX; ++t) e[t] = (t == 0) ? 1.0 : 0.0;
    for (int s = 0; s < a; ++s) etab_step(e, h, pa);
    double* base = E + axis * taxis + a * (lb + 1) * trow;
    for (int b = 0; b <= lb; ++b) {
      double* row = base + b * trow;
#pragma unroll
      for (int t = 0; t < TMAX; ++t)
        if (t < trow) row[t] = (alt_sign && (t & 1)) ? -e[t] : e[t];
      for (int t = TMAX; t < trow; ++t) row[t] = 0.0;  // beyond a+b
      if (b < lb) etab_step(e, h, pb);
    }
  }
}

// Hermite index table: ordinal -> (t,u,v) in lexicographic order over
// t+u+v <= Lh, packed t | u<<8 | v<<16 | t<<24 together with its part of the R
// offset (box: t*S2 + u*S1 + v; slab: u*S1 + v, the slab of the summed t,
// taken from bits 24.., is added per gather).  Entries n..n_alloc-1 are
// padding: E index (Lh+1, 0, 0), whose value is 0, and R index (0,0,0).
template <int NT = kThreads>
__device__ void build_htab(int2* tab, int Lh, int n, int n_alloc, int S1, int S2, bool slab, int tid) {
  const int ncol = (Lh + 1) * (Lh + 2) / 2;
  for (int c = tid; c < ncol; c += NT) {
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
  for (int i = n + tid; i < n_alloc; i += NT) tab[i] = make_int2(Lh + 1, 0);
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

// The same recursion between two boxes (R0, R1 of the same layout): level m
// reads [.]^(m+1) from one box and writes [.]^(m) to the other, so one barrier
// per level suffices.  Level m writes R0 when m is even, so [r]^(0) ends in R0.
template <int NE>
__device__ void hermite_r_lds2(double* R0, double* R1, const double* baseM, int L, const double* PQ,
                               const uint2 (&ent_in)[NE], int tid) {
  uint2 ent[NE];
#pragma unroll
  for (int k = 0; k < NE; ++k) ent[k] = ent_in[k];
  const int Roff = (int)(R1 - R0);  // R1 = R0 + Roff (same LDS array)
  if (tid == 0) R0[(L & 1) ? Roff : 0] = baseM[L];
  __syncthreads();
  const double px = PQ[0], py = PQ[1], pz = PQ[2];
  for (int m = L - 1; m >= 0; --m) {
    const int src = ((m + 1) & 1) ? Roff : 0, dst = (m & 1) ? Roff : 0;
    const int nact = nherm(L - m);
    const int kact = (nact + kThreads - 1) / kThreads;  // entry slots in use at this level (uniform)
#pragma unroll
    for (int k = 0; k < NE; ++k) {
      if (k < kact) {
        asm volatile("" : "+v"(ent[k].x), "+v"(ent[k].y));
        const int e = tid + k * kThreads;
        const int o1 = (int)(ent[k].x >> 16);
        const int o2 = (int)(ent[k].y & 0xffffu);
        const int dir = (int)((ent[k].y >> 16) & 3u);
        const int ri = (int)(ent[k].y >> 18);
        const double c1 = dir == 0 ? px : (dir == 1 ? py : pz);
        const double v = c1 * R0[src + o1] + (double)max(ri - 1, 0) * R0[src + o2];
        if (e < nact && e > 0) R0[dst + (int)(ent[k].x & 0xffffu)] = v;
      }
    }
    if (tid == 0) R0[dst] = baseM[m];
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
// gemm1_range runs the k steps kbeg..kend-1 (multiples of 4) only.
template <int NR, int NC, bool SLAB, bool F32>
__device__ __forceinline__ void gemm1_range(typename Acc<F32>::type (&acc)[NR][NC], const double* __restrict__ brae,
                                            const double* __restrict__ R, const int2* __restrict__ ptab,
                                            const int (&rowx)[NR], const int (&rowy)[NR], const int (&rowz)[NR],
                                            const int (&offq)[NC], const int (&tq)[NC], int kbeg, int kend, int L,
                                            int S1, int lane) {
  if (kbeg >= kend) return;
  const int g = lane >> 4;
  int2 pt = ptab[kbeg + g];
  for (int kk = kbeg; kk < kend; kk += 4) {
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
    pt = ptab[min(kk + 4, kend - 4) + g];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const double a = ex[r] * ey[r] * ez[r];
#pragma unroll
      for (int c = 0; c < NC; ++c) acc[r][c] = mfma16<F32>(a, b[c], acc[r][c]);
    }
  }
}

template <int NR, int NC, bool SLAB, bool F32>
__device__ __forceinline__ void gemm1_pair(typename Acc<F32>::type (&acc)[NR][NC], const double* __restrict__ brae,
                                           const double* __restrict__ R, const int2* __restrict__ ptab,
                                           const int (&rowx)[NR], const int (&rowy)[NR], const int (&rowz)[NR],
                                           const int (&offq)[NC], const int (&tq)[NC], int np4, int L, int S1,
                                           int lane) {
  gemm1_range<NR, NC, SLAB, F32>(acc, brae, R, ptab, rowx, rowy, rowz, offq, tq, 0, np4, L, S1, lane);
}

// Second transform for one group of NC output column blocks (cb0, cb0+CSTRIDE, ...)
// and NR row blocks, then the output write:
//   out[ab][cd] (+)= sum_q X[ab][q] E_cd[cd][q]
// E_cd is the product of three ket-table entries (sign of eq. (pq) folded in).
template <int NR, int NC, bool F32, int CSTRIDE = 8>
__device__ __forceinline__ void gemm2_group(const ClassParams& cp, const double* __restrict__ X,
                                            const double* __restrict__ kete, const int2* __restrict__ qtab,
                                            int cb0, int row0, double* __restrict__ outq, bool first,
                                            double unscale, int lane) {
  const int g = lane >> 4, n = lane & 15;
  int kx[NC], ky[NC], kz[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const int cd = (cb0 + CSTRIDE * c) * 16 + n;
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
  auto load = [&](int kk, int pk, double (&aa)[NR], double (&xx)[NC], double (&yy)[NC], double (&zz)[NC]) {
    const int tq = pk & 0xff, uq = (pk >> 8) & 0xff, vq = (pk >> 16) & 0xff;
#pragma unroll
    for (int r = 0; r < NR; ++r) aa[r] = X[(r * 16 + n) * xs + kk + g];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      xx[c] = kete[kx[c] + tq];
      yy[c] = kete[ky[c] + uq];
      zz[c] = kete[kz[c] + vq];
    }
  };
  auto step = [&](const double (&aa)[NR], const double (&xx)[NC], const double (&yy)[NC], const double (&zz)[NC]) {
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const double b = xx[c] * yy[c] * zz[c];
#pragma unroll
      for (int r = 0; r < NR; ++r) acc[r][c] = mfma16<F32>(aa[r], b, acc[r][c]);
    }
  };
  if constexpr (NR <= 2) {
    // the operands of step k+4 are read before the MFMAs of step k are issued
    // (measured: 1-2% on tiles of up to 32 rows; not kept for 64-row tiles,
    // whose doubled operand registers cost more than it gains)
    double a[NR], fx[NC], fy[NC], fz[NC];
    load(0, qtab[g].x, a, fx, fy, fz);
    int pk = qtab[min(4, nq4 - 4) + g].x;
    for (int kk = 0; kk < nq4; kk += 4) {
      double an[NR], fxn[NC], fyn[NC], fzn[NC];
      load(min(kk + 4, nq4 - 4), pk, an, fxn, fyn, fzn);
      pk = qtab[min(kk + 8, nq4 - 4) + g].x;
      asm volatile("" ::: "memory");  // keep the prefetch ahead of the MFMAs
      step(a, fx, fy, fz);
#pragma unroll
      for (int r = 0; r < NR; ++r) a[r] = an[r];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        fx[c] = fxn[c];
        fy[c] = fyn[c];
        fz[c] = fzn[c];
      }
    }
  } else {
    int pk = qtab[g].x;
    for (int kk = 0; kk < nq4; kk += 4) {
      double a[NR], fx[NC], fy[NC], fz[NC];
      load(kk, pk, a, fx, fy, fz);
      pk = qtab[min(kk + 4, nq4 - 4) + g].x;
      step(a, fx, fy, fz);
    }
  }
#pragma unroll
  for (int r = 0; r < NR; ++r)
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const int cd = (cb0 + CSTRIDE * c) * 16 + n;
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

// Solid-harmonic mode: the transform matrices H = (C_a x C_b) E of one
// primitive pair come from device memory (solid_h_kernel), stored in the
// operand order of the matrix cores: for row (or column) block u and k step s,
// 64 doubles, lane l holding H[16u + (l & 15)][4s + (l >> 4)].  A wave's load of
// one operand is one contiguous 512-byte read.

// First transform, A operand from H: acc[r][c] += sum_p H[row block r][p] [p|q].
// H points at this lane's element of row block 0, k step 0; operands of step
// k+8 are requested while step k runs.
template <int NR, int NC, bool SLAB>
__device__ __forceinline__ void gemm1_h(typename Acc<false>::type (&acc)[NR][NC], const double* __restrict__ H,
                                        const double* __restrict__ R, const int2* __restrict__ ptab,
                                        const int (&offq)[NC], const int (&tq)[NC], int np4, int L, int S1,
                                        int lane) {
  const int g = lane >> 4;
  const int rs = np4 * 16;  // doubles per row block
  double a0[NR], a1[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    a0[r] = H[r * rs];
    a1[r] = H[r * rs + min(4, np4 - 4) * 16];
  }
  int2 pt = ptab[g];
  for (int kk = 0; kk < np4; kk += 4) {
    double b[NC], a2[NR];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      if constexpr (SLAB) {
        const int t = (pt.x >> 24) + tq[c];
        b[c] = R[slab_base(t, L, S1) + pt.y + offq[c]];
      } else {
        b[c] = R[pt.y + offq[c]];
      }
    }
    pt = ptab[min(kk + 4, np4 - 4) + g];
    const int k2 = min(kk + 8, np4 - 4);
#pragma unroll
    for (int r = 0; r < NR; ++r) a2[r] = H[r * rs + k2 * 16];
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int c = 0; c < NC; ++c) acc[r][c] = mfma16<false>(a0[r], b[c], acc[r][c]);
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      a0[r] = a1[r];
      a1[r] = a2[r];
    }
  }
}

// Second transform for one group of NC output column blocks, B operand from
// H_cd (Hk: this lane's element of column block 0, k step 0), then the output
// write, as gemm2_group.
template <int NR, int NC>
__device__ __forceinline__ void gemm2_group_h(const ClassParams& cp, const double* __restrict__ X,
                                              const double* __restrict__ Hk, int cb0, int row0,
                                              double* __restrict__ outq, bool first, int lane) {
  const int g = lane >> 4, n = lane & 15;
  const int cs = cp.nq4 * 16;  // doubles per column block
  typename Acc<false>::type acc[NR][NC];
#pragma unroll
  for (int r = 0; r < NR; ++r)
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[r][c] = acc_zero<false>();
  const int xs = cp.xs, nq4 = cp.nq4;
  double b0[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) b0[c] = Hk[(cb0 + 8 * c) * cs];
  for (int kk = 0; kk < nq4; kk += 4) {
    double a[NR], b1[NC];
#pragma unroll
    for (int r = 0; r < NR; ++r) a[r] = X[(r * 16 + n) * xs + kk + g];
    const int kn = min(kk + 4, nq4 - 4);
#pragma unroll
    for (int c = 0; c < NC; ++c) b1[c] = Hk[(cb0 + 8 * c) * cs + kn * 16];
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int r = 0; r < NR; ++r) acc[r][c] = mfma16<false>(a[r], b0[c], acc[r][c]);
#pragma unroll
    for (int c = 0; c < NC; ++c) b0[c] = b1[c];
  }
#pragma unroll
  for (int r = 0; r < NR; ++r)
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const int cd = (cb0 + 8 * c) * 16 + n;
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) {
        const int ab = row0 + r * 16 + acc_row<false>(jj, g);
        if (ab < cp.nab && cd < cp.ncd) {
          double* o = outq + (int64_t)ab * cp.ncd + cd;
          const double v = acc[r][c][jj];
          if (first)
            __builtin_nontemporal_store(v, o);
          else
            *o += v;
        }
      }
    }
}

// Exchange mode: bra row order.  Padded row pr of a quartet is shell-b
// component pr / P and shell-a component pr % P, with P = 16 * ceil(na / 16)
// rows per b (components a >= na are padding).
__device__ __forceinline__ int exch_rows_per_b(const ClassParams& cp) { return 16 * ((cp.na + 15) / 16); }
__device__ __forceinline__ void exch_row(const ClassParams& cp, int pr, int& ia, int& ib) {
  const int P = exch_rows_per_b(cp);
  ib = pr / P;
  ia = pr - ib * P;
}

// y blocks of one ket pair: block i of this wave (blk = wave + 8 i) is row
// block r = blk / ncc and column block cc = blk % ncc (c = 16 cc + lane % 16):
//   y[r][cc] += sum_q X[row block r][q] F^b[q][cc],  b the row block's shell-b component.
// F^b of this ket pair at F + (b * ncc + cc) * nq4 * 16 in operand order (k
// step s, lane l: F^b[4 s + l / 16][16 cc + l % 16]).  The operands of eight k
// steps are read before their products are issued.
template <int NR>
__device__ __forceinline__ void exch_gemm(const ClassParams& cp, const double* __restrict__ X,
                                          const double* __restrict__ F, int row0, int wave, int lane, d4 (&yacc)[2]) {
  const int g = lane >> 4, n = lane & 15;
  const int ncc = (cp.nc + 15) / 16;
  const int P = exch_rows_per_b(cp);
  const int64_t fs = (int64_t)cp.nq4 * 16;
  const int nq4 = cp.nq4;
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int blk = wave + 8 * i;
    if (blk >= NR * ncc) break;
    const int r = blk / ncc, cc = blk - (blk / ncc) * ncc;
    const int ib = (row0 + r * 16) / P;  // one b per row block
    if (ib >= cp.nb) continue;           // padding rows past the last b
    const double* __restrict__ Fb = F + ((int64_t)ib * ncc + cc) * fs + lane;
    const double* __restrict__ Xr = X + (r * 16 + n) * cp.xs + g;
    d4 acc = yacc[i];
    int kk = 0;
    for (; kk + 32 <= nq4; kk += 32) {
      double a[8], b[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) b[u] = Fb[(kk + 4 * u) * 16];
#pragma unroll
      for (int u = 0; u < 8; ++u) a[u] = Xr[kk + 4 * u];
#pragma unroll
      for (int u = 0; u < 8; ++u) acc = mfma16<false>(a[u], b[u], acc);
    }
    for (; kk < nq4; kk += 4) acc = mfma16<false>(Xr[kk], Fb[kk * 16], acc);
    yacc[i] = acc;
  }
}

// y of this wave's blocks to outq[(b * na + a) * nc + c] (valid a, b, c only).
template <int NR>
__device__ __forceinline__ void exch_store(const ClassParams& cp, const d4 (&yacc)[2], double* __restrict__ outq,
                                           int row0, int wave, int lane) {
  const int g = lane >> 4, n = lane & 15;
  const int ncc = (cp.nc + 15) / 16;
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int blk = wave + 8 * i;
    if (blk >= NR * ncc) break;
    const int r = blk / ncc, cc = blk - (blk / ncc) * ncc;
    const int ic = 16 * cc + n;
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) {
      int ia, ib;
      exch_row(cp, row0 + r * 16 + acc_row<false>(jj, g), ia, ib);
      if (ia < cp.na && ib < cp.nb && ic < cp.nc) outq[((int64_t)ib * cp.na + ia) * cp.nc + ic] = yacc[i][jj];
    }
  }
}

// LDS regions of the fused kernel (see make_params for the layout).
struct Lds {
  double *sh, *baseM, *kpair, *bpair, *pqv, *box, *box1, *brae, *X, *kete;
  int2 *ptab, *qtab;
};

// P - Q into s.pqv and [0]^(m) = (-2 rho)^m 2 pi^(5/2) / (zp zq sqrt(zp + zq))
// w_bra w_ket F_m(rho |PQ|^2) for m = 0..L into s.baseM (eq. (md1)'s start,
// with the pair weights of s.bpair[1], s.kpair[1] and the scale s.kpair[11]
// folded in), for the pairs in s.bpair and s.kpair.  Called by one wave.
__device__ __forceinline__ void hermite_base(const Lds& s, int L, const double* __restrict__ boys_tab, int lane) {
  if (lane < 3) s.pqv[lane] = s.bpair[2 + lane] - s.kpair[2 + lane];
  if (lane <= L) {
    const double pref = 2.0 * pow(M_PI, 2.5);
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
}

constexpr int kGroup = 4;  // output column blocks per second-transform pass

// Power-of-two scale of [0]^(m) for the ket pair in s.kpair (FP32 transforms
// only; 1 otherwise), into kpair[11] and its inverse into kpair[12].  The scale
// brings the largest product of bra and ket pair weights near 1 so that the
// FP32 operands of both transforms stay inside FP32's exponent range for
// quartets with tiny integrals; the output write divides it out.
template <bool F32>
__device__ __forceinline__ void ket_scale(const Lds& s, int kmax, int Ka, int Kb) {
  if constexpr (F32) {
    const double* A = s.sh;
    const double* B = s.sh + 3;
    const double* ex = s.sh + 12;
    const double* co = s.sh + 12 + 4 * kmax;
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

// Everything a workgroup does after its prologue, for NR valid row blocks and
// NC1 first-transform column blocks of this wave.
// SOLID: rows and columns are real solid harmonics and both transforms read
// their H matrices from hb / hk (this quartet's, hbs / hks doubles per
// primitive pair, pair (i, j) of shells with K1, K2 primitives at slot
// i * K2 + j); FP64 only.
// EXCH: no second transform either; bra rows are ordered (b, a) with a padded
// to a multiple of 16 (exch_row), so each 16-row block has one b, and [ab|q]
// is contracted on the matrix cores with F^b[q][c] = sum_d E_cd^q D_bd of ket
// pair (k, l) (exchange_f_kernel, at hk + (k * kmax + l) * hks in operand
// order), accumulated over the ket pairs into y[a][c] = sum_d (ab|cd) D_bd,
// written to outq[(b * na + a) * nc + c] for the tile's b (FP64, Cartesian).
template <int NR, int NC1, int LAY, bool F32, bool SOLID = false, bool EXCH = false>
__device__ __forceinline__ void fused_body(const ClassParams& cp, const Lds& s, const double* __restrict__ boys_tab,
                           const uint2 (&rent)[LAY == kLaySlab ? kRPerThread : kRPerBox], double* __restrict__ outq,
                           int row0, int Ka, int Kb, int Kc, int Kd, int tid, int wave, int lane,
                           const double* __restrict__ hb = nullptr, const double* __restrict__ hk = nullptr,
                           int64_t hbs = 0, int64_t hks = 0) {
  static_assert(!(SOLID && F32), "solid-harmonic output runs FP64 transforms");
  static_assert(!(EXCH && (F32 || SOLID)), "the exchange contraction runs FP64 Cartesian transforms");
  constexpr bool SLAB = LAY == kLaySlab;
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
  for (int r = 0; r < NR && !SOLID; ++r) {
    int ia, ib;
    bool valid;
    if constexpr (EXCH) {
      exch_row(cp, row0 + r * 16 + (lane & 15), ia, ib);
      valid = ia < cp.na && ib < cp.nb;
    } else {
      const int ab = row0 + r * 16 + (lane & 15);
      valid = ab < cp.nab;
      ia = ab / cp.nb;
      ib = ab - ia * cp.nb;
    }
    if (valid) {
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

  StageClock clk;
  clk.start();
  // EXCH: y blocks (row block, 16 columns c) of this wave, kept over the ket pairs
  d4 yacc[2] = {acc_zero<false>(), acc_zero<false>()};

  for (int kl = 0; kl < Kc * Kd; ++kl) {
    if (tid == 0) {
      const int k = kl / Kd, l = kl - (kl / Kd) * Kd;
      make_pair(s.kpair, ex[2 * kmax + k], ex[3 * kmax + l], co[2 * kmax + k], co[3 * kmax + l], C, D);
      ket_scale<F32>(s, kmax, Ka, Kb);
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
      ERI4_STAGE(kStPair);
      if (wave == 0) {
        hermite_base(s, cp.L, boys_tab, lane);
      } else if constexpr (!SOLID) {
        if (wave == 1)
          build_etab(s.brae, cp.la, cp.lb, cp.tbrow, cp.tbaxis, 0.5 / s.bpair[0], s.bpair + 5, s.bpair + 8, false,
                     lane);
      }
      __syncthreads();
      ERI4_STAGE(kStBoysE);
      if constexpr (LAY == kLayBox2)
        hermite_r_lds2(s.box, s.box1, s.baseM, cp.L, s.pqv, rent, tid);
      else
        hermite_r_lds(s.box, s.baseM, cp.L, s.pqv, rent, tid);
      ERI4_STAGE(kStR);
      // first transform, accumulated over ij: [ab|q] += E_ab^p [p|q]
      if constexpr (NC1 > 0 && SOLID) {
        const int i = ij / Kb, j = ij - (ij / Kb) * Kb;
        gemm1_h<NR, NC1, SLAB>(acc1, hb + (i * Kb + j) * hbs + (row0 / 16) * (cp.np4 * 16) + lane, s.box, s.ptab,
                               offq, tq, cp.np4, cp.L, cp.S1, lane);
      } else if constexpr (NC1 > 0) {
        gemm1_pair<NR, NC1, SLAB, F32>(acc1, s.brae, s.box, s.ptab, rowx, rowy, rowz, offq, tq, cp.np4, cp.L, cp.S1, lane);
      }
      __syncthreads();
      ERI4_STAGE(kStGemm1);
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
    if constexpr (EXCH) {
      // y[a][c] += sum_q [ab|q] F^b[q][c] for this ket pair; the barrier after
      // it protects the tile (aliased by the next pair's R box) until all reads
      __syncthreads();
      const int k = kl / Kd, l = kl - (kl / Kd) * Kd;
      exch_gemm<NR>(cp, s.X, hk + (k * kmax + l) * hks, row0, wave, lane, yacc);
      __syncthreads();
      continue;
    }
    if constexpr (!SOLID) {
      if (wave == 0)
        build_etab(s.kete, cp.lc, cp.ld, cp.tkrow, cp.tkaxis, 0.5 / s.kpair[0], s.kpair + 5, s.kpair + 8, true, lane);
    }
    __syncthreads();
    ERI4_STAGE(kStMove);

    // second transform, written to HBM (accumulated over kl); groups of
    // kGroup column blocks (2 with four row blocks, for the accumulators)
    const double unscale = s.kpair[12];
    constexpr int G2 = NR >= 4 ? 2 : kGroup;
    for (int g0 = 0; g0 < ncbw; g0 += G2) {
      const int ng = min(G2, ncbw - g0);
      const int cb0 = wave + 8 * g0;
      const bool first = kl == 0;
      if constexpr (SOLID) {
        const int k = kl / Kd, l = kl - (kl / Kd) * Kd;
        const double* hkp = hk + (k * Kd + l) * hks + lane;
        if (ng >= 2 && G2 >= 2)
          gemm2_group_h<NR, 2>(cp, s.X, hkp, cb0, row0, outq, first, lane);
        else
          gemm2_group_h<NR, 1>(cp, s.X, hkp, cb0, row0, outq, first, lane);
        if (ng == 3) gemm2_group_h<NR, 1>(cp, s.X, hkp, cb0 + 16, row0, outq, first, lane);
        if (ng == 4) gemm2_group_h<NR, 2>(cp, s.X, hkp, cb0 + 16, row0, outq, first, lane);
      } else if constexpr (G2 == 4) {
        if (ng == 4)
          gemm2_group<NR, 4, F32>(cp, s.X, s.kete, s.qtab, cb0, row0, outq, first, unscale, lane);
        else if (ng == 3)
          gemm2_group<NR, 3, F32>(cp, s.X, s.kete, s.qtab, cb0, row0, outq, first, unscale, lane);
        else if (ng == 2)
          gemm2_group<NR, 2, F32>(cp, s.X, s.kete, s.qtab, cb0, row0, outq, first, unscale, lane);
        else
          gemm2_group<NR, 1, F32>(cp, s.X, s.kete, s.qtab, cb0, row0, outq, first, unscale, lane);
      } else {
        if (ng == 2)
          gemm2_group<NR, 2, F32>(cp, s.X, s.kete, s.qtab, cb0, row0, outq, first, unscale, lane);
        else
          gemm2_group<NR, 1, F32>(cp, s.X, s.kete, s.qtab, cb0, row0, outq, first, unscale, lane);
      }
    }
    __syncthreads();
    ERI4_STAGE(kStGemm2);
  }
  clk.flush(tid);
  if constexpr (EXCH) exch_store<NR>(cp, yacc, outq, row0, wave, lane);
}

// Shell data of quartet q into LDS: centres A B C D in sh[0..11], then the
// exponents and the coefficients of shells a b c d (kmax each), and the four
// contraction lengths in shn[0..3].  PAIRS: the bra pair is entry q / nket of
// the bra list (centers, exps, coefs as [n][2][...]) and the ket pair entry
// q % nket of the ket list.  Called by all threads; the caller synchronises.
template <bool PAIRS>
__device__ __forceinline__ void load_shells(double* sh, int* shn, int kmax, const double* __restrict__ centers,
                                            const double* __restrict__ exps, const double* __restrict__ coefs,
                                            const int32_t* __restrict__ nprim, int64_t q,
                                            const double* __restrict__ kcenters, const double* __restrict__ kexps,
                                            const double* __restrict__ kcoefs, int64_t nket, int tid) {
  if constexpr (!PAIRS) {
    if (tid < 12) {
      sh[tid] = centers[q * 12 + tid];
    } else if (tid < 12 + 8 * kmax) {
      const int j = tid - 12;
      sh[tid] = (j < 4 * kmax) ? exps[q * 4 * kmax + j] : coefs[q * 4 * kmax + (j - 4 * kmax)];
    } else if (tid >= 256 && tid < 260) {
      shn[tid - 256] = nprim[q * 4 + (tid - 256)];
    }
  } else {
    const int64_t ib = q / nket, ik = q - ib * nket;
    if (tid < 12) {
      sh[tid] = tid < 6 ? centers[ib * 6 + tid] : kcenters[ik * 6 + (tid - 6)];
    } else if (tid < 12 + 8 * kmax) {
      const int j = tid - 12;
      const bool ex = j < 4 * kmax;
      const int jj = ex ? j : j - 4 * kmax;  // shell jj / kmax, primitive jj % kmax
      if (jj < 2 * kmax)
        sh[tid] = (ex ? exps : coefs)[ib * 2 * kmax + jj];
      else
        sh[tid] = (ex ? kexps : kcoefs)[ik * 2 * kmax + (jj - 2 * kmax)];
    } else if (tid >= 256 && tid < 260) {
      shn[tid - 256] = nprim[q * 4 + (tid - 256)];
    }
  }
}

// All the work of one tile: quartet q, bra rows rt*RB*16.., whose integrals
// start at outq.  Called by every thread of the workgroup; ends with a barrier.
// Shells of quartet q: from per-quartet arrays (PAIRS false: centers
// [q][4][3], exps/coefs [q][4][kmax]) or from a bra and a ket list of shell
// pairs (PAIRS true: bra pair q / nket, ket pair q % nket, each list centers
// [i][2][3], exps/coefs [i][2][kmax]; centers/exps/coefs are the bra list).
// SOLID: solid-harmonic rows and columns, H matrices from hb / hk (fused_body).
template <int RB, int LAY, bool F32, bool PAIRS, bool SOLID = false, bool EXCH = false>
__device__ __forceinline__ void process_tile(const ClassParams& cp, unsigned char* lds,
                                             const double* __restrict__ boys_tab,
                                             const uint2* __restrict__ rtab_L,
                                             const double* __restrict__ centers, const double* __restrict__ exps,
                                             const double* __restrict__ coefs, const int32_t* __restrict__ nprim,
                                             double* __restrict__ outq, int64_t q, int rt, int tid, int wave,
                                             int lane, const double* __restrict__ kcenters,
                                             const double* __restrict__ kexps, const double* __restrict__ kcoefs,
                                             int64_t nket, const double* __restrict__ hb = nullptr,
                                             const double* __restrict__ hk = nullptr, int64_t hbs = 0,
                                             int64_t hks = 0) {
  constexpr bool SLAB = LAY == kLaySlab;
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
  s.box1 = (double*)(lds + cp.o_box1);
  s.brae = (double*)(lds + cp.o_brae);
  s.X = (double*)(lds + cp.o_union);
  s.kete = (double*)(lds + cp.o_kete);
  int* shn = (int*)(s.sh + 12 + 8 * kmax);
  load_shells<PAIRS>(s.sh, shn, kmax, centers, exps, coefs, nprim, q, kcenters, kexps, kcoefs, nket, tid);
  build_htab(s.ptab, cp.Lb, cp.np, cp.np4, cp.S1, cp.S2, SLAB, tid);
  build_htab(s.qtab, cp.Lk, cp.nq, 16 * cp.nqb, cp.S1, cp.S2, SLAB, tid);
  uint2 rent[SLAB ? kRPerThread : kRPerBox];
  load_rtab(rent, rtab_L, cp.L, tid);
  __syncthreads();

  const int Ka = shn[0], Kb = shn[1], Kc = shn[2], Kd = shn[3];
  const int row0 = rt * RB * 16;
  if (Ka < 1 || Ka > kmax || Kb < 1 || Kb > kmax || Kc < 1 || Kc > kmax || Kd < 1 || Kd > kmax) {
    if constexpr (EXCH) {
      // this tile's rows (b, a) of y
      for (int i = tid; i < RB * 16 * cp.nc; i += kThreads) {
        int ia, ib;
        exch_row(cp, row0 + i / cp.nc, ia, ib);
        if (ia < cp.na && ib < cp.nb) outq[((int64_t)ib * cp.na + ia) * cp.nc + i % cp.nc] = __builtin_nan("");
      }
    } else {
      const int nrows = min(RB * 16, cp.nab - row0);
      const int ncols = cp.ncd;
      double* o = outq + (int64_t)row0 * ncols;
      for (int i = tid; i < nrows * ncols; i += kThreads) o[i] = __builtin_nan("");
    }
    __syncthreads();
    return;
  }
  const int nc1 = (wave < cp.nqb) ? min(kMaxC1, (cp.nqb - wave + 7) / 8) : 0;  // [ab|q] column blocks of this wave
  const int nrows_all = EXCH ? cp.nb * 16 * ((cp.na + 15) / 16) : cp.nab;           // (padded) bra rows
  const int nrv = min(RB, (nrows_all - row0 + 15) / 16);                          // valid row blocks of this tile
#define BODY(NR, NC1) \
  fused_body<NR, NC1, LAY, F32, SOLID, EXCH>(cp, s, boys_tab, rent, outq, row0, Ka, Kb, Kc, Kd, tid, wave, lane, hb, \
                                             hk, hbs, hks)
  constexpr int NR2 = RB >= 2 ? 2 : 1;
  if constexpr (RB == 4) {
    // 64-row tiles (kets with at most 2 column blocks per wave): the last tile
    // of a quartet runs with padding rows, whose outputs are not written
    switch (nc1) {
      case 0: BODY(4, 0); break;
      case 1: BODY(4, 1); break;
      default: BODY(4, 2); break;
    }
  } else if (nrv == NR2 && NR2 == 2) {
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
template <int RB, int LAY>
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
  process_tile<RB, LAY, false, false>(cp, lds, boys_tab, rtab + cp.rtab_off, centers, exps, coefs, nprim,
                                      out + q * (int64_t)cp.nab * cp.ncd, q, rt, tid, wave, lane, nullptr,
                                      nullptr, nullptr, 0);
}

// Solid-harmonic output, one class: as eri4_fused_kernel with rows and columns
// over real solid harmonics (cp.nab = (2la+1)(2lb+1), cp.ncd = (2lc+1)(2ld+1)).
// The H matrices of quartet q0 + i sit at hbra + i * kmax^2 * hbs and
// hket + i * kmax^2 * hks (solid_h_kernel).
template <int RB, int LAY>
__global__ __launch_bounds__(kThreads, 1) void eri4_solid_kernel(
    const ClassParams cp, const double* __restrict__ boys_tab, const uint2* __restrict__ rtab,
    const double* __restrict__ centers, const double* __restrict__ exps,
    const double* __restrict__ coefs, const int32_t* __restrict__ nprim, double* __restrict__ out,
    int64_t q0, const double* __restrict__ hbra, const double* __restrict__ hket, int64_t hbs, int64_t hks) {
  extern __shared__ __align__(16) unsigned char lds[];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t i = blockIdx.x / cp.nrt;
  const int64_t q = q0 + i;
  const int rt = blockIdx.x % cp.nrt;
  const int64_t kk2 = (int64_t)cp.kmax * cp.kmax;
  process_tile<RB, LAY, false, false, true>(cp, lds, boys_tab, rtab + cp.rtab_off, centers, exps, coefs, nprim,
                                            out + q * (int64_t)cp.nab * cp.ncd, q, rt, tid, wave, lane, nullptr,
                                            nullptr, nullptr, 0, hbra + i * kk2 * hbs, hket + i * kk2 * hks, hbs,
                                            hks);
}

// Persistent kernel for a plan: work items {quartet, row tile | class << 16},
// largest first, taken from a device counter until none are left (every
// workgroup exits once the counter passes nitems).  qoff[q] is where quartet
// q's integrals start in out.  Each class brings its own tile height and R
// layout.  F32: both transforms on FP32 matrix cores (eri4_plan_create).
template <bool F32, bool PAIRS>
__global__ __launch_bounds__(kThreads, 1) void eri4_plan_kernel(
    const ClassParams* __restrict__ classes, const int2* __restrict__ items, int nitems,
    const int64_t* __restrict__ qoff, const int32_t* __restrict__ nprim, int* __restrict__ counter,
    const double* __restrict__ boys_tab, const uint2* __restrict__ rtab,
    const double* __restrict__ centers, const double* __restrict__ exps,
    const double* __restrict__ coefs, double* __restrict__ out, const double* __restrict__ kcenters,
    const double* __restrict__ kexps, const double* __restrict__ kcoefs, int64_t nket) {
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
    const int lay = cp.lay;
    if (lay == kLaySlab) {
      if (cp.rb == 2)
        process_tile<2, kLaySlab, F32, PAIRS>(cp, lds, boys_tab, rt_L, centers, exps, coefs, nprim, oq, q, rt, tid, wave,
                                              lane, kcenters, kexps, kcoefs, nket);
      else
        process_tile<1, kLaySlab, F32, PAIRS>(cp, lds, boys_tab, rt_L, centers, exps, coefs, nprim, oq, q, rt, tid, wave,
                                              lane, kcenters, kexps, kcoefs, nket);
    } else if (lay == kLayBox2) {
      if (cp.rb == 4)
        process_tile<4, kLayBox2, F32, PAIRS>(cp, lds, boys_tab, rt_L, centers, exps, coefs, nprim, oq, q, rt, tid, wave,
                                              lane, kcenters, kexps, kcoefs, nket);
      else if (cp.rb == 2)
        process_tile<2, kLayBox2, F32, PAIRS>(cp, lds, boys_tab, rt_L, centers, exps, coefs, nprim, oq, q, rt, tid, wave,
                                              lane, kcenters, kexps, kcoefs, nket);
      else
        process_tile<1, kLayBox2, F32, PAIRS>(cp, lds, boys_tab, rt_L, centers, exps, coefs, nprim, oq, q, rt, tid, wave,
                                              lane, kcenters, kexps, kcoefs, nket);
    } else {
      if (cp.rb == 4)
        process_tile<4, kLayBox, F32, PAIRS>(cp, lds, boys_tab, rt_L, centers, exps, coefs, nprim, oq, q, rt, tid, wave,
                                              lane, kcenters, kexps, kcoefs, nket);
      else if (cp.rb == 2)
        process_tile<2, kLayBox, F32, PAIRS>(cp, lds, boys_tab, rt_L, centers, exps, coefs, nprim, oq, q, rt, tid, wave,
                                              lane, kcenters, kexps, kcoefs, nket);
      else
        process_tile<1, kLayBox, F32, PAIRS>(cp, lds, boys_tab, rt_L, centers, exps, coefs, nprim, oq, q, rt, tid, wave,
                                              lane, kcenters, kexps, kcoefs, nket);
    }
  }
}

template <bool F32, bool PAIRS>
hipError_t plan_set_attrs_t() {
  return hipFuncSetAttribute((const void*)eri4_plan_kernel<F32, PAIRS>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             kMaxLdsBytes - 64);
}

template <bool F32, bool PAIRS>
hipError_t plan_occupancy_t(int lds_bytes, int* per_cu) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, (const void*)eri4_plan_kernel<F32, PAIRS>, kThreads,
                                                      lds_bytes);
}

template <bool F32, bool PAIRS>
hipError_t plan_launch_t(dim3 grid, int lds_bytes, hipStream_t s, const Tables& t, const PlanArgs& a) {
  const Shells& h = a.shells;
  hipLaunchKernelGGL((eri4_plan_kernel<F32, PAIRS>), grid, dim3(kThreads), lds_bytes, s, a.classes, a.items,
                     a.nitems, a.qoff, a.nprim, a.counter, t.boys, t.rtab, h.centers, h.exps, h.coefs, a.out,
                     h.kcenters, h.kexps, h.kcoefs, h.nket);
  return hipGetLastError();
}

template <int RB, int LAY>
hipError_t solid_launch_t(const ClassParams& p, dim3 grid, hipStream_t s, const Tables& t, const double* centers,
                          const double* exps, const double* coefs, const int32_t* nprim, double* out, int64_t q0,
                          const double* hbra, const double* hket, int64_t hbs, int64_t hks) {
  hipLaunchKernelGGL((eri4_solid_kernel<RB, LAY>), grid, dim3(kThreads), p.lds_bytes, s, p, t.boys, t.rtab, centers,
                     exps, coefs, nprim, out, q0, hbra, hket, hbs, hks);
  return hipGetLastError();
}

}  // namespace
}  // namespace eri4
