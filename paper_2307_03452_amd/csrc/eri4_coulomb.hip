// eri4_coulomb.hip -- Coulomb contraction without forming (ab|cd) (FP64,
// Cartesian): J_ab = sum_cd (ab|cd) D_cd per quartet.  The ket density is first
// taken to Hermite space per ket primitive pair, dket^kl_q = sum_cd E_cd^q D_cd
// (sign of eq. (pq) included).  Since (ab|cd) = sum_pq E_ab^p [p+q] E_cd^q
// (eqs. (abcd_to_hermite), (pq)), J_ab = sum_p E_ab^p w_p with
// w_p = sum_kl sum_q [p+q]^kl dket^kl_q: the density is carried through the
// Hermite integrals as a matrix-vector product per primitive quartet, and the
// bra transform is a matrix-vector product per bra primitive pair, instead of
// the matrix-matrix products that form [ab|q] (a J-engine).
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

// Hermite-space J of bra primitive pairs ij0..ij1-1 of the quartet whose
// shells are in s.sh (contraction lengths Ka..Kd), summed over them into
// outJ[ab] (nab doubles, plain stores).  For each bra pair ij:
//   w_p  = sum over ket pairs kl, sum_q [p+q]^(0) dket^kl_q
//   J_ab += sum_p E_ab^p w_p
// with dket^kl at dket + (k * kmax + l) * ds (coulomb_dket_kernel).  The
// matrix-vector product runs with thread p on row p; when the bra has at most
// 256 Hermite functions, G groups of waves take every G-th q and their partial
// w are added in a fixed order.  The bra transform runs with thread ab on row
// ab, over p in the Hermite table's (t, u, v) order, the z factors of the row
// in registers.  NPT: Hermite functions per thread (2 when np > 512).
// Called by all threads; ends with a barrier.
constexpr int kJV = 2 * kTableLMax + 1;  // longest v run of a bra Hermite table
constexpr int kJAb = (ncart(kTableLMax) * ncart(kTableLMax) + kThreads - 1) / kThreads;  // J rows per thread

template <int LAY, int NPT>
__device__ void jengine_body(const ClassParams& cp, const Lds& s, double* __restrict__ wb,
                             const double* __restrict__ boys_tab,
                             const uint2 (&rent)[LAY == kLaySlab ? kRPerThread : kRPerBox], int Ka, int Kb, int Kc,
                             int Kd, int ij0, int ij1, const double* __restrict__ dket, int64_t ds,
                             double* __restrict__ outJ, int tid, int wave, int lane) {
  constexpr bool SLAB = LAY == kLaySlab;
  const int kmax = cp.kmax, np = cp.np, nq = cp.nq, L = cp.L, S1 = cp.S1, Lb = cp.Lb;
  const double* A = s.sh;
  const double* B = s.sh + 3;
  const double* C = s.sh + 6;
  const double* D = s.sh + 9;
  const double* ex = s.sh + 12;
  const double* co = s.sh + 12 + 4 * kmax;
  // matrix-vector rows of this thread: group g of G, rows pbase + lane (+ 512)
  const int P64 = NPT == 1 ? (np + 63) >> 6 : kWaves;
  const int G = NPT == 1 ? kWaves / P64 : 1;
  const int g = wave / P64;
  const int pbase = (wave - g * P64) * 64;
  const int gstride = P64 * 64;
  int pidx[NPT];
  int2 pt[NPT];
  bool pv[NPT];
#pragma unroll
  for (int r = 0; r < NPT; ++r) {
    pidx[r] = pbase + lane + r * kThreads;
    pv[r] = g < G && pidx[r] < np;
    pt[r] = pv[r] ? s.ptab[pidx[r]] : make_int2(0, 0);
  }
  // J rows of this thread and their 1-d table rows
  int rx[kJAb], ry[kJAb], rz[kJAb];
  bool av[kJAb];
#pragma unroll
  for (int r = 0; r < kJAb; ++r) {
    const int ab = tid + r * kThreads;
    av[r] = ab < cp.nab;
    rx[r] = ry[r] = rz[r] = 0;
    if (av[r]) {
      const int ia = ab / cp.nb, ib = ab - (ab / cp.nb) * cp.nb;
      int ax, ay, az, bx, by, bz;
      cart_of(cp.la, ia, ax, ay, az);
      cart_of(cp.lb, ib, bx, by, bz);
      rx[r] = (ax * (cp.lb + 1) + bx) * cp.tbrow;
      ry[r] = cp.tbaxis + (ay * (cp.lb + 1) + by) * cp.tbrow;
      rz[r] = 2 * cp.tbaxis + (az * (cp.lb + 1) + bz) * cp.tbrow;
    }
  }
  double J[kJAb];
#pragma unroll
  for (int r = 0; r < kJAb; ++r) J[r] = 0.0;

  for (int ij = ij0; ij < ij1; ++ij) {
    if (tid == 64) {
      const int i = ij / Kb, j = ij - (ij / Kb) * Kb;
      make_pair(s.bpair, ex[i], ex[kmax + j], co[i], co[kmax + j], A, B);
    }
    __syncthreads();
    if (wave == 1)
      build_etab(s.brae, cp.la, cp.lb, cp.tbrow, cp.tbaxis, 0.5 / s.bpair[0], s.bpair + 5, s.bpair + 8, false, lane);
    double w[NPT];
#pragma unroll
    for (int r = 0; r < NPT; ++r) w[r] = 0.0;
    for (int kl = 0; kl < Kc * Kd; ++kl) {
      const int k = kl / Kd, l = kl - (kl / Kd) * Kd;
      if (tid == 0) {
        make_pair(s.kpair, ex[2 * kmax + k], ex[3 * kmax + l], co[2 * kmax + k], co[3 * kmax + l], C, D);
        s.kpair[11] = 1.0;
      }
      __syncthreads();
      if (wave == 0) hermite_base(s, L, boys_tab, lane);
      __syncthreads();
      if constexpr (LAY == kLayBox2)
        hermite_r_lds2(s.box, s.box1, s.baseM, L, s.pqv, rent, tid);
      else
        hermite_r_lds(s.box, s.baseM, L, s.pqv, rent, tid);
      // w_p += sum_q [p+q] dket_q (the sign of eq. (pq) is in dket)
      const double* __restrict__ dq = dket + (int64_t)(k * kmax + l) * ds;
      if (g < G) {
        int q = g;
        for (; q + 3 * G < nq; q += 4 * G) {
          int2 qe[4];
          double d[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            qe[u] = s.qtab[q + u * G];
            d[u] = dq[q + u * G];
          }
#pragma unroll
          for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int r = 0; r < NPT; ++r) {
              const int sb = SLAB ? slab_base((pt[r].x >> 24) + (int)((unsigned)qe[u].x >> 24), L, S1) : 0;
              w[r] += s.box[sb + pt[r].y + qe[u].y] * d[u];
            }
        }
        for (; q < nq; q += G) {
          const int2 qe = s.qtab[q];
          const double d = dq[q];
#pragma unroll
          for (int r = 0; r < NPT; ++r) {
            const int sb = SLAB ? slab_base((pt[r].x >> 24) + (int)((unsigned)qe.x >> 24), L, S1) : 0;
            w[r] += s.box[sb + pt[r].y + qe.y] * d;
          }
        }
      }
    }
    __syncthreads();  // the last matrix-vector product has read R
#pragma unroll
    for (int r = 0; r < NPT; ++r)
      if (pv[r]) wb[g * gstride + pidx[r]] = w[r];
    __syncthreads();
    if (G > 1) {
      if (g == 0 && pv[0]) {
        double a = wb[pidx[0]];
        for (int gg = 1; gg < G; ++gg) a += wb[gg * gstride + pidx[0]];
        wb[pidx[0]] = a;
      }
      __syncthreads();
    }
    // J_ab += sum_p E_ab^p w_p, p in the (t, u, v) order of the Hermite table
#pragma unroll
    for (int r = 0; r < kJAb; ++r) {
      if (!av[r]) continue;
      double ez[kJV];
#pragma unroll
      for (int v = 0; v < kJV; ++v) ez[v] = v <= Lb ? s.brae[rz[r] + v] : 0.0;
      double acc = 0.0;
      int p = 0;
      for (int t = 0; t <= Lb; ++t) {
        const double et = s.brae[rx[r] + t];
        for (int u = 0; u <= Lb - t; ++u) {
          const double eu = et * s.brae[ry[r] + u];
          const int nv = Lb - t - u + 1;
          double sv = 0.0;
#pragma unroll
          for (int v = 0; v < kJV; ++v)
            if (v < nv) sv += ez[v] * wb[p + v];
          acc += eu * sv;
          p += nv;
        }
      }
      J[r] += acc;
    }
    __syncthreads();  // brae and wb are rewritten for the next bra pair
  }
#pragma unroll
  for (int r = 0; r < kJAb; ++r)
    if (av[r]) outJ[tid + r * kThreads] = J[r];
}

// Prologue and body for quartet q (shells from the quartet arrays, or PAIRS:
// from the bra and ket lists) and its bra pairs ij0..ij1-1 (or all of them,
// ij1 < 0); returns without writing when the contraction lengths are out of
// range or ij0 is not a pair of the quartet.
template <int LAY, int NPT, bool PAIRS>
__device__ void jengine_quartet(const ClassParams& cp, unsigned char* lds, const double* __restrict__ boys_tab,
                                const uint2* __restrict__ rtab_L, const double* __restrict__ centers,
                                const double* __restrict__ exps, const double* __restrict__ coefs,
                                const int32_t* __restrict__ nprim, int64_t q, const double* __restrict__ kcenters,
                                const double* __restrict__ kexps, const double* __restrict__ kcoefs, int64_t nket,
                                int i0, int j0, bool all, const double* __restrict__ dket, int64_t ds,
                                double* __restrict__ outJ, int64_t jstride, int tid, int wave, int lane) {
  constexpr bool SLAB = LAY == kLaySlab;
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
  double* wb = (double*)(lds + cp.o_jw);
  int* shn = (int*)(s.sh + 12 + 8 * cp.kmax);
  load_shells<PAIRS>(s.sh, shn, cp.kmax, centers, exps, coefs, nprim, q, kcenters, kexps, kcoefs, nket, tid);
  build_htab(s.ptab, cp.Lb, cp.np, cp.np4, cp.S1, cp.S2, SLAB, tid);
  build_htab(s.qtab, cp.Lk, cp.nq, 16 * cp.nqb, cp.S1, cp.S2, SLAB, tid);
  uint2 rent[SLAB ? kRPerThread : kRPerBox];
  load_rtab(rent, rtab_L, cp.L, tid);
  __syncthreads();
  const int kmax = cp.kmax;
  const int Ka = shn[0], Kb = shn[1], Kc = shn[2], Kd = shn[3];
  const bool ok = Ka >= 1 && Ka <= kmax && Kb >= 1 && Kb <= kmax && Kc >= 1 && Kc <= kmax && Kd >= 1 && Kd <= kmax;
  if (!ok || (!all && (i0 >= Ka || j0 >= Kb))) {
    __syncthreads();
    return;
  }
  const int ij0 = all ? 0 : i0 * Kb + j0;
  const int ij1 = all ? Ka * Kb : ij0 + 1;
  jengine_body<LAY, NPT>(cp, s, wb, boys_tab, rent, Ka, Kb, Kc, Kd, ij0, ij1, dket, ds,
                         outJ + (all ? 0 : (int64_t)ij0 * jstride), tid, wave, lane);
}

// Batch form: one workgroup per (quartet q0 + blockIdx.x / kmax^2, bra
// primitive pair (i, j) = divmod(blockIdx.x % kmax^2, kmax)); its J^ij goes to
// part + ((blockIdx.x / kmax^2) * kmax^2 + i * Kb + j) * nab.
template <int LAY, int NPT>
__global__ __launch_bounds__(kThreads, 1) void eri4_coulomb_kernel(
    const ClassParams cp, const double* __restrict__ boys_tab, const uint2* __restrict__ rtab,
    const double* __restrict__ centers, const double* __restrict__ exps, const double* __restrict__ coefs,
    const int32_t* __restrict__ nprim, double* __restrict__ part, int64_t q0, const double* __restrict__ dket,
    int64_t ds) {
  extern __shared__ __align__(16) unsigned char lds[];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t kk2 = (int64_t)cp.kmax * cp.kmax;
  const int64_t iq = blockIdx.x / kk2;
  const int slot = (int)(blockIdx.x - iq * kk2);
  const int i = slot / cp.kmax, j = slot - (slot / cp.kmax) * cp.kmax;
  jengine_quartet<LAY, NPT, false>(cp, lds, boys_tab, rtab + cp.rtab_off, centers, exps, coefs, nprim, q0 + iq,
                                   nullptr, nullptr, nullptr, 0, i, j, false, dket + iq * kk2 * ds, ds,
                                   part + iq * kk2 * cp.nab, cp.nab, tid, wave, lane);
}

// J of quartet q0 + blockIdx.x: the sum over its bra primitive pairs s = 0 ..
// Ka*Kb-1, in that order, of part[(blockIdx.x * kmax^2 + s) * nab ..]; NaN for
// a quartet whose contraction lengths are out of range.
__global__ void coulomb_pairsum_kernel(const ClassParams cp, const int32_t* __restrict__ nprim,
                                       const double* __restrict__ part, double* __restrict__ out, int64_t q0) {
  const int64_t iq = blockIdx.x, q = q0 + iq;
  const int kmax = cp.kmax;
  const int Ka = nprim[q * 4], Kb = nprim[q * 4 + 1], Kc = nprim[q * 4 + 2], Kd = nprim[q * 4 + 3];
  const bool ok = Ka >= 1 && Ka <= kmax && Kb >= 1 && Kb <= kmax && Kc >= 1 && Kc <= kmax && Kd >= 1 && Kd <= kmax;
  const int64_t kk2 = (int64_t)kmax * kmax;
  const double* p = part + iq * kk2 * cp.nab;
  for (int ab = threadIdx.x; ab < cp.nab; ab += blockDim.x) {
    double a = ok ? 0.0 : __builtin_nan("");
    if (ok)
      for (int s = 0; s < Ka * Kb; ++s) a += p[(int64_t)s * cp.nab + ab];
    out[q * cp.nab + ab] = a;
  }
}

template <int LAY, int NPT>
hipError_t coulomb_launch_t(const ClassParams& p, dim3 grid, hipStream_t s, const Tables& t, const double* centers,
                            const double* exps, const double* coefs, const int32_t* nprim, double* part, int64_t q0,
                            const double* dket, int64_t ds) {
  hipLaunchKernelGGL((eri4_coulomb_kernel<LAY, NPT>), grid, dim3(kThreads), p.lds_bytes, s, p, t.boys, t.rtab,
                     centers, exps, coefs, nprim, part, q0, dket, ds);
  return hipGetLastError();
}

// Persistent kernel of a Coulomb pair-list plan: work items are whole quartets
// (largest first); each sums J over all its bra primitive pairs with the dket
// of its ket entry (dket + dkoff[q % nket]) and writes it to jpart + qoff[q].
__global__ __launch_bounds__(kThreads, 1) void eri4_plan_coulomb_kernel(
    const ClassParams* __restrict__ classes, const int2* __restrict__ items, int nitems,
    const int64_t* __restrict__ qoff, const int32_t* __restrict__ nprim, int* __restrict__ counter,
    const double* __restrict__ boys_tab, const uint2* __restrict__ rtab, const double* __restrict__ centers,
    const double* __restrict__ exps, const double* __restrict__ coefs, double* __restrict__ jpart,
    const double* __restrict__ kcenters, const double* __restrict__ kexps, const double* __restrict__ kcoefs,
    int64_t nket, const int64_t* __restrict__ dkoff, const double* __restrict__ dket) {
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
    const uint2* rt_L = rtab + cp.rtab_off;
    const int64_t ik = q - (q / nket) * nket;
    const double* dk = dket + dkoff[ik];
    const int64_t ds = 16 * (int64_t)cp.nqb;
#define T(LAY, NPT)                                                                                                \
  jengine_quartet<LAY, NPT, true>(cp, lds, boys_tab, rt_L, centers, exps, coefs, nprim, q, kcenters, kexps, kcoefs, \
                                  nket, 0, 0, true, dk, ds, jpart + qoff[q], 0, tid, wave, lane)
    const bool two = cp.np > kThreads;
    if (cp.lay == kLaySlab) {
      if (two) T(kLaySlab, 2); else T(kLaySlab, 1);
    } else if (cp.lay == kLayBox2) {
      if (two) T(kLayBox2, 2); else T(kLayBox2, 1);
    } else {
      if (two) T(kLayBox, 2); else T(kLayBox, 1);
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
                             kMaxLdsBytes - 64);
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
  const void* k[6] = {(const void*)eri4_coulomb_kernel<kLayBox, 1>,  (const void*)eri4_coulomb_kernel<kLayBox, 2>,
                      (const void*)eri4_coulomb_kernel<kLaySlab, 1>, (const void*)eri4_coulomb_kernel<kLaySlab, 2>,
                      (const void*)eri4_coulomb_kernel<kLayBox2, 1>, (const void*)eri4_coulomb_kernel<kLayBox2, 2>};
  for (const void* f : k) {
    const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLdsBytes);
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

// J of quartets q0..q0+nq-1: the J^ij of every bra primitive pair into part
// (kmax^2 * nab doubles per quartet), then their sum per quartet into out.
hipError_t coulomb_launch(const ClassParams& p, int64_t nq, hipStream_t s, const Tables& t, const double* centers,
                          const double* exps, const double* coefs, const int32_t* nprim, double* part, double* out,
                          int64_t q0, const double* dket, int64_t ds) {
  const dim3 grid((unsigned)(nq * p.kmax * p.kmax));
  const bool two = p.np > kThreads;
  hipError_t e;
#define L(LAY, NPT) coulomb_launch_t<LAY, NPT>(p, grid, s, t, centers, exps, coefs, nprim, part, q0, dket, ds)
  switch (p.lay) {
    case kLaySlab:
      e = two ? L(kLaySlab, 2) : L(kLaySlab, 1);
      break;
    case kLayBox2:
      e = two ? L(kLayBox2, 2) : L(kLayBox2, 1);
      break;
    default:
      e = two ? L(kLayBox, 2) : L(kLayBox, 1);
  }
#undef L
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(coulomb_pairsum_kernel, dim3((unsigned)nq), dim3(256), 0, s, p, nprim, part, out, q0);
  return hipGetLastError();
}

}  // namespace eri4
