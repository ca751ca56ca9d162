// eri4_internal.h -- constants and parameter blocks shared by the host side and
// the gfx950 kernels of liberi4.  Not part of the public ABI.
#pragma once
#include <stdint.h>

namespace eri4 {

// Largest l per shell the index tables are sized for, and the largest total
// Hermite order L = la+lb+lc+ld (Boys orders 0..L).
constexpr int kTableLMax = 7;
constexpr int kMaxL = 4 * kTableLMax;  // 28

// Boys-function interpolation grid (Sec. 2, eq. (boys)): F_k(T_i) at
// T_i = i * kBoysH for i < kBoysRows, k < kBoysCols, used as a Taylor expansion
// F_m(T_i + d) = sum_j F_{m+j}(T_i) (-d)^j / j!, j <= kBoysJ.  kBoysH is a
// power of two so that T_i and d = T - T_i are exact.  Beyond kBoysTMax the
// asymptotic form F_m(T) = (2m-1)!! / 2^(m+1) sqrt(pi / T^(2m+1)) is used; its
// neglected part is below 1e-20 relative there for m <= kMaxL.
constexpr double kBoysH = 1.0 / 32.0;
constexpr double kBoysInvH = 32.0;
constexpr int kBoysJ = 7;
constexpr double kBoysTMax = 120.0;
constexpr int kBoysRows = 120 * 32 + 2;
constexpr int kBoysCols = kMaxL + kBoysJ + 2;  // 37
// Row kBoysRows of the uploaded table holds the asymptotic coefficients
// (2m-1)!! sqrt(pi) / 2^(m+1) = Gamma(m+1/2)/2, so F_m(T) = c_m / (T^m sqrt(T)).
constexpr int kBoysAsymRow = kBoysRows;

// Strides of the R box used for total order L: offset(t,u,v) = t*S2 + u*S1 + v.
// S1 is the even number >= L+1 so that entries of one total order, which sit
// S1-1 doubles apart, spread over the LDS banks; S2 = S1*(L+1).
__host__ __device__ constexpr int box_s1(int L) { return ((L + 1) & 1) ? L + 2 : L + 1; }
__host__ __device__ constexpr int box_s2(int L) { return box_s1(L) * (L + 1); }
// Odd row length >= n for the 1-d E tables (rows of one table read by the
// lanes of a wave then fall in different LDS banks).
__host__ __device__ constexpr int odd_row(int n) { return n | 1; }

// Pyramidal number: Hermite functions with total order <= n.
__host__ __device__ constexpr int nherm(int n) { return (n + 1) * (n + 2) * (n + 3) / 6; }
__host__ __device__ constexpr int ncart(int l) { return (l + 1) * (l + 2) / 2; }

// Two LDS layouts of the Hermite integrals [r] with t+u+v <= L:
//   box  (L+1)^3 cells:   offset = t*S2 + u*S1 + v,        S2 = S1*(L+1)
//   slab t-slabs of (L+1-t) rows: offset = slab_base(t) + u*S1 + v
// The box makes the index p+q of eq. (pq) an address sum; the slab needs one
// more term (slab_base of the summed t) but about half the space, which is
// what lets L = 26, 28 fit in LDS.
__host__ __device__ constexpr int slab_base(int t, int L, int S1) { return S1 * (t * (2 * L + 3 - t) / 2); }
__host__ __device__ constexpr int r_cells(bool slab, int L) {
  return slab ? box_s1(L) * (L + 1) * (L + 2) / 2 : (L + 1) * box_s2(L);
}
__host__ __device__ constexpr int r_offset(bool slab, int L, int t, int u, int v) {
  return (slab ? slab_base(t, L, box_s1(L)) : t * box_s2(L)) + u * box_s1(L) + v;
}

// Hermite recursion tables: for each layout (0 box, 1 slab) and each L in
// 0..kMaxL, the nherm(L) triples (t,u,v) with t+u+v <= L ordered by total
// order, each as two 32-bit words
//   x: offset of (t,u,v) | offset of (t,u,v) - 1_i << 16
//   y: offset of (t,u,v) - 2*1_i (or of -1_i when r_i < 2) | i << 16 | r_i << 18
// where i is the axis eq. (md1) raises to reach (t,u,v) (the last non-zero of
// t, u, v).  The first entry of each table is (0,0,0) with all fields 0.
constexpr int kRtabEntries = 35960;  // sum_{L=0}^{28} nherm(L), per layout

// Solid-harmonic coefficient table (make_solid_table): per (l, m) one entry of
// kSolidEntry doubles, the count and up to kSolidTerms (Cartesian index,
// coefficient) pairs; kSolidRows = 2 * kTableLMax + 1 rows per l.
constexpr int kSolidTerms = 16;
constexpr int kSolidEntry = 1 + 2 * kSolidTerms;
constexpr int kSolidRows = 2 * kTableLMax + 1;
// Hermite functions of one side (total order <= 2 * kTableLMax), padded to 4,
// and the doubles of that side's three 1-d E tables.
constexpr int kMaxHerm = (nherm(2 * kTableLMax) + 3) & ~3;
constexpr int kMaxEtab = 3 * ((kTableLMax + 1) * (kTableLMax + 1) + 1) * odd_row(2 * kTableLMax + 2);

// Units of 16 rows (bra) or columns (ket) of the H matrices of one pair-list
// entry: bra rows are padded to 64, a whole tile of any height.
__host__ __device__ constexpr int solid_pair_units(int l1, int l2, bool ket) {
  return ket ? ((2 * l1 + 1) * (2 * l2 + 1) + 15) / 16 : 4 * (((2 * l1 + 1) * (2 * l2 + 1) + 63) / 64);
}

// Dynamic LDS (bytes) of the H-matrix builder for shells l1, l2 with nk4
// Hermite indices: one chunk of P[2 l1 + 1][ncart(l2)][16], the three 1-d E
// tables, the Hermite index table.
__host__ __device__ constexpr int solid_h_lds(int l1, int l2, int nk4) {
  return (2 * l1 + 1) * ncart(l2) * 16 * 8 + 3 * ((l1 + 1) * (l2 + 1) + 1) * odd_row(l1 + l2 + 2) * 8 + nk4 * 8;
}

// Doubles of the Coulomb kernels' w buffer: the bra Hermite functions of up to
// 8 groups of waves (at most 512 in all), or 2 per thread when there are more
// than 512 (la + lb >= 13).
constexpr int kJw = 1024;

// LDS of one compute unit (gfx950).
constexpr int kMaxLdsBytes = 160 * 1024;

// One-wave kernel for classes whose shells all have l <= kSmallLMax
// (eri4_small.hip): its largest dynamic LDS.
constexpr int kSmallLMax = 3;
constexpr int kSmallLdsMax = 64 * 1024;

// One workgroup computes a tile of 16 or 32 bra rows (ab) of one quartet.
constexpr int kWaves = 8;
constexpr int kThreads = kWaves * 64;
constexpr int kRPerThread = (nherm(kMaxL) + kThreads - 1) / kThreads;  // 9, slab layout (L <= 28)
constexpr int kBoxLMax = 24;                                              // box layout only up to here
constexpr int kRPerBox = (nherm(kBoxLMax) + kThreads - 1) / kThreads;     // 6
constexpr int kMaxC1 = 6;  // first-transform column blocks per wave (L_ket <= 14)
// Layouts of the R recursion (template parameter of the kernels):
//   kLayBox   box, eq. (md1) in place (two barriers per level)
//   kLaySlab  slab, in place
//   kLayBox2  two boxes, levels alternate between them (one barrier per
//             level); [r]^(0) ends in the first.  Fits in LDS up to total
//             order kBox2LMax.
constexpr int kLayBox = 0, kLaySlab = 1, kLayBox2 = 2;
constexpr int kBox2LMax = 19;

// Everything the fused kernel needs to know about one class (la lb|lc ld).
struct ClassParams {
  int la, lb, lc, ld;
  int na, nb, nc, nd;
  int nab, ncd;
  int Lb, Lk, L;
  int np, nq;      // Hermite functions of the bra and the ket
  int np4, nq4;    // padded to a multiple of 4 (MFMA K step)
  int nqb;         // 16-wide column blocks of [ab|q]
  int ncdb;        // 16-wide column blocks of (ab|cd)
  int nrt;         // row tiles per quartet
  int S1, S2;      // strides of the R box: u -> S1, t -> S2 (box_s1, box_s2)
  int tbrow, tkrow;    // 1-d E table row lengths (Lb+2, Lk+2); last entry is 0
  int tbaxis, tkaxis;  // doubles per axis of the bra / ket tables (incl. zero row)
  int xs;              // row stride (doubles) of the [ab|q] tile in LDS
  int kmax;
  int rtab_off;        // first entry (uint2 units) of the recursion table for this layout and L
  int slab;            // R layout: 0 box, 1 slab
  int rb;              // 16-row blocks per tile (1, 2, or 4 with a box layout)
  int lay;             // kLayBox, kLaySlab or kLayBox2 (slab == (lay == kLaySlab))
  int o_box1;          // kLayBox2: byte offset of the second R box
  // LDS layout (byte offsets)
  int o_union;   // phase 1: R box then bra tables; phase 2: [ab|q] tile then ket tables
  int o_brae;    // bra tables (phase 1)
  int o_kete;    // ket tables (phase 2)
  int o_ptab, o_qtab, o_base, o_shell;
  int o_jw;      // Coulomb (J-engine) kernels: the Hermite-space J vector w
  int lds_bytes;
};

}  // namespace eri4
