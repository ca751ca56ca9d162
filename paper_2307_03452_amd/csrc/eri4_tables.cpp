// eri4_tables.cpp -- host-side generation of the constant tables liberi4 uploads
// to each device: the Boys-function Taylor grid, the Hermite recursion tables
// and the solid-harmonic coefficients.  Plain host C++, built into liberi4.so.
#include <cmath>
#include <vector>

#include "eri4_internal.h"

namespace eri4 {

// F_k(T) for k = 0..kmax at one T, in long double (64-bit mantissa).
// The Boys integral of eq. (boys) expands as
//   F_K(T) = exp(-T) sum_{j>=0} (2T)^j / ((2K+1)(2K+3)...(2K+2j+1)),
// a sum of positive terms; lower orders follow from
//   F_k(T) = (2T F_{k+1}(T) + exp(-T)) / (2k+1),
// which is stable in the downward direction.
static void boys_column(int kmax, long double T, long double* F) {
  const long double ex = expl(-T);
  long double term = 1.0L / (2 * kmax + 1);
  long double sum = term;
  for (int j = 1; j < 4000; ++j) {
    term *= 2.0L * T / (2 * kmax + 2 * j + 1);
    sum += term;
    if (term < sum * 1e-22L) break;
  }
  F[kmax] = ex * sum;
  for (int k = kmax - 1; k >= 0; --k) F[k] = (2.0L * T * F[k + 1] + ex) / (2 * k + 1);
}

void make_boys_table(std::vector<double>& tab) {
  tab.assign((size_t)(kBoysRows + 1) * kBoysCols, 0.0);
  {  // Gamma(m+1/2)/2 = (2m-1)!! sqrt(pi) / 2^(m+1)
    long double c = sqrtl(3.14159265358979323846264338327950288L) / 2.0L;
    for (int m = 0; m < kBoysCols; ++m) {
      tab[(size_t)kBoysAsymRow * kBoysCols + m] = (double)c;
      c *= (2.0L * m + 1.0L) / 2.0L;
    }
  }
  std::vector<long double> F(kBoysCols);
  for (int i = 0; i < kBoysRows; ++i) {
    const long double T = (long double)i * (long double)kBoysH;  // exact grid point
    boys_column(kBoysCols - 1, T, F.data());
    for (int k = 0; k < kBoysCols; ++k) tab[(size_t)i * kBoysCols + k] = (double)F[k];
  }
}

// Triples (t,u,v), t+u+v <= L, by total order; within one total order any
// order works because entries of one order only read lower orders.  Layout 0
// (box) comes first, then layout 1 (slab); start[layout*(kMaxL+1) + L] is the
// first entry (in uint32 pairs) of a table.
void make_rtabs(std::vector<uint32_t>& tab, std::vector<int>& start) {
  tab.clear();
  start.assign(2 * (kMaxL + 1), 0);
  for (int layout = 0; layout < 2; ++layout)
    for (int L = 0; L <= kMaxL; ++L) {
      start[layout * (kMaxL + 1) + L] = (int)(tab.size() / 2);
      const bool slab = layout == 1;
      for (int n = 0; n <= L; ++n)
        for (int t = n; t >= 0; --t)
          for (int u = n - t; u >= 0; --u) {
            const int v = n - t - u;
            const uint32_t off = (uint32_t)r_offset(slab, L, t, u, v);
            uint32_t dir = 0, ri = 0, o1 = 0, o2 = 0;
            if (n > 0) {
              int a[3] = {t, u, v};
              dir = v > 0 ? 2 : (u > 0 ? 1 : 0);
              ri = (uint32_t)a[dir];
              a[dir] -= 1;
              o1 = (uint32_t)r_offset(slab, L, a[0], a[1], a[2]);
              if (ri >= 2) {
                a[dir] -= 1;
                o2 = (uint32_t)r_offset(slab, L, a[0], a[1], a[2]);
              } else {
                o2 = o1;
              }
            }
            tab.push_back(off | (o1 << 16));
            tab.push_back(o2 | (dir << 16) | (ri << 18));
          }
    }
}

// Real solid harmonics in Cartesian monomials (the coefficient matrices that
// turn E into H, Sec. 2), from the closed-form expansion
//   S_lm = N_lm sum_{t,u,v} (-1)^(t+v-v_m) 4^-t C(l,t) C(l-t,|m|+t) C(t,u) C(|m|,2v)
//                          x^(2t+|m|-2(u+v)) y^(2(u+v)) z^(l-2t-|m|),
//   N_lm = sqrt(2 (l+|m|)! (l-|m|)! / 2^delta(m,0)) / (2^|m| l!),
// t = 0..(l-|m|)/2, u = 0..t, v = v_m, v_m+1, ... <= |m|/2 with v_m = 0 for
// m >= 0 and 1/2 for m < 0 (Helgaker, Jorgensen and Olsen, Sec. 6.4.2).  Rows
// m = -l..l; columns in the integrals' Cartesian order; unit-norm functions
// when the Cartesian components share the coefficient that normalises x^l.
// Every term before the final scaling by N_lm is an exact binary fraction.
void solid_dense(int l, double* C) {
  auto binom = [](int n, int k) {
    if (k < 0 || k > n) return 0.0;
    double r = 1.0;
    for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
    return r;
  };
  auto fact = [](int n) {
    double r = 1.0;
    for (int i = 2; i <= n; ++i) r *= i;
    return r;
  };
  const int nc = ncart(l);
  for (int i = 0; i < (2 * l + 1) * nc; ++i) C[i] = 0.0;
  for (int m = -l; m <= l; ++m) {
    const int am = m < 0 ? -m : m;
    double* row = C + (m + l) * nc;
    const int w0 = m < 0 ? 1 : 0;  // 2 v_m
    for (int t = 0; t <= (l - am) / 2; ++t)
      for (int u = 0; u <= t; ++u)
        for (int w = w0; w <= am; w += 2) {  // w = 2v
          const double sign = (((2 * t + w - w0) / 2) & 1) ? -1.0 : 1.0;
          const double c = sign * binom(l, t) * binom(l - t, am + t) * binom(t, u) * binom(am, w) / std::ldexp(1.0, 2 * t);
          const int py = 2 * u + w, px = 2 * t + am - py, pz = l - 2 * t - am;
          if (px < 0) continue;
          row[(l - px) * (l - px + 1) / 2 + pz] += c;
        }
    const double n = std::sqrt(2.0 * fact(l + am) * fact(l - am) / (m == 0 ? 2.0 : 1.0)) /
                     (std::ldexp(1.0, am) * fact(l));
    for (int k = 0; k < nc; ++k) row[k] *= n;
  }
}

// Sparse form for the device: entry (l, m + l) at ((l * kSolidRows) + m + l) *
// kSolidEntry doubles: [0] number of non-zero terms n, [1 + 2j] Cartesian index,
// [2 + 2j] coefficient, j < n.
void make_solid_table(std::vector<double>& tab) {
  tab.assign((kTableLMax + 1) * kSolidRows * kSolidEntry, 0.0);
  std::vector<double> C;
  for (int l = 0; l <= kTableLMax; ++l) {
    const int nc = ncart(l);
    C.assign((2 * l + 1) * nc, 0.0);
    solid_dense(l, C.data());
    for (int m = 0; m < 2 * l + 1; ++m) {
      double* e = tab.data() + (l * kSolidRows + m) * kSolidEntry;
      int n = 0;
      for (int k = 0; k < nc; ++k)
        if (C[m * nc + k] != 0.0) {
          e[1 + 2 * n] = k;
          e[2 + 2 * n] = C[m * nc + k];
          ++n;
        }
      e[0] = n;
    }
  }
}

}  // namespace eri4
