// eri4_tables.cpp -- host-side generation of the constant tables liberi4 uploads
// to each device: the Boys-function Taylor grid and the Hermite recursion
// tables.  Plain host C++, built into liberi4.so.
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

}  // namespace eri4
