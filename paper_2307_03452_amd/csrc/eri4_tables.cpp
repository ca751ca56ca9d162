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
// order works because entries of one order only read lower orders.
void make_rtabs(std::vector<uint32_t>& tab, std::vector<int>& start) {
  tab.clear();
  start.assign(kMaxL + 2, 0);
  for (int L = 0; L <= kMaxL; ++L) {
    start[L] = (int)tab.size();
    const int S1 = box_s1(L), S2 = box_s2(L);
    for (int n = 0; n <= L; ++n)
      for (int t = n; t >= 0; --t)
        for (int u = n - t; u >= 0; --u) {
          const int v = n - t - u;
          const uint32_t off = (uint32_t)(t * S2 + u * S1 + v);
          uint32_t dir, ri;
          if (v > 0) {
            dir = 2;
            ri = v;
          } else if (u > 0) {
            dir = 1;
            ri = u;
          } else {
            dir = 0;
            ri = t;
          }
          tab.push_back(off | (dir << 16) | (ri << 18));
        }
  }
  start[kMaxL + 1] = (int)tab.size();
}

}  // namespace eri4
