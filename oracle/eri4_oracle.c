/*
 * eri4_oracle.c -- reference CPU evaluation of 4-center Coulomb integrals (ab|cd)
 * over contracted Cartesian Gaussian shells.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this code.  The product path (the HIP
 * library) never calls it and shares no code, header or table with it.
 *
 * Two independent schemes are implemented, both plain and unoptimised:
 *
 *   oracle_eri_md4  the McMurchie-Davidson scheme exactly as the paper states it
 *                   (Sec. 2): Hermite expansion coefficients E by the two
 *                   recursions following eq. (cart2herm-2), the auxiliary
 *                   integrals [0]^(m) from the Boys function, the recursion of
 *                   eq. (md1), the sign relation of eq. (pq), and the two
 *                   Hermite-to-Cartesian transforms of eqs. (ab_to_hermite) and
 *                   (cd_to_hermite), summed over primitives.
 *
 *   oracle_eri_os   the Obara-Saika vertical recurrence followed by the
 *                   Head-Gordon-Pople horizontal recurrence (the scheme the paper
 *                   uses as its CPU reference, Sec. 1 and Sec. 4).  Its formulas
 *                   come from those original papers, not from this paper; it is a
 *                   second, independent recurrence used to pin the first.
 *
 * Readings of points the paper leaves open (all documented with the design):
 *   - Gaussian product prefactor: exp(-za*zb/zp |A-B|^2) for the bra and likewise
 *     for the ket multiply the primitive integral; the paper's E base value
 *     (E)^0_00 = 1 and its [0]^(m) omit it.
 *   - Hermite Gaussians are derivatives with respect to the centre coordinate,
 *     which is the convention under which the paper's E recursions and the sign
 *     (-1)^{l_q} of eq. (pq) hold together.
 *   - E^t_{ab} = 0 for t < 0 or t > a+b.
 *   - Cartesian components of a shell are ordered ax = l..0, then ay = l-ax..0.
 *   - Coefficients multiply unnormalised primitives x^ax y^ay z^az exp(-z r^2).
 *
 * Floating point: FP64, except the Boys function which is evaluated in
 * __float128 and rounded once to double.  Build with -O2 -ffp-contract=off.
 */
#include <math.h>
#include <quadmath.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_LMAX 8

int oracle_ncart(int l) { return (l < 0) ? -1 : (l + 1) * (l + 2) / 2; }

/* Cartesian components of shell l in the order ax = l..0, ay = l-ax..0. */
static void cart_list(int l, int q[][3]) {
  int i = 0;
  for (int ax = l; ax >= 0; --ax)
    for (int ay = l - ax; ay >= 0; --ay) {
      q[i][0] = ax;
      q[i][1] = ay;
      q[i][2] = l - ax - ay;
      ++i;
    }
}

/* ------------------------------------------------------------------------ */
/* Boys function, eq. (boys): F_m(x) = int_0^1 y^{2m} exp(-x y^2) dy.         */
/* Small x: the power series of the integrand's exponential integrated term   */
/* by term after one integration by parts,                                    */
/*   F_M(x) = exp(-x) sum_k (2x)^k / ((2M+1)(2M+3)...(2M+2k+1)),              */
/* evaluated at M = mmax (all terms positive), then the downward relation     */
/*   F_m(x) = (2x F_{m+1}(x) + exp(-x)) / (2m+1),                             */
/* which follows from integrating eq. (boys) by parts.  Large x: F_0 from the */
/* error function, F_0(x) = sqrt(pi/x) erf(sqrt x) / 2, and the same relation */
/* used upward (stable while 2m+1 < 2x).  All in __float128.                  */
/* ------------------------------------------------------------------------ */
void oracle_boys(int mmax, double T, double* F) {
  __float128 x = (__float128)T;
  const double T_SWITCH = 50.0;
  if (mmax < 0) return;
  if (T < T_SWITCH) {
    __float128 ex = expq(-x);
    __float128 term = 1.0Q / (2 * mmax + 1);
    __float128 sum = term;
    for (int k = 1; k < 100000; ++k) {
      term *= 2 * x / (2 * mmax + 2 * k + 1);
      sum += term;
      if (term < sum * 1e-36Q) break;
    }
    __float128 f = ex * sum;
    F[mmax] = (double)f;
    for (int m = mmax - 1; m >= 0; --m) {
      f = (2 * x * f + ex) / (2 * m + 1);
      F[m] = (double)f;
    }
  } else {
    __float128 ex = expq(-x);
    __float128 f = 0.5Q * sqrtq(M_PIq / x) * erfq(sqrtq(x));
    F[0] = (double)f;
    for (int m = 0; m < mmax; ++m) {
      f = ((2 * m + 1) * f - ex) / (2 * x);
      F[m + 1] = (double)f;
    }
  }
}

/* ------------------------------------------------------------------------ */
/* McMurchie-Davidson pieces, Sec. 2.                                         */
/* ------------------------------------------------------------------------ */

/* One Cartesian axis of the Hermite expansion of a primitive product,
 * eq. (cart2herm-2): E(a,b,t) for 0<=a<=la, 0<=b<=lb, 0<=t<=la+lb, using the
 * two recursions stated right after it, started from E(0,0,0) = 1.
 * Layout E[(a*(lb+1)+b)*(la+lb+1)+t]; entries with t > a+b stay zero. */
static void md_etab_axis(int la, int lb, double zp, double PA, double PB, double* E) {
  const int nt = la + lb + 1;
#define EIX(a, b, t) (((a) * (lb + 1) + (b)) * nt + (t))
  memset(E, 0, sizeof(double) * (size_t)(la + 1) * (lb + 1) * nt);
  const double h = 1.0 / (2.0 * zp);
  E[EIX(0, 0, 0)] = 1.0;
  /* raise a with b = 0 */
  for (int a = 0; a < la; ++a)
    for (int t = 0; t <= a + 1; ++t) {
      double v = 0.0;
      if (t >= 1) v += h * E[EIX(a, 0, t - 1)];
      if (t <= a) v += PA * E[EIX(a, 0, t)];
      if (t + 1 <= a) v += (t + 1) * E[EIX(a, 0, t + 1)];
      E[EIX(a + 1, 0, t)] = v;
    }
  /* raise b for every a */
  for (int a = 0; a <= la; ++a)
    for (int b = 0; b < lb; ++b)
      for (int t = 0; t <= a + b + 1; ++t) {
        double v = 0.0;
        if (t >= 1) v += h * E[EIX(a, b, t - 1)];
        if (t <= a + b) v += PB * E[EIX(a, b, t)];
        if (t + 1 <= a + b) v += (t + 1) * E[EIX(a, b, t + 1)];
        E[EIX(a, b + 1, t)] = v;
      }
#undef EIX
}

/* Public: the three axes for one primitive pair, E[axis][a][b][t]. */
void oracle_md4_etab(int la, int lb, double za, double zb, const double* A, const double* B,
                     double* E) {
  const double zp = za + zb;
  const size_t n = (size_t)(la + 1) * (lb + 1) * (la + lb + 1);
  for (int i = 0; i < 3; ++i) {
    const double P = (za * A[i] + zb * B[i]) / zp;
    md_etab_axis(la, lb, zp, P - A[i], P - B[i], E + i * n);
  }
}

/* Auxiliary integrals [r]^(m) (Sec. 2): [0]^(m) = (-2 rho)^m 2 pi^{5/2} /
 * (zp zq sqrt(zp+zq)) F_m(rho |P-Q|^2), then eq. (md1) raising r one unit at a
 * time.  Stored as a plain 4-d array R[m][t][u][v], each index in 0..L.
 * The direction raised is the first of x, y, z with a non-zero index. */
static void md_rtuv_all(int L, double zp, double zq, const double* P, const double* Q,
                        double* R) {
  const int n1 = L + 1;
#define RIX(m, t, u, v) ((((size_t)(m) * n1 + (t)) * n1 + (u)) * n1 + (v))
  const double rho = zp * zq / (zp + zq);
  const double X[3] = {P[0] - Q[0], P[1] - Q[1], P[2] - Q[2]};
  const double T = rho * (X[0] * X[0] + X[1] * X[1] + X[2] * X[2]);
  double F[4 * ORACLE_LMAX + 2];
  oracle_boys(L, T, F);
  const double pref = 2.0 * pow(M_PI, 2.5) / (zp * zq * sqrt(zp + zq));
  double pw = 1.0;
  for (int m = 0; m <= L; ++m) {
    R[RIX(m, 0, 0, 0)] = pw * pref * F[m];
    pw *= -2.0 * rho;
  }
  for (int n = 1; n <= L; ++n)
    for (int t = 0; t <= n; ++t)
      for (int u = 0; u <= n - t; ++u) {
        const int v = n - t - u;
        for (int m = 0; m <= L - n; ++m) {
          double val;
          if (t > 0) {
            val = X[0] * R[RIX(m + 1, t - 1, u, v)];
            if (t > 1) val += (t - 1) * R[RIX(m + 1, t - 2, u, v)];
          } else if (u > 0) {
            val = X[1] * R[RIX(m + 1, t, u - 1, v)];
            if (u > 1) val += (u - 1) * R[RIX(m + 1, t, u - 2, v)];
          } else {
            val = X[2] * R[RIX(m + 1, t, u, v - 1)];
            if (v > 1) val += (v - 1) * R[RIX(m + 1, t, u, v - 2)];
          }
          R[RIX(m, t, u, v)] = val;
        }
      }
#undef RIX
}

/* Public: R^(0)[t][u][v] ((L+1)^3 dense, entries with t+u+v > L set to zero) for
 * one primitive quartet, without contraction coefficients or Gaussian product
 * prefactors. */
void oracle_md4_rtuv(int L, double zp, double zq, const double* P, const double* Q, double* R0) {
  const int n1 = L + 1;
  double* R = (double*)calloc((size_t)n1 * n1 * n1 * n1, sizeof(double));
  md_rtuv_all(L, zp, zq, P, Q, R);
  for (int t = 0; t <= L; ++t)
    for (int u = 0; u <= L; ++u)
      for (int v = 0; v <= L; ++v)
        R0[((size_t)t * n1 + u) * n1 + v] = (t + u + v <= L) ? R[((size_t)t * n1 + u) * n1 + v] : 0.0;
  free(R);
}

/* One primitive quartet, accumulated into out[ab][cd] with weight w:
 *   [ab|q] = sum_p E_ab^p [p|q]            eq. (ab_to_hermite)
 *   [ab|cd] = sum_q E_cd^q [ab|q]          eq. (cd_to_hermite)
 *   [p|q] = (-1)^{|q|} [p+q]^(0)           eq. (pq)
 * with the sums over p (and q) running over p_i <= a_i + b_i as in
 * eq. (cart2herm-2). */
static void md4_primitive(int la, int lb, int lc, int ld, const double* A, const double* B,
                          const double* C, const double* D, double za, double zb, double zc,
                          double zd, double w, double* out) {
  const int Lb = la + lb, Lk = lc + ld, L = Lb + Lk;
  const int na = oracle_ncart(la), nb = oracle_ncart(lb), nc = oracle_ncart(lc), nd = oracle_ncart(ld);
  int ca[45][3], cb[45][3], cc[45][3], cd[45][3];
  cart_list(la, ca);
  cart_list(lb, cb);
  cart_list(lc, cc);
  cart_list(ld, cd);

  const double zp = za + zb, zq = zc + zd;
  double P[3], Q[3], AB2 = 0, CD2 = 0;
  for (int i = 0; i < 3; ++i) {
    P[i] = (za * A[i] + zb * B[i]) / zp;
    Q[i] = (zc * C[i] + zd * D[i]) / zq;
    AB2 += (A[i] - B[i]) * (A[i] - B[i]);
    CD2 += (C[i] - D[i]) * (C[i] - D[i]);
  }
  /* Gaussian product prefactors (reading of the missing K_AB, K_CD). */
  const double Kab = exp(-za * zb / zp * AB2), Kcd = exp(-zc * zd / zq * CD2);
  const double scale = w * Kab * Kcd;

  const size_t nEb = (size_t)(la + 1) * (lb + 1) * (Lb + 1);
  const size_t nEk = (size_t)(lc + 1) * (ld + 1) * (Lk + 1);
  double* Eb = (double*)malloc(sizeof(double) * 3 * nEb);
  double* Ek = (double*)malloc(sizeof(double) * 3 * nEk);
  oracle_md4_etab(la, lb, za, zb, A, B, Eb);
  oracle_md4_etab(lc, ld, zc, zd, C, D, Ek);
#define EB(i, a, b, t) Eb[(i) * nEb + ((size_t)(a) * (lb + 1) + (b)) * (Lb + 1) + (t)]
#define EK(i, c, d, t) Ek[(i) * nEk + ((size_t)(c) * (ld + 1) + (d)) * (Lk + 1) + (t)]

  const int n1 = L + 1;
  double* R = (double*)calloc((size_t)n1 * n1 * n1 * n1, sizeof(double));
  md_rtuv_all(L, zp, zq, P, Q, R);
#define R0(t, u, v) R[((size_t)(t) * n1 + (u)) * n1 + (v)] /* m = 0 slice */

  /* bra transform into Xq[ab][tq][uq][vq] (dense (Lk+1)^3 per ab) */
  const int k1 = Lk + 1;
  const size_t nq3 = (size_t)k1 * k1 * k1;
  double* Xq = (double*)calloc((size_t)na * nb * nq3, sizeof(double));
  for (int ia = 0; ia < na; ++ia)
    for (int ib = 0; ib < nb; ++ib) {
      const int* a = ca[ia];
      const int* b = cb[ib];
      double* x = Xq + ((size_t)ia * nb + ib) * nq3;
      for (int tq = 0; tq <= Lk; ++tq)
        for (int uq = 0; uq <= Lk - tq; ++uq)
          for (int vq = 0; vq <= Lk - tq - uq; ++vq) {
            const double sgn = ((tq + uq + vq) & 1) ? -1.0 : 1.0;
            double s = 0.0;
            for (int tp = 0; tp <= a[0] + b[0]; ++tp)
              for (int up = 0; up <= a[1] + b[1]; ++up)
                for (int vp = 0; vp <= a[2] + b[2]; ++vp)
                  s += EB(0, a[0], b[0], tp) * EB(1, a[1], b[1], up) * EB(2, a[2], b[2], vp) *
                       sgn * R0(tp + tq, up + uq, vp + vq);
            x[((size_t)tq * k1 + uq) * k1 + vq] = s;
          }
    }
  /* ket transform */
  for (int iab = 0; iab < na * nb; ++iab) {
    const double* x = Xq + (size_t)iab * nq3;
    for (int ic = 0; ic < nc; ++ic)
      for (int id = 0; id < nd; ++id) {
        const int* c = cc[ic];
        const int* d = cd[id];
        double s = 0.0;
        for (int tq = 0; tq <= c[0] + d[0]; ++tq)
          for (int uq = 0; uq <= c[1] + d[1]; ++uq)
            for (int vq = 0; vq <= c[2] + d[2]; ++vq)
              s += EK(0, c[0], d[0], tq) * EK(1, c[1], d[1], uq) * EK(2, c[2], d[2], vq) *
                   x[((size_t)tq * k1 + uq) * k1 + vq];
        out[(size_t)iab * nc * nd + (size_t)ic * nd + id] += scale * s;
      }
  }
#undef EB
#undef EK
#undef R0
  free(Xq);
  free(R);
  free(Eb);
  free(Ek);
}

/* ------------------------------------------------------------------------ */
/* Obara-Saika vertical recurrence + Head-Gordon-Pople horizontal recurrence. */
/* Formulas from Obara & Saika (1986) and Head-Gordon & Pople (1988); this    */
/* paper only names the scheme.                                               */
/* ------------------------------------------------------------------------ */

/* compact ordinal of all triples with t+u+v <= n, looked up through a dense cube */
typedef struct {
  int n, count;
  int* ord; /* (n+1)^3, -1 where t+u+v > n */
  int (*tri)[3];
} triples_t;

static void triples_init(triples_t* s, int n) {
  const int n1 = n + 1;
  s->n = n;
  s->ord = (int*)malloc(sizeof(int) * n1 * n1 * n1);
  s->tri = malloc(sizeof(int[3]) * (size_t)n1 * n1 * n1);
  int c = 0;
  for (int i = 0; i < n1 * n1 * n1; ++i) s->ord[i] = -1;
  for (int l = 0; l <= n; ++l) /* grouped by total */
    for (int x = l; x >= 0; --x)
      for (int y = l - x; y >= 0; --y) {
        const int z = l - x - y;
        s->ord[(x * n1 + y) * n1 + z] = c;
        s->tri[c][0] = x;
        s->tri[c][1] = y;
        s->tri[c][2] = z;
        ++c;
      }
  s->count = c;
}
static void triples_free(triples_t* s) {
  free(s->ord);
  free(s->tri);
}
static int tord(const triples_t* s, int x, int y, int z) {
  if (x < 0 || y < 0 || z < 0 || x + y + z > s->n) return -1;
  return s->ord[(x * (s->n + 1) + y) * (s->n + 1) + z];
}

/* Primitive [e0|f0]^(0) for all |e| <= Le, |f| <= Lf by the Obara-Saika VRR,
 * accumulated with weight w into I[e][f] (compact ordinals). */
static void os_vrr_primitive(const triples_t* te, const triples_t* tf, const double* A,
                             const double* B, const double* C, const double* D, double za,
                             double zb, double zc, double zd, double w, double* I) {
  const int Le = te->n, Lf = tf->n, L = Le + Lf, M = L + 1;
  const int ne = te->count, nf = tf->count;
  const double p = za + zb, q = zc + zd, rho = p * q / (p + q);
  double P[3], Q[3], W[3], AB2 = 0, CD2 = 0, PQ2 = 0;
  for (int i = 0; i < 3; ++i) {
    P[i] = (za * A[i] + zb * B[i]) / p;
    Q[i] = (zc * C[i] + zd * D[i]) / q;
    W[i] = (p * P[i] + q * Q[i]) / (p + q);
    AB2 += (A[i] - B[i]) * (A[i] - B[i]);
    CD2 += (C[i] - D[i]) * (C[i] - D[i]);
    PQ2 += (P[i] - Q[i]) * (P[i] - Q[i]);
  }
  double F[4 * ORACLE_LMAX + 2];
  oracle_boys(L, rho * PQ2, F);
  const double base = 2.0 * pow(M_PI, 2.5) / (p * q * sqrt(p + q)) * exp(-za * zb / p * AB2) *
                      exp(-zc * zd / q * CD2);
  double* V = (double*)calloc((size_t)ne * nf * M, sizeof(double));
#define V_(e, f, m) V[((size_t)(e) * nf + (f)) * M + (m)]
  for (int m = 0; m <= L; ++m) V_(0, 0, m) = base * F[m];
  /* electron 1 with f = 0 */
  for (int e = 1; e < ne; ++e) {
    const int* et = te->tri[e];
    const int le = et[0] + et[1] + et[2];
    const int i = (et[0] > 0) ? 0 : (et[1] > 0) ? 1 : 2;
    int e1t[3] = {et[0], et[1], et[2]};
    e1t[i] -= 1;
    const int e1 = tord(te, e1t[0], e1t[1], e1t[2]);
    int e2t[3] = {e1t[0], e1t[1], e1t[2]};
    e2t[i] -= 1;
    const int e2 = tord(te, e2t[0], e2t[1], e2t[2]);
    for (int m = 0; m <= L - le; ++m) {
      double v = (P[i] - A[i]) * V_(e1, 0, m) + (W[i] - P[i]) * V_(e1, 0, m + 1);
      if (e2 >= 0) v += e1t[i] / (2.0 * p) * (V_(e2, 0, m) - rho / p * V_(e2, 0, m + 1));
      V_(e, 0, m) = v;
    }
  }
  /* electron 2 */
  for (int f = 1; f < nf; ++f) {
    const int* ft = tf->tri[f];
    const int lf = ft[0] + ft[1] + ft[2];
    const int i = (ft[0] > 0) ? 0 : (ft[1] > 0) ? 1 : 2;
    int f1t[3] = {ft[0], ft[1], ft[2]};
    f1t[i] -= 1;
    const int f1 = tord(tf, f1t[0], f1t[1], f1t[2]);
    int f2t[3] = {f1t[0], f1t[1], f1t[2]};
    f2t[i] -= 1;
    const int f2 = tord(tf, f2t[0], f2t[1], f2t[2]);
    for (int e = 0; e < ne; ++e) {
      const int* et = te->tri[e];
      const int le = et[0] + et[1] + et[2];
      int eit[3] = {et[0], et[1], et[2]};
      eit[i] -= 1;
      const int ei = tord(te, eit[0], eit[1], eit[2]);
      for (int m = 0; m <= L - le - lf; ++m) {
        double v = (Q[i] - C[i]) * V_(e, f1, m) + (W[i] - Q[i]) * V_(e, f1, m + 1);
        if (f2 >= 0) v += f1t[i] / (2.0 * q) * (V_(e, f2, m) - rho / q * V_(e, f2, m + 1));
        if (ei >= 0) v += et[i] / (2.0 * (p + q)) * V_(ei, f1, m + 1);
        V_(e, f, m) = v;
      }
    }
  }
  for (int e = 0; e < ne; ++e)
    for (int f = 0; f < nf; ++f) I[(size_t)e * nf + f] += w * V_(e, f, 0);
#undef V_
  free(V);
}

/* Horizontal recurrence (a, b+1_i| = (a+1_i, b| + (A_i - B_i)(a, b| applied to the
 * contracted I[e][f] on one side.  in[e][k] (e over triples of Le = la+lb, k an
 * opaque trailing index of length nk) -> out[ia][ib][k] in shell component order. */
static void hgp_hrr(int la, int lb, const double* AB, const triples_t* te, const double* in,
                    int nk, double* out) {
  const int Le = la + lb;
  /* level tables: H_j[e][b] for |b| = j and la <= |e| <= Le - j, stored over all
   * triples of e and all triples of b (|b| <= lb) for plainness. */
  triples_t tb;
  triples_init(&tb, lb);
  const int ne = te->count, nbt = tb.count;
  double* H = (double*)calloc((size_t)ne * nbt * nk, sizeof(double));
#define H_(e, b, k) H[((size_t)(e) * nbt + (b)) * nk + (k)]
  for (int e = 0; e < ne; ++e)
    for (int k = 0; k < nk; ++k) H_(e, 0, k) = in[(size_t)e * nk + k];
  for (int b = 1; b < nbt; ++b) { /* triples grouped by total, so lower levels come first */
    const int* bt = tb.tri[b];
    const int lbb = bt[0] + bt[1] + bt[2];
    const int i = (bt[0] > 0) ? 0 : (bt[1] > 0) ? 1 : 2;
    int b1t[3] = {bt[0], bt[1], bt[2]};
    b1t[i] -= 1;
    const int b1 = tord(&tb, b1t[0], b1t[1], b1t[2]);
    for (int e = 0; e < ne; ++e) {
      const int* et = te->tri[e];
      const int le = et[0] + et[1] + et[2];
      if (le < la || le > Le - lbb) continue;
      int ept[3] = {et[0], et[1], et[2]};
      ept[i] += 1;
      const int ep = tord(te, ept[0], ept[1], ept[2]);
      for (int k = 0; k < nk; ++k) H_(e, b, k) = H_(ep, b1, k) + AB[i] * H_(e, b1, k);
    }
  }
  const int na = oracle_ncart(la), nb = oracle_ncart(lb);
  int ca[45][3], cb[45][3];
  cart_list(la, ca);
  cart_list(lb, cb);
  for (int ia = 0; ia < na; ++ia)
    for (int ib = 0; ib < nb; ++ib) {
      const int e = tord(te, ca[ia][0], ca[ia][1], ca[ia][2]);
      const int b = tord(&tb, cb[ib][0], cb[ib][1], cb[ib][2]);
      for (int k = 0; k < nk; ++k) out[((size_t)ia * nb + ib) * nk + k] = H_(e, b, k);
    }
#undef H_
  free(H);
  triples_free(&tb);
}

static void os_quartet(int la, int lb, int lc, int ld, const double* ctr, const double* ex,
                       const double* co, const int32_t* np, int kmax, double* out) {
  const double *A = ctr, *B = ctr + 3, *C = ctr + 6, *D = ctr + 9;
  triples_t te, tf;
  triples_init(&te, la + lb);
  triples_init(&tf, lc + ld);
  const int ne = te.count, nf = tf.count;
  double* I = (double*)calloc((size_t)ne * nf, sizeof(double));
  for (int i = 0; i < np[0]; ++i)
    for (int j = 0; j < np[1]; ++j)
      for (int k = 0; k < np[2]; ++k)
        for (int l = 0; l < np[3]; ++l) {
          const double w = co[0 * kmax + i] * co[1 * kmax + j] * co[2 * kmax + k] * co[3 * kmax + l];
          os_vrr_primitive(&te, &tf, A, B, C, D, ex[0 * kmax + i], ex[1 * kmax + j],
                           ex[2 * kmax + k], ex[3 * kmax + l], w, I);
        }
  const int nab = oracle_ncart(la) * oracle_ncart(lb);
  const int ncd = oracle_ncart(lc) * oracle_ncart(ld);
  double AB[3], CD[3];
  for (int i = 0; i < 3; ++i) {
    AB[i] = A[i] - B[i];
    CD[i] = C[i] - D[i];
  }
  /* bra HRR: I[e][f] -> J[ab][f] */
  double* J = (double*)calloc((size_t)nab * nf, sizeof(double));
  hgp_hrr(la, lb, AB, &te, I, nf, J);
  /* ket HRR on the transpose: Jt[f][ab] -> K[cd][ab] */
  double* Jt = (double*)malloc(sizeof(double) * (size_t)nf * nab);
  for (int x = 0; x < nab; ++x)
    for (int f = 0; f < nf; ++f) Jt[(size_t)f * nab + x] = J[(size_t)x * nf + f];
  double* K = (double*)calloc((size_t)ncd * nab, sizeof(double));
  hgp_hrr(lc, ld, CD, &tf, Jt, nab, K);
  for (int x = 0; x < nab; ++x)
    for (int y = 0; y < ncd; ++y) out[(size_t)x * ncd + y] = K[(size_t)y * nab + x];
  free(K);
  free(Jt);
  free(J);
  free(I);
  triples_free(&te);
  triples_free(&tf);
}

static void md4_quartet(int la, int lb, int lc, int ld, const double* ctr, const double* ex,
                        const double* co, const int32_t* np, int kmax, double* out) {
  const size_t n = (size_t)oracle_ncart(la) * oracle_ncart(lb) * oracle_ncart(lc) * oracle_ncart(ld);
  memset(out, 0, n * sizeof(double));
  for (int i = 0; i < np[0]; ++i)
    for (int j = 0; j < np[1]; ++j)
      for (int k = 0; k < np[2]; ++k)
        for (int l = 0; l < np[3]; ++l) {
          const double w = co[0 * kmax + i] * co[1 * kmax + j] * co[2 * kmax + k] * co[3 * kmax + l];
          md4_primitive(la, lb, lc, ld, ctr, ctr + 3, ctr + 6, ctr + 9, ex[0 * kmax + i],
                        ex[1 * kmax + j], ex[2 * kmax + k], ex[3 * kmax + l], w, out);
        }
}

static int check_args(int la, int lb, int lc, int ld, int64_t nq, const int32_t* np, int kmax) {
  if (la < 0 || lb < 0 || lc < 0 || ld < 0) return 1;
  if (la > ORACLE_LMAX || lb > ORACLE_LMAX || lc > ORACLE_LMAX || ld > ORACLE_LMAX) return 1;
  if (nq < 0 || kmax < 1) return 1;
  for (int64_t i = 0; i < 4 * nq; ++i)
    if (np[i] < 1 || np[i] > kmax) return 1;
  return 0;
}

typedef void (*quartet_fn)(int, int, int, int, const double*, const double*, const double*,
                           const int32_t*, int, double*);

static int run_batch(quartet_fn fn, int la, int lb, int lc, int ld, int64_t nq,
                     const double* centers, const double* exps, const double* coefs,
                     const int32_t* nprim, int kmax, double* out, int nthreads) {
  if (check_args(la, lb, lc, ld, nq, nprim, kmax)) return 1;
  const size_t n = (size_t)oracle_ncart(la) * oracle_ncart(lb) * oracle_ncart(lc) * oracle_ncart(ld);
#ifdef _OPENMP
  if (nthreads < 1) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
#endif
  for (int64_t q = 0; q < nq; ++q)
    fn(la, lb, lc, ld, centers + 12 * q, exps + 4 * kmax * q, coefs + 4 * kmax * q, nprim + 4 * q,
       kmax, out + n * q);
  (void)nthreads;
  return 0;
}

/* Batched entry points. Layouts: centers [nq][4][3], exps/coefs [nq][4][kmax],
 * nprim [nq][4], out [nq][Na][Nb][Nc][Nd], all host memory.  Returns 0, or 1 on
 * invalid arguments (nothing written). nthreads < 1 means all available. */
int oracle_eri_md4(int la, int lb, int lc, int ld, int64_t nq, const double* centers,
                   const double* exps, const double* coefs, const int32_t* nprim, int kmax,
                   double* out, int nthreads) {
  return run_batch(md4_quartet, la, lb, lc, ld, nq, centers, exps, coefs, nprim, kmax, out, nthreads);
}

int oracle_eri_os(int la, int lb, int lc, int ld, int64_t nq, const double* centers,
                  const double* exps, const double* coefs, const int32_t* nprim, int kmax,
                  double* out, int nthreads) {
  return run_batch(os_quartet, la, lb, lc, ld, nq, centers, exps, coefs, nprim, kmax, out, nthreads);
}

int oracle_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Quad-precision instance of the McMurchie-Davidson scheme (truth values).   */
/*                                                                            */
/* The same steps as md4_primitive above (Sec. 2: the E recursions after      */
/* eq. (cart2herm-2), [0]^(m) from eq. (boys), eq. (md1), eq. (pq), then       */
/* eqs. (ab_to_hermite) and (cd_to_hermite)), every quantity in __float128:   */
/* the inputs are converted exactly, the Boys function is kept in quad, and   */
/* only the final sums are rounded to double.  Its rounding error is ~1e-30   */
/* of the terms' size, so it measures the FP64 oracle's own error on the same */
/* inputs.  Slow (software arithmetic): for subsamples only.                  */
/* ------------------------------------------------------------------------ */

typedef __float128 quad;

static void boys_q(int mmax, quad x, quad* F) {
  if (mmax < 0) return;
  quad ex = expq(-x);
  if (x < 50) {
    quad term = 1.0Q / (2 * mmax + 1);
    quad sum = term;
    for (int k = 1; k < 100000; ++k) {
      term *= 2 * x / (2 * mmax + 2 * k + 1);
      sum += term;
      if (term < sum * 1e-36Q) break;
    }
    quad f = ex * sum;
    F[mmax] = f;
    for (int m = mmax - 1; m >= 0; --m) {
      f = (2 * x * f + ex) / (2 * m + 1);
      F[m] = f;
    }
  } else {
    quad f = 0.5Q * sqrtq(M_PIq / x) * erfq(sqrtq(x));
    F[0] = f;
    for (int m = 0; m < mmax; ++m) {
      f = ((2 * m + 1) * f - ex) / (2 * x);
      F[m + 1] = f;
    }
  }
}

static void md_etab_axis_q(int la, int lb, quad zp, quad PA, quad PB, quad* E) {
  const int nt = la + lb + 1;
#define EIX(a, b, t) (((a) * (lb + 1) + (b)) * nt + (t))
  for (int i = 0; i < (la + 1) * (lb + 1) * nt; ++i) E[i] = 0;
  const quad h = 1 / (2 * zp);
  E[EIX(0, 0, 0)] = 1;
  for (int a = 0; a < la; ++a)
    for (int t = 0; t <= a + 1; ++t) {
      quad v = 0;
      if (t >= 1) v += h * E[EIX(a, 0, t - 1)];
      if (t <= a) v += PA * E[EIX(a, 0, t)];
      if (t + 1 <= a) v += (t + 1) * E[EIX(a, 0, t + 1)];
      E[EIX(a + 1, 0, t)] = v;
    }
  for (int a = 0; a <= la; ++a)
    for (int b = 0; b < lb; ++b)
      for (int t = 0; t <= a + b + 1; ++t) {
        quad v = 0;
        if (t >= 1) v += h * E[EIX(a, b, t - 1)];
        if (t <= a + b) v += PB * E[EIX(a, b, t)];
        if (t + 1 <= a + b) v += (t + 1) * E[EIX(a, b, t + 1)];
        E[EIX(a, b + 1, t)] = v;
      }
#undef EIX
}

static void md_rtuv_all_q(int L, quad zp, quad zq, const quad* P, const quad* Q, quad* R) {
  const int n1 = L + 1;
#define RIX(m, t, u, v) ((((size_t)(m) * n1 + (t)) * n1 + (u)) * n1 + (v))
  const quad rho = zp * zq / (zp + zq);
  const quad X[3] = {P[0] - Q[0], P[1] - Q[1], P[2] - Q[2]};
  quad F[4 * ORACLE_LMAX + 2];
  boys_q(L, rho * (X[0] * X[0] + X[1] * X[1] + X[2] * X[2]), F);
  const quad pref = 2 * powq(M_PIq, 2.5Q) / (zp * zq * sqrtq(zp + zq));
  quad pw = 1;
  for (int m = 0; m <= L; ++m) {
    R[RIX(m, 0, 0, 0)] = pw * pref * F[m];
    pw *= -2 * rho;
  }
  for (int n = 1; n <= L; ++n)
    for (int t = 0; t <= n; ++t)
      for (int u = 0; u <= n - t; ++u) {
        const int v = n - t - u;
        for (int m = 0; m <= L - n; ++m) {
          quad val;
          if (t > 0) {
            val = X[0] * R[RIX(m + 1, t - 1, u, v)];
            if (t > 1) val += (t - 1) * R[RIX(m + 1, t - 2, u, v)];
          } else if (u > 0) {
            val = X[1] * R[RIX(m + 1, t, u - 1, v)];
            if (u > 1) val += (u - 1) * R[RIX(m + 1, t, u - 2, v)];
          } else {
            val = X[2] * R[RIX(m + 1, t, u, v - 1)];
            if (v > 1) val += (v - 1) * R[RIX(m + 1, t, u, v - 2)];
          }
          R[RIX(m, t, u, v)] = val;
        }
      }
#undef RIX
}

static void md4_primitive_q(int la, int lb, int lc, int ld, const double* A_, const double* B_, const double* C_,
                            const double* D_, double za_, double zb_, double zc_, double zd_, quad w, quad* out) {
  const int Lb = la + lb, Lk = lc + ld, L = Lb + Lk;
  const int na = oracle_ncart(la), nb = oracle_ncart(lb), nc = oracle_ncart(lc), nd = oracle_ncart(ld);
  int ca[45][3], cb[45][3], cc[45][3], cd[45][3];
  cart_list(la, ca);
  cart_list(lb, cb);
  cart_list(lc, cc);
  cart_list(ld, cd);
  const quad za = za_, zb = zb_, zc = zc_, zd = zd_;
  const quad zp = za + zb, zq = zc + zd;
  quad A[3], B[3], C[3], D[3], P[3], Q[3], AB2 = 0, CD2 = 0;
  for (int i = 0; i < 3; ++i) {
    A[i] = A_[i], B[i] = B_[i], C[i] = C_[i], D[i] = D_[i];
    P[i] = (za * A[i] + zb * B[i]) / zp;
    Q[i] = (zc * C[i] + zd * D[i]) / zq;
    AB2 += (A[i] - B[i]) * (A[i] - B[i]);
    CD2 += (C[i] - D[i]) * (C[i] - D[i]);
  }
  const quad scale = w * expq(-za * zb / zp * AB2) * expq(-zc * zd / zq * CD2);
  const size_t nEb = (size_t)(la + 1) * (lb + 1) * (Lb + 1);
  const size_t nEk = (size_t)(lc + 1) * (ld + 1) * (Lk + 1);
  quad* Eb = (quad*)malloc(sizeof(quad) * 3 * nEb);
  quad* Ek = (quad*)malloc(sizeof(quad) * 3 * nEk);
  for (int i = 0; i < 3; ++i) {
    md_etab_axis_q(la, lb, zp, P[i] - A[i], P[i] - B[i], Eb + i * nEb);
    md_etab_axis_q(lc, ld, zq, Q[i] - C[i], Q[i] - D[i], Ek + i * nEk);
  }
#define EB(i, a, b, t) Eb[(i) * nEb + ((size_t)(a) * (lb + 1) + (b)) * (Lb + 1) + (t)]
#define EK(i, c, d, t) Ek[(i) * nEk + ((size_t)(c) * (ld + 1) + (d)) * (Lk + 1) + (t)]
  const int n1 = L + 1;
  quad* R = (quad*)calloc((size_t)n1 * n1 * n1 * n1, sizeof(quad));
  md_rtuv_all_q(L, zp, zq, P, Q, R);
#define R0(t, u, v) R[((size_t)(t) * n1 + (u)) * n1 + (v)]
  const int k1 = Lk + 1;
  const size_t nq3 = (size_t)k1 * k1 * k1;
  quad* Xq = (quad*)calloc((size_t)na * nb * nq3, sizeof(quad));
  for (int ia = 0; ia < na; ++ia)
    for (int ib = 0; ib < nb; ++ib) {
      const int* a = ca[ia];
      const int* b = cb[ib];
      quad* x = Xq + ((size_t)ia * nb + ib) * nq3;
      for (int tq = 0; tq <= Lk; ++tq)
        for (int uq = 0; uq <= Lk - tq; ++uq)
          for (int vq = 0; vq <= Lk - tq - uq; ++vq) {
            const quad sgn = ((tq + uq + vq) & 1) ? -1 : 1;
            quad s = 0;
            for (int tp = 0; tp <= a[0] + b[0]; ++tp)
              for (int up = 0; up <= a[1] + b[1]; ++up)
                for (int vp = 0; vp <= a[2] + b[2]; ++vp)
                  s += EB(0, a[0], b[0], tp) * EB(1, a[1], b[1], up) * EB(2, a[2], b[2], vp) * sgn *
                       R0(tp + tq, up + uq, vp + vq);
            x[((size_t)tq * k1 + uq) * k1 + vq] = s;
          }
    }
  for (int iab = 0; iab < na * nb; ++iab) {
    const quad* x = Xq + (size_t)iab * nq3;
    for (int ic = 0; ic < nc; ++ic)
      for (int id = 0; id < nd; ++id) {
        const int* c = cc[ic];
        const int* d = cd[id];
        quad s = 0;
        for (int tq = 0; tq <= c[0] + d[0]; ++tq)
          for (int uq = 0; uq <= c[1] + d[1]; ++uq)
            for (int vq = 0; vq <= c[2] + d[2]; ++vq)
              s += EK(0, c[0], d[0], tq) * EK(1, c[1], d[1], uq) * EK(2, c[2], d[2], vq) *
                   x[((size_t)tq * k1 + uq) * k1 + vq];
        out[(size_t)iab * nc * nd + (size_t)ic * nd + id] += scale * s;
      }
  }
#undef EB
#undef EK
#undef R0
  free(Xq);
  free(R);
  free(Eb);
  free(Ek);
}

static void md4_quartet_q(int la, int lb, int lc, int ld, const double* ctr, const double* ex, const double* co,
                          const int32_t* np, int kmax, double* out) {
  const size_t n = (size_t)oracle_ncart(la) * oracle_ncart(lb) * oracle_ncart(lc) * oracle_ncart(ld);
  quad* acc = (quad*)calloc(n, sizeof(quad));
  for (int i = 0; i < np[0]; ++i)
    for (int j = 0; j < np[1]; ++j)
      for (int k = 0; k < np[2]; ++k)
        for (int l = 0; l < np[3]; ++l) {
          const quad w = (quad)co[0 * kmax + i] * co[1 * kmax + j] * co[2 * kmax + k] * co[3 * kmax + l];
          md4_primitive_q(la, lb, lc, ld, ctr, ctr + 3, ctr + 6, ctr + 9, ex[0 * kmax + i], ex[1 * kmax + j],
                          ex[2 * kmax + k], ex[3 * kmax + l], w, acc);
        }
  for (size_t i = 0; i < n; ++i) out[i] = (double)acc[i];
  free(acc);
}

/* As oracle_eri_md4, every step in __float128, the result rounded to double. */
int oracle_eri_md4_quad(int la, int lb, int lc, int ld, int64_t nq, const double* centers, const double* exps,
                        const double* coefs, const int32_t* nprim, int kmax, double* out, int nthreads) {
  return run_batch(md4_quartet_q, la, lb, lc, ld, nq, centers, exps, coefs, nprim, kmax, out, nthreads);
}
