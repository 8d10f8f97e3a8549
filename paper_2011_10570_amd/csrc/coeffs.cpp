// Exact-rational RK coefficient tables for LTS stage conversion.
//
// eq. rk_schemes (Sec. 3.4): p-stage explicit RK, stage argument
// u + dt sum_q a_sq k_q, update u + dt sum_i b_i k_i.
// eq. rk_crrection (Sec. 3.6.2), read as K = C P_dt D: for u' = L u,
// k_i = sum_j C_ij dt^(j-1) L^j u with C_i1 = 1, C_i,j+1 = sum_m a_im C_mj.
// eqs. fc_1 / fc_2: stages of a record (step dt_n) seen from a receiver step dt_r
// starting Delta later are k~ = C P_r B_Delta P_n^-1 C^-1 K, B_Delta the Taylor
// shift (B)_jm = Delta^(m-j)/(m-j)!.  The receiver's stage state is
// Y_s = u(t_r) + dt_r sum_{q<s} a_sq k~_q with u(t_r) = U0 + sum_j Delta^j/j! D_j,
// i.e. Y_s = U0 + dt_r sum_i w^_si K_i in the variables delta = Delta/dt_r,
// rho = dt_n/dt_r.  Four (delta, rho) pairs occur on a ghost-reach-balanced mesh:
// (0,1), (0,1/2), (0,2), (1,2).
#include <cstdint>
#include <cstdlib>

#include "lts_impl.h"

namespace lts {

namespace {

struct Q {  // rational with 128-bit intermediates
  int64_t n = 0, d = 1;
  Q() = default;
  Q(int64_t a, int64_t b = 1) : n(a), d(b) { norm(); }
  static int64_t gcd(int64_t a, int64_t b) {
    a = a < 0 ? -a : a;
    b = b < 0 ? -b : b;
    while (b) {
      int64_t t = a % b;
      a = b;
      b = t;
    }
    return a ? a : 1;
  }
  void norm() {
    if (d < 0) { n = -n; d = -d; }
    int64_t g = gcd(n, d);
    n /= g;
    d /= g;
  }
  static Q make(__int128 a, __int128 b) {
    // reduce in 128 bits before narrowing
    __int128 x = a < 0 ? -a : a, y = b < 0 ? -b : b;
    while (y) { __int128 t = x % y; x = y; y = t; }
    if (x == 0) x = 1;
    a /= x; b /= x;
    if (b < 0) { a = -a; b = -b; }
    Q q;
    q.n = (int64_t)a;
    q.d = (int64_t)b;
    return q;
  }
  Q operator+(const Q& o) const { return make((__int128)n * o.d + (__int128)o.n * d, (__int128)d * o.d); }
  Q operator-(const Q& o) const { return make((__int128)n * o.d - (__int128)o.n * d, (__int128)d * o.d); }
  Q operator*(const Q& o) const { return make((__int128)n * o.n, (__int128)d * o.d); }
  Q operator/(const Q& o) const { return make((__int128)n * o.d, (__int128)d * o.n); }
  bool zero() const { return n == 0; }
  double f64() const { return (double)n / (double)d; }  // |n|, d < 2^53: one rounding
};

Q qpow(Q x, int e) {
  if (e < 0) { x = Q(1) / x; e = -e; }
  Q r(1);
  for (int i = 0; i < e; ++i) r = r * x;
  return r;
}

int64_t fact(int k) {
  int64_t r = 1;
  for (int i = 2; i <= k; ++i) r *= i;
  return r;
}

struct Tab {
  int p;
  Q a[4][4];
  Q b[4];
};

bool get_tab(int tableau, Tab& t) {
  for (auto& row : t.a)
    for (auto& x : row) x = Q(0);
  if (tableau == LTS_RK4) {
    t.p = 4;
    t.a[1][0] = Q(1, 2);
    t.a[2][1] = Q(1, 2);
    t.a[3][2] = Q(1);
    t.b[0] = Q(1, 6); t.b[1] = Q(1, 3); t.b[2] = Q(1, 3); t.b[3] = Q(1, 6);
    return true;
  }
  if (tableau == LTS_SSPRK3) {
    t.p = 3;
    t.a[1][0] = Q(1);
    t.a[2][0] = Q(1, 4);
    t.a[2][1] = Q(1, 4);
    t.b[0] = Q(1, 6); t.b[1] = Q(1, 6); t.b[2] = Q(2, 3);
    return true;
  }
  return false;
}

}  // namespace

int tableau_stages(int tableau) {
  Tab t;
  return get_tab(tableau, t) ? t.p : 0;
}

bool coefficient_tables(int tableau, double* w, double* a, double* b) {
  Tab t;
  if (!get_tab(tableau, t)) return false;
  const int p = t.p;
  Q C[4][4], Ci[4][4];
  for (int i = 0; i < p; ++i) C[i][0] = Q(1);
  for (int j = 1; j < p; ++j)
    for (int i = 0; i < p; ++i) {
      Q s(0);
      for (int m = 0; m < p; ++m) s = s + t.a[i][m] * C[m][j - 1];
      C[i][j] = s;
    }
  // C^-1 by forward substitution (C lower triangular)
  for (int col = 0; col < p; ++col)
    for (int i = 0; i < p; ++i) {
      Q acc(i == col ? 1 : 0);
      for (int k = 0; k < i; ++k) acc = acc - C[i][k] * Ci[k][col];
      if (C[i][i].zero()) return false;
      Ci[i][col] = acc / C[i][i];
    }
  const Q cases[4][2] = {{Q(0), Q(1)}, {Q(0), Q(1, 2)}, {Q(0), Q(2)}, {Q(1), Q(2)}};
  for (int c = 0; c < 4; ++c) {
    const Q delta = cases[c][0], rho = cases[c][1];
    // M = C diag(rho^(1-m)) shifted:  k~_q = sum_i T_qi K_i
    Q T[4][4];
    for (int q = 0; q < p; ++q)
      for (int j = 1; j <= p; ++j) {
        if (C[q][j - 1].zero()) continue;
        for (int m = j; m <= p; ++m) {
          const Q f = C[q][j - 1] * qpow(delta, m - j) / Q(fact(m - j)) * qpow(rho, 1 - m);
          for (int i = 0; i < p; ++i) T[q][i] = T[q][i] + f * Ci[m - 1][i];
        }
      }
    // Taylor part of u(t_r)
    Q tay[4];
    for (int j = 1; j <= p; ++j) {
      const Q f = qpow(delta, j) * qpow(rho, 1 - j) / Q(fact(j));
      for (int i = 0; i < p; ++i) tay[i] = tay[i] + f * Ci[j - 1][i];
    }
    for (int s = 0; s < p; ++s)
      for (int i = 0; i < p; ++i) {
        Q v = tay[i];
        for (int q = 0; q < s; ++q) v = v + t.a[s][q] * T[q][i];
        w[(c * p + s) * p + i] = v.f64();
      }
  }
  for (int s = 0; s < p; ++s)
    for (int i = 0; i < p; ++i) a[s * p + i] = t.a[s][i].f64();
  for (int i = 0; i < p; ++i) b[i] = t.b[i].f64();
  return true;
}

}  // namespace lts
