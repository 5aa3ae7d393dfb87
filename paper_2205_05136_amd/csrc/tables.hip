// Host-side 1D quadrature rules and Lagrange matrices for the device tables.
//
// GLL (p+1 points: +-1 and the roots of P_p') and Legendre-Gauss (roots of P_q)
// rules on [-1, 1] (Section 3, the SEM and SEM-NI quadrature), found by Newton
// iteration on the Legendre recurrence; Lagrange polynomials on the GLL nodes
// from their product definition.
#include <cmath>

#include "internal.hpp"

namespace mfsem {

namespace {
// Legendre P_n(x), P_n'(x) and P_n''(x) by recurrence and Legendre's equation.
void legendre(int n, long double x, long double* P, long double* dP) {
  long double p0 = 1.0L, p1 = x, d0 = 0.0L, d1 = 1.0L;
  if (n == 0) { *P = 1.0L; *dP = 0.0L; return; }
  for (int k = 1; k < n; ++k) {
    long double p2 = ((2 * k + 1) * x * p1 - k * p0) / (k + 1);
    long double d2 = d0 + (2 * k + 1) * p1;
    p0 = p1; p1 = p2; d0 = d1; d1 = d2;
  }
  *P = p1;
  *dP = d1;
}
}  // namespace

void gauss_rule(int q, std::vector<double>& x, std::vector<double>& w) {
  x.assign(q, 0.0);
  w.assign(q, 0.0);
  const long double pi = 3.14159265358979323846264338327950288L;
  for (int i = 0; i < q; ++i) {
    long double t = -std::cos(pi * (i + 0.75L) / (q + 0.5L));
    for (int it = 0; it < 100; ++it) {
      long double P, dP;
      legendre(q, t, &P, &dP);
      long double dt = P / dP;
      t -= dt;
      if (std::fabs((double)dt) < 1e-19) break;
    }
    long double P, dP;
    legendre(q, t, &P, &dP);
    x[i] = (double)t;
    w[i] = (double)(2.0L / ((1.0L - t * t) * dP * dP));
  }
}

void gll_rule(int p, std::vector<double>& x, std::vector<double>& w) {
  x.assign(p + 1, 0.0);
  w.assign(p + 1, 0.0);
  const long double pi = 3.14159265358979323846264338327950288L;
  for (int i = 0; i <= p; ++i) {
    long double t;
    if (i == 0) t = -1.0L;
    else if (i == p) t = 1.0L;
    else {
      t = -std::cos(pi * i / (long double)p);
      for (int it = 0; it < 100; ++it) {
        long double P, dP;
        legendre(p, t, &P, &dP);
        long double d2P = (2.0L * t * dP - p * (p + 1.0L) * P) / (1.0L - t * t);
        long double dt = dP / d2P;
        t -= dt;
        if (std::fabs((double)dt) < 1e-19) break;
      }
    }
    long double P, dP;
    legendre(p, t, &P, &dP);
    x[i] = (double)t;
    w[i] = (double)(2.0L / (p * (p + 1.0L) * P * P));
  }
}

void lagrange_matrices(const std::vector<double>& nodes, const std::vector<double>& x,
                       std::vector<double>* L, std::vector<double>* D) {
  const int P = (int)nodes.size(), Q = (int)x.size();
  if (L) L->assign((size_t)Q * P, 0.0);
  if (D) D->assign((size_t)Q * P, 0.0);
  for (int k = 0; k < Q; ++k) {
    for (int a = 0; a < P; ++a) {
      if (L) {
        long double v = 1.0L;
        for (int m = 0; m < P; ++m)
          if (m != a) v *= ((long double)x[k] - nodes[m]) / ((long double)nodes[a] - nodes[m]);
        (*L)[(size_t)k * P + a] = (double)v;
      }
      if (D) {
        long double s = 0.0L;
        for (int m = 0; m < P; ++m) {
          if (m == a) continue;
          long double t = 1.0L / ((long double)nodes[a] - nodes[m]);
          for (int n = 0; n < P; ++n)
            if (n != a && n != m) t *= ((long double)x[k] - nodes[n]) / ((long double)nodes[a] - nodes[n]);
          s += t;
        }
        (*D)[(size_t)k * P + a] = (double)s;
      }
    }
  }
}

TableOffsets table_offsets(int P, int Q, int Pm) {
  TableOffsets o;
  int at = 0;
  o.B = at;  at += Q * P;
  o.Db = at; at += Q * P;
  o.Dq = at; at += Q * Q;
  o.Bm = at; at += Q * Pm;
  o.Dm = at; at += Q * Pm;
  o.w = at;  at += Q;
  o.iw2 = at; at += Q;
  o.total = at;
  return o;
}

std::vector<double> build_tables(int p, int quad, int Q, int pm) {
  const int P = p + 1, Pm = pm + 1;
  std::vector<double> nodes, wn, pts, w, mnodes, wm;
  gll_rule(p, nodes, wn);
  gll_rule(pm, mnodes, wm);
  if (quad == MFSEM_GLL) { pts = nodes; w = wn; }
  else gauss_rule(Q, pts, w);
  TableOffsets o = table_offsets(P, Q, Pm);
  std::vector<double> t(o.total, 0.0), L, D;
  lagrange_matrices(nodes, pts, &L, &D);
  for (int i = 0; i < Q * P; ++i) { t[o.B + i] = L[i]; t[o.Db + i] = D[i]; }
  lagrange_matrices(pts, pts, nullptr, &D);
  for (int i = 0; i < Q * Q; ++i) t[o.Dq + i] = D[i];
  lagrange_matrices(mnodes, pts, &L, &D);
  for (int i = 0; i < Q * Pm; ++i) { t[o.Bm + i] = L[i]; t[o.Dm + i] = D[i]; }
  for (int k = 0; k < Q; ++k) t[o.w + k] = w[k];
  for (int k = 0; k < Q; ++k) t[o.iw2 + k] = 1.0 / (w[k] * w[k]);
  return t;
}

}  // namespace mfsem
