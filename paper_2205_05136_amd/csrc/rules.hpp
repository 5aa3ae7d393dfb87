// Compile-time 1D rules and Lagrange matrices for the apply kernels.
//
// The same objects as the run-time tables (Section 3: GLL nodes carry the
// degree-p Lagrange basis; SEM-NI integrates on those nodes, SEM on q
// Legendre-Gauss points), evaluated by the compiler for each (P, Q) a kernel
// is instantiated for.  A kernel that contracts a lane's own pencil along the
// third direction needs every entry of a 1D matrix in every lane; as literal
// constants they become scalar moves and direct operands of the vector FMAs,
// with no loads, no waits on the counter that LDS reads share, and nothing to
// keep alive between phases.  Run-time tables loaded by lane-uniform scalar
// loads stay live across the kernel's barriers, and from 9 points in FP64
// they no longer fit the scalar registers and are parked in vector-register
// lanes (one v_readlane per 32 bits at every use).
//
// Points: Newton's method on the Legendre three-term recurrence (roots of P_q
// for Gauss; +-1 and the roots of P_p' for GLL), started from the Chebyshev-
// like guesses; the cosine of the guess is a Taylor sum, so everything here is
// a constant expression.  Lagrange values and derivatives from the product
// formula.  In double precision; the run-time tables agree to rounding.
#pragma once

namespace mfsem {
namespace rules {

template <int N>
struct Vec {
  double v[N];
};

constexpr double kPi = 3.14159265358979323846;

constexpr double absd(double x) { return x < 0 ? -x : x; }

// cos(x) for 0 <= x <= pi by its Taylor sum (only the Newton start needs it)
constexpr double cos_taylor(double x) {
  double x2 = x * x, term = 1.0, sum = 1.0;
  for (int n = 1; n < 40; ++n) {
    term *= -x2 / ((2.0 * n - 1.0) * (2.0 * n));
    sum += term;
  }
  return sum;
}

// P_n(x) and P_n'(x)
constexpr void legendre(int n, double x, double& Pn, double& dPn) {
  double p0 = 1.0, p1 = x, d0 = 0.0, d1 = 1.0;
  if (n == 0) {
    Pn = 1.0;
    dPn = 0.0;
    return;
  }
  for (int k = 1; k < n; ++k) {
    const double p2 = ((2 * k + 1) * x * p1 - k * p0) / (k + 1);
    const double d2 = d0 + (2 * k + 1) * p1;
    p0 = p1;
    p1 = p2;
    d0 = d1;
    d1 = d2;
  }
  Pn = p1;
  dPn = d1;
}

template <int Q>
constexpr Vec<Q> gauss_points() {
  Vec<Q> r{};
  for (int i = 0; i < Q; ++i) {
    double t = -cos_taylor(kPi * (i + 0.75) / (Q + 0.5));
    for (int it = 0; it < 60; ++it) {
      double Pn = 0, dPn = 0;
      legendre(Q, t, Pn, dPn);
      const double dt = Pn / dPn;
      t -= dt;
      if (absd(dt) < 1e-17) break;
    }
    r.v[i] = t;
  }
  return r;
}

// 1 / w_k^2 for the Q-point Gauss weights w = 2 / ((1 - x^2) P_Q'(x)^2)
template <int Q>
constexpr Vec<Q> gauss_inverse_square_weights() {
  const Vec<Q> x = gauss_points<Q>();
  Vec<Q> r{};
  for (int i = 0; i < Q; ++i) {
    double Pn = 0, dPn = 0;
    legendre(Q, x.v[i], Pn, dPn);
    const double w = 2.0 / ((1.0 - x.v[i] * x.v[i]) * dPn * dPn);
    r.v[i] = 1.0 / (w * w);
  }
  return r;
}

// the P = p + 1 GLL nodes
template <int P>
constexpr Vec<P> gll_points() {
  constexpr int p = P - 1;
  Vec<P> r{};
  for (int i = 0; i <= p; ++i) {
    double t = i == 0 ? -1.0 : 1.0;
    if (i > 0 && i < p) {
      t = -cos_taylor(kPi * i / p);
      for (int it = 0; it < 60; ++it) {
        double Pn = 0, dPn = 0;
        legendre(p, t, Pn, dPn);
        // P_p'' from Legendre's equation
        const double d2 = (2.0 * t * dPn - p * (p + 1.0) * Pn) / (1.0 - t * t);
        const double dt = dPn / d2;
        t -= dt;
        if (absd(dt) < 1e-17) break;
      }
    }
    r.v[i] = t;
  }
  return r;
}

// L[k][a] = l_a(x_k), l_a the Lagrange polynomial of node a
template <int NP, int NQ>
constexpr Vec<NQ * NP> lagrange_values(const Vec<NP>& nodes, const Vec<NQ>& x) {
  Vec<NQ * NP> L{};
  for (int k = 0; k < NQ; ++k)
    for (int a = 0; a < NP; ++a) {
      double v = 1.0;
      for (int m = 0; m < NP; ++m)
        if (m != a) v *= (x.v[k] - nodes.v[m]) / (nodes.v[a] - nodes.v[m]);
      L.v[k * NP + a] = v;
    }
  return L;
}

// D[k][a] = l_a'(x_k)
template <int NP, int NQ>
constexpr Vec<NQ * NP> lagrange_derivatives(const Vec<NP>& nodes, const Vec<NQ>& x) {
  Vec<NQ * NP> D{};
  for (int k = 0; k < NQ; ++k)
    for (int a = 0; a < NP; ++a) {
      double s = 0.0;
      for (int m = 0; m < NP; ++m) {
        if (m == a) continue;
        double t = 1.0 / (nodes.v[a] - nodes.v[m]);
        for (int n = 0; n < NP; ++n)
          if (n != a && n != m) t *= (x.v[k] - nodes.v[n]) / (nodes.v[a] - nodes.v[n]);
        s += t;
      }
      D.v[k * NP + a] = s;
    }
  return D;
}

// SEM-NI: D[c][m] = l_m'(xi_c) on the P GLL nodes (the run-time table Db)
template <int P>
struct GllTables {
  static constexpr Vec<P> nodes = gll_points<P>();
  static constexpr Vec<P * P> D = lagrange_derivatives<P, P>(nodes, nodes);
};

// SEM: B[k][a] = l_a(x_k) from the P GLL nodes to the Q Gauss points, the
// collocation derivative Dq[k][m] = L_m'(x_k) of the Lagrange basis on the
// Gauss points, and 1/w_k^2 (the run-time tables B, Dq and iw2)
template <int P, int Q>
struct SemTables {
  static constexpr Vec<P> nodes = gll_points<P>();
  static constexpr Vec<Q> points = gauss_points<Q>();
  static constexpr Vec<Q * P> B = lagrange_values<P, Q>(nodes, points);
  static constexpr Vec<Q * Q> Dq = lagrange_derivatives<Q, Q>(points, points);
  static constexpr Vec<Q> iw2 = gauss_inverse_square_weights<Q>();
};

}  // namespace rules
}  // namespace mfsem
