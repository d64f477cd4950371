// 1-D reference data of the GLL-Lagrange Q_p basis (host, FP64).
//
// The fine space is the continuous Q_p space of Sec. 3.1 on square cells;
// the element basis here is the Lagrange basis on the Gauss-Lobatto-Legendre
// points of each cell (the paper's NGSolve hierarchical basis spans the same
// space).  Reference matrices on [0,1] are integrated exactly with a
// (p+2)-point Gauss-Legendre rule; the interpolation table is the degree-p/2
// Lagrange basis on the equispaced coarse points of a cell (Sec. 4.2),
// evaluated at the fine GLL points.
#include <cmath>
#include <vector>

#include "common.hpp"

namespace th {

namespace {

// Legendre P_n(x) and P_n'(x) by the three-term recurrence.
void legendre(int n, double x, double &pn, double &dpn) {
  double p0 = 1.0, p1 = x;
  if (n == 0) { pn = 1.0; dpn = 0.0; return; }
  for (int k = 2; k <= n; ++k) {
    double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
    p0 = p1;
    p1 = p2;
  }
  pn = p1;
  // derivative from (1 - x^2) P_n' = n (P_{n-1} - x P_n); end points by limit
  if (std::fabs(1.0 - x * x) < 1e-300) {
    double s = (x > 0) ? 1.0 : ((n % 2) ? 1.0 : -1.0);
    dpn = s * 0.5 * n * (n + 1.0);
  } else {
    dpn = n * (p0 - x * p1) / (1.0 - x * x);
  }
}

}  // namespace

// GLL points (ascending) and weights on [-1, 1]: end points plus the roots of
// P_p', found by Newton's method from Chebyshev-Gauss-Lobatto guesses.
void gll_points(int p, std::vector<double> &x, std::vector<double> &w) {
  x.assign(p + 1, 0.0);
  w.assign(p + 1, 0.0);
  x[0] = -1.0;
  x[p] = 1.0;
  for (int i = 1; i < p; ++i) {
    double t = -std::cos(M_PI * i / p);
    for (int it = 0; it < 100; ++it) {
      double pn, dpn;
      legendre(p, t, pn, dpn);
      // second derivative from the Legendre ODE
      double d2 = (2.0 * t * dpn - p * (p + 1.0) * pn) / (1.0 - t * t);
      double dt = dpn / d2;
      t -= dt;
      if (std::fabs(dt) < 1e-16) break;
    }
    x[i] = t;
  }
  for (int i = 0; i <= p; ++i) {
    double pn, dpn;
    legendre(p, x[i], pn, dpn);
    w[i] = 2.0 / (p * (p + 1.0) * pn * pn);
  }
  // enforce symmetry
  for (int i = 0; i <= p / 2; ++i) {
    double a = 0.5 * (x[p - i] - x[i]);
    x[i] = -a;
    x[p - i] = a;
    double b = 0.5 * (w[i] + w[p - i]);
    w[i] = w[p - i] = b;
  }
}

// Gauss-Legendre points/weights on [-1,1] (Newton on P_n).
void gauss_points(int n, std::vector<double> &x, std::vector<double> &w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    double t = -std::cos(M_PI * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      double pn, dpn;
      legendre(n, t, pn, dpn);
      double dt = pn / dpn;
      t -= dt;
      if (std::fabs(dt) < 1e-16) break;
    }
    double pn, dpn;
    legendre(n, t, pn, dpn);
    x[i] = t;
    w[i] = 2.0 / ((1.0 - t * t) * dpn * dpn);
  }
}

// Lagrange basis through nodes[0..n) at point t: values and derivatives.
static void lagrange_eval(const std::vector<double> &nodes, double t, std::vector<double> &val,
                          std::vector<double> &der) {
  int n = (int)nodes.size();
  val.assign(n, 0.0);
  der.assign(n, 0.0);
  for (int j = 0; j < n; ++j) {
    double denom = 1.0, v = 1.0, d = 0.0;
    for (int m = 0; m < n; ++m) {
      if (m == j) continue;
      denom *= nodes[j] - nodes[m];
      // d/dt of the running product
      d = d * (t - nodes[m]) + v;
      v *= (t - nodes[m]);
    }
    val[j] = v / denom;
    der[j] = d / denom;
  }
}

// Fill K, M (on [0,1]) and the coarse interpolation table L for order p.
void make_ref1d(int p, Ref1D &ref) {
  std::vector<double> xg, wg, xq, wq;
  gll_points(p, xg, wg);
  std::vector<double> nodes(p + 1);
  for (int i = 0; i <= p; ++i) nodes[i] = 0.5 * (xg[i] + 1.0);
  gauss_points(p + 2, xq, wq);
  for (int i = 0; i < (kMaxP + 1) * (kMaxP + 1); ++i) ref.K[i] = ref.M[i] = 0.0;
  std::vector<double> val, der;
  for (int q = 0; q < p + 2; ++q) {
    double t = 0.5 * (xq[q] + 1.0), wt = 0.5 * wq[q];
    lagrange_eval(nodes, t, val, der);
    for (int a = 0; a <= p; ++a)
      for (int b = 0; b <= p; ++b) {
        ref.K[a * (p + 1) + b] += wt * der[a] * der[b];
        ref.M[a * (p + 1) + b] += wt * val[a] * val[b];
      }
  }
  int r = p / 2;
  std::vector<double> cpts(r + 1);
  for (int b = 0; b <= r; ++b) cpts[b] = (double)b / r;
  for (int i = 0; i < (kMaxP + 1) * (kMaxP / 2 + 1); ++i) ref.L[i] = 0.0;
  for (int a = 0; a <= p; ++a) {
    lagrange_eval(cpts, nodes[a], val, der);
    for (int b = 0; b <= r; ++b) {
      double v = val[b];
      if (std::fabs(v) < 1e-15) v = 0.0;
      if (std::fabs(v - 1.0) < 1e-15) v = 1.0;
      ref.L[a * (r + 1) + b] = v;
    }
  }
}

}  // namespace th
