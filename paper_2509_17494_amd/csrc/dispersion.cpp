// Fine-level discrete dispersion of the Q_p scheme and the plain
// dispersion-matching coarse stencil (host, FP64).
//
// Discrete dispersion (Sec. 6.2 and the appendix): Bloch waves of the FE
// matrix exist where det A^(theta) = 0.  For the tensor-product element the
// 2-D symbol is K^(tx) x M^(ty) + M^(tx) x K^(ty) - (kh)^2 M^(tx) x M^(ty)
// with the 1-D symbols K^, M^ (h = 1), so in the basis of the 1-D generalised
// eigenvectors it is diagonal and det A^ = 0 exactly when
//     mu(theta_x) + mu(theta_y) = (kh)^2
// for 1-D branches mu(theta) of the pencil (K^, M^).  The acoustic branch is
// the one through mu(0) = 0.  It is evaluated by condensing the element's
// interior nodes: for E(mu) = K1 - mu M1 on one cell the Schur complement on
// the two end nodes is [[s0, s1], [s1, s0]], and the 1-D Bloch condition of
// the condensed 3-point scheme gives cos(theta) = -s0(mu) / s1(mu) =: F(mu),
// which decreases from 1 at mu = 0 to -1 at the first interior resonance.
//
// Plain fit: the 9-point family of QSFEM (Sec. 3.2, P0 = 4) with P1, P2 such
// that the coarse symbol vanishes at the fine discrete wave vectors of the two
// QSFEM directions t = pi/16, 3 pi/16, scaled so that sigma(0) = -eta^2
// (eq. scaling_factor_QSFEM).  "shift" = eps / k^2 enters as the real
// wavenumber of the damped medium, k Re sqrt(1 + i shift).
#include <algorithm>
#include <cmath>
#include <complex>
#include <thread>
#include <vector>

#include "ctx.hpp"

namespace th {

namespace {

constexpr double kT1 = M_PI / 16.0, kT2 = 3.0 * M_PI / 16.0;

struct Pencil1D {
  int p;
  double K[(kMaxP + 1) * (kMaxP + 1)], M[(kMaxP + 1) * (kMaxP + 1)];
};

// F(mu) = -s0/s1 of the condensed cell; false when E_ii(mu) is not positive
// definite (mu at or past the first interior resonance).
bool condensed_F(const Pencil1D &q, double mu, double &F) {
  const int p = q.p, n = p + 1;
  auto E = [&](int a, int b) { return q.K[a * n + b] - mu * q.M[a * n + b]; };
  if (p == 1) {
    F = -E(0, 0) / E(0, 1);
    return true;
  }
  const int m = p - 1;  // interior nodes 1..p-1
  double L[kMaxP * kMaxP];
  for (int i = 0; i < m; ++i)
    for (int j = 0; j <= i; ++j) {
      double s = E(i + 1, j + 1);
      for (int k = 0; k < j; ++k) s -= L[i * m + k] * L[j * m + k];
      if (i == j) {
        if (!(s > 0.0)) return false;
        L[i * m + i] = std::sqrt(s);
      } else {
        L[i * m + j] = s / L[j * m + j];
      }
    }
  // z = E_ii^{-1} e_ib for the two boundary columns (nodes 0 and p)
  double z0[kMaxP], zp[kMaxP];
  for (int col = 0; col < 2; ++col) {
    const int b = col == 0 ? 0 : p;
    double *z = col == 0 ? z0 : zp;
    for (int i = 0; i < m; ++i) {
      double s = E(i + 1, b);
      for (int k = 0; k < i; ++k) s -= L[i * m + k] * z[k];
      z[i] = s / L[i * m + i];
    }
    for (int i = m - 1; i >= 0; --i) {
      double s = z[i];
      for (int k = i + 1; k < m; ++k) s -= L[k * m + i] * z[k];
      z[i] = s / L[i * m + i];
    }
  }
  double s0 = E(0, 0), s1 = E(0, p);
  for (int i = 0; i < m; ++i) {
    s0 -= E(0, i + 1) * z0[i];
    s1 -= E(0, i + 1) * zp[i];
  }
  F = -s0 / s1;
  return true;
}

// Illinois (modified regula falsi) on a bracket [a, b] with f(a) > 0 > f(b).
template <typename Fn>
double illinois(Fn f, double a, double fa, double b, double fb, double tol) {
  int side = 0;
  for (int it = 0; it < 200; ++it) {
    const double c = (fa * b - fb * a) / (fa - fb);
    const double fc = f(c);
    if (fc == 0.0 || std::fabs(b - a) <= tol * std::fabs(c)) return c;
    if (fc > 0.0) {
      a = c;
      fa = fc;
      if (side == 1) fb *= 0.5;
      side = 1;
    } else {
      b = c;
      fb = fc;
      if (side == -1) fa *= 0.5;
      side = -1;
    }
  }
  return 0.5 * (a + b);
}

}  // namespace

// Acoustic branch mu(theta), theta in [0, pi).
static double mu_acoustic(const Pencil1D &q, double theta) {
  theta = std::fabs(theta);
  if (theta == 0.0) return 0.0;
  const double c = std::cos(theta);
  // f(mu) = F(mu) - cos(theta): positive at 0, negative past the root;
  // beyond the resonance treat as negative
  auto f = [&](double mu) {
    double F;
    if (!condensed_F(q, mu, F)) return -1.0 - c;
    return F - c;
  };
  double a = 0.0, fa = 1.0 - c;
  double b = std::max(1.2 * theta * theta, 1e-12), fb = f(b);
  int guard = 0;
  while (fb > 0.0 && guard++ < 200) {
    a = b;
    fa = fb;
    b *= 1.5;
    fb = f(b);
  }
  return illinois(f, a, fa, b, fb, 1e-15);
}

// Radius r (h = 1) of the fine Q_p dispersion curve along direction t, kh < pi.
static double fine_radius(const Pencil1D &q, double kh, double t) {
  const double ct = std::fabs(std::cos(t)), st = std::fabs(std::sin(t));
  const double k2 = kh * kh;
  auto g = [&](double r) { return k2 - (mu_acoustic(q, r * ct) + mu_acoustic(q, r * st)); };
  const double rmax = 0.999 * M_PI / std::max(ct, st);
  double a = 0.5 * kh, b = std::min(1.5 * kh, rmax);
  double ga = g(a), gb = g(b);
  if (!(ga > 0.0 && gb < 0.0)) return kh;  // outside the supported regime
  return illinois(g, a, ga, b, gb, 1e-15);
}

static void make_pencil(int p, Pencil1D &q) {
  Ref1D ref;
  make_ref1d(p, ref);
  q.p = p;
  for (int i = 0; i < (kMaxP + 1) * (kMaxP + 1); ++i) {
    q.K[i] = ref.K[i];
    q.M[i] = ref.M[i];
  }
}

double effective_eta(double eta_c, double shift) {
  return eta_c * std::sqrt(std::complex<double>(1.0, shift)).real();
}

// Relative fine dispersion errors e_m = r(t_m) / kh - 1 at the QSFEM
// directions for a coarse cell with eta_c = h_c k (fine kh = eta p / 2).
void fine_errors(int p, double eta_c, double shift, double e[2]) {
  Pencil1D q;
  make_pencil(p, q);
  const double eta = effective_eta(eta_c, shift);
  const double kh = eta * p / 2.0;
  e[0] = fine_radius(q, kh, kT1) / kh - 1.0;
  e[1] = fine_radius(q, kh, kT2) / kh - 1.0;
}

// Weights (q0, q_edge, q_diag) whose symbol vanishes at eta (1 + e_m) along t_m.
void fit_from_errors(double eta, const double e[2], double qw[3]) {
  const double z1 = eta * (1.0 + e[0]), z2 = eta * (1.0 + e[1]);
  const double c1 = std::cos(z1 * std::cos(kT1)), s1 = std::cos(z1 * std::sin(kT1));
  const double c2 = std::cos(z2 * std::cos(kT2)), s2 = std::cos(z2 * std::sin(kT2));
  const double den = c2 * s2 * (c1 + s1) - c1 * s1 * (c2 + s2);
  const double P0 = 4.0;
  const double P1 = 2.0 * (c1 * s1 - c2 * s2) / den;
  const double P2 = (c2 + s2 - c1 - s1) / den;
  const double Nn = -eta * eta / (P0 + 4.0 * P1 + 4.0 * P2);
  qw[0] = Nn * P0 / 4.0;
  qw[1] = Nn * P1 / 2.0;
  qw[2] = Nn * P2;
}

// Plain fit for n cells (inputs eta_c, p, shift per cell), threaded.
void plain_fit_batch(const double *x, int n, double *e_out, double *q_out) {
  unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  nt = std::min<unsigned>(nt, (unsigned)std::max(1, n / 64));
  auto work = [&](int i0, int i1) {
    int last_p = -1;
    Pencil1D q;
    for (int i = i0; i < i1; ++i) {
      const double eta_c = x[3 * i], shift = x[3 * i + 2];
      const int p = (int)std::lround(x[3 * i + 1]);
      if (p != last_p) {
        make_pencil(p, q);
        last_p = p;
      }
      const double eta = effective_eta(eta_c, shift);
      const double kh = eta * p / 2.0;
      double e[2] = {fine_radius(q, kh, kT1) / kh - 1.0, fine_radius(q, kh, kT2) / kh - 1.0};
      if (e_out) {
        e_out[2 * i] = e[0];
        e_out[2 * i + 1] = e[1];
      }
      if (q_out) fit_from_errors(eta, e, q_out + 3 * i);
    }
  };
  std::vector<std::thread> ts;
  const int chunk = (n + nt - 1) / nt;
  for (unsigned t = 0; t < nt; ++t) {
    const int i0 = t * chunk, i1 = std::min(n, (int)(t + 1) * chunk);
    if (i0 < i1) ts.emplace_back(work, i0, i1);
  }
  for (auto &t : ts) t.join();
}

// ---------------------------------------------------------------------------
// 3-D: the compact 27-point family with classes P0 = 8 (centre), P1 (face),
// P2 (edge), P3 (corner),
//   sigma(xi) = P0 + 2 P1 sum c_i + 4 P2 sum_{i<j} c_i c_j + 8 P3 c_1 c_2 c_3,
// c_i = cos(h_c xi_i), whose zero set is put through three points along fixed
// directions of the symmetry sector (normalised (1, .2, .1), (1, .6, .3),
// (1, .9, .7)); N = -eta^2 / sigma(0); element weights N P0 / 8, N P1 / 4,
// N P2 / 2, N P3 for vertex pairs at Hamming distance 0..3 (the quasi-FE
// distribution of Sec. 3.3 in three dimensions).  The fine 3-D Q_p dispersion
// separates as mu(theta_x) + mu(theta_y) + mu(theta_z) = (kh)^2.

static void dirs27(double d[3][3]) {
  const double raw[3][3] = {{1.0, 0.2, 0.1}, {1.0, 0.6, 0.3}, {1.0, 0.9, 0.7}};
  for (int m = 0; m < 3; ++m) {
    const double n = std::sqrt(raw[m][0] * raw[m][0] + raw[m][1] * raw[m][1] + raw[m][2] * raw[m][2]);
    for (int i = 0; i < 3; ++i) d[m][i] = raw[m][i] / n;
  }
}

// Weights (q0, q_face, q_edge, q_corner) with zeros at radius z[m] along the
// m-th direction (z[m] = eta gives the exact-wavenumber stencil).
void fit27_from_radii(double eta, const double z[3], double qw[4]) {
  double d[3][3];
  dirs27(d);
  double A[3][4];
  for (int m = 0; m < 3; ++m) {
    const double c0 = std::cos(z[m] * d[m][0]), c1 = std::cos(z[m] * d[m][1]),
                 c2 = std::cos(z[m] * d[m][2]);
    A[m][0] = 2.0 * (c0 + c1 + c2);
    A[m][1] = 4.0 * (c0 * c1 + c0 * c2 + c1 * c2);
    A[m][2] = 8.0 * c0 * c1 * c2;
    A[m][3] = -8.0;
  }
  // Gaussian elimination with partial pivoting
  for (int k = 0; k < 3; ++k) {
    int piv = k;
    for (int i = k + 1; i < 3; ++i)
      if (std::fabs(A[i][k]) > std::fabs(A[piv][k])) piv = i;
    if (piv != k)
      for (int j = 0; j < 4; ++j) std::swap(A[k][j], A[piv][j]);
    for (int i = k + 1; i < 3; ++i) {
      const double f = A[i][k] / A[k][k];
      for (int j = k; j < 4; ++j) A[i][j] -= f * A[k][j];
    }
  }
  double P[3];
  for (int i = 2; i >= 0; --i) {
    double t = A[i][3];
    for (int j = i + 1; j < 3; ++j) t -= A[i][j] * P[j];
    P[i] = t / A[i][i];
  }
  const double P0 = 8.0;
  const double Nn = -eta * eta / (P0 + 6.0 * P[0] + 12.0 * P[1] + 8.0 * P[2]);
  qw[0] = Nn * P0 / 8.0;
  qw[1] = Nn * P[0] / 4.0;
  qw[2] = Nn * P[1] / 2.0;
  qw[3] = Nn * P[2];
}

// Radius (h = 1) of the fine 3-D Q_p dispersion surface along unit vector d.
static double fine_radius3(const Pencil1D &q, double kh, const double d[3]) {
  const double a0 = std::fabs(d[0]), a1 = std::fabs(d[1]), a2 = std::fabs(d[2]);
  const double k2 = kh * kh;
  auto g = [&](double r) {
    return k2 - (mu_acoustic(q, r * a0) + mu_acoustic(q, r * a1) + mu_acoustic(q, r * a2));
  };
  const double rmax = 0.999 * M_PI / std::max(a0, std::max(a1, a2));
  double a = 0.5 * kh, b = std::min(1.5 * kh, rmax);
  double ga = g(a), gb = g(b);
  if (!(ga > 0.0 && gb < 0.0)) return kh;  // outside the supported regime
  return illinois(g, a, ga, b, gb, 1e-15);
}

// Plain 3-D fit for n cells (inputs eta_c, p, shift per cell): q_out[4 i ...],
// and the relative fine errors e_out[3 i ...] when requested.
void plain_fit27_batch(const double *x, int n, double *e_out, double *q_out) {
  unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  nt = std::min<unsigned>(nt, (unsigned)std::max(1, n / 64));
  double d[3][3];
  dirs27(d);
  auto work = [&](int i0, int i1) {
    int last_p = -1;
    Pencil1D q;
    for (int i = i0; i < i1; ++i) {
      const double eta_c = x[3 * i], shift = x[3 * i + 2];
      const int p = (int)std::lround(x[3 * i + 1]);
      if (p != last_p) {
        make_pencil(p, q);
        last_p = p;
      }
      const double eta = effective_eta(eta_c, shift);
      const double kh = eta * p / 2.0;
      double z[3];
      for (int m = 0; m < 3; ++m) {
        const double e = fine_radius3(q, kh, d[m]) / kh - 1.0;
        if (e_out) e_out[3 * i + m] = e;
        z[m] = eta * (1.0 + e);
      }
      if (q_out) fit27_from_radii(eta, z, q_out + 4 * i);
    }
  };
  std::vector<std::thread> ts;
  const int chunk = (n + nt - 1) / nt;
  for (unsigned t = 0; t < nt; ++t) {
    const int i0 = t * chunk, i1 = std::min(n, (int)(t + 1) * chunk);
    if (i0 < i1) ts.emplace_back(work, i0, i1);
  }
  for (auto &t : ts) t.join();
}

}  // namespace th
