// Per-cell coarse stencils from the surrogate network's output, and the
// fallback check of each stencil against the fine discrete dispersion, on the
// device.
//
// The network predicts the fine dispersion errors e_m at the fit directions
// (standardised log values); the stencil weights follow from them by the
// plain-fit formulas (the coarse symbol vanishes at eta (1 + e_m) along t_m,
// scaled so that sigma(0) = -eta^2, eq. scaling_factor_QSFEM).  The check
// measures how far the zero set of that stencil lies from the fine Q_p
// dispersion curve over the whole symmetry sector, not only at the fit
// directions: the fine curve is traced parametrically through the separation
// of the tensor-product symbol, mu(theta_x) + mu(theta_y) (+ mu(theta_z)) =
// (kh)^2 (the discrete dispersion relation of the appendix), with
// theta = acos F(mu) from the condensed one-cell pencil (F(mu) = -s0/s1 of the
// Schur complement of K - mu M on the cell's end nodes), so no root is
// searched.  At every traced point phi_f (in coarse phase units) the radial
// distance to the coarse zero set is estimated by one Newton step,
// delta = -sigma(phi_f) / (grad sigma . phi_f); the cell's mismatch is
// max |delta| |phi_f| / eta over the points.  A cell whose mismatch exceeds
// the caller's tau (or is not finite) takes the exact plain fit on the host.
#include <cmath>

#include "ctx.hpp"

namespace th {

constexpr int kCheckPts2 = 16;    // traced points of the fine curve in the sector 0 <= t <= pi/4
constexpr int kCheckGrid3 = 5;    // 3-D: barycentric grid of the sector simplex (21 points)

struct NetScale {
  double out_mean[3], out_std[3];
  double floor;
};

// cos(theta) of the condensed 3-point scheme at eigenvalue mu of the 1-D pencil
// (K, M) of order p; false past the first interior resonance.
__device__ bool dev_condensed_F(const Ref1D &ref, int p, double mu, double &F) {
  const int n = p + 1;
  auto E = [&](int a, int b) { return ref.K[a * n + b] - mu * ref.M[a * n + b]; };
  if (p == 1) {
    F = -E(0, 0) / E(0, 1);
    return true;
  }
  const int m = p - 1;
  double L[(kMaxP - 1) * (kMaxP - 1)];
  for (int i = 0; i < m; ++i)
    for (int j = 0; j <= i; ++j) {
      double s = E(i + 1, j + 1);
      for (int k = 0; k < j; ++k) s -= L[i * m + k] * L[j * m + k];
      if (i == j) {
        if (!(s > 0.0)) return false;
        L[i * m + i] = sqrt(s);
      } else {
        L[i * m + j] = s / L[j * m + j];
      }
    }
  double z0[kMaxP - 1], zp[kMaxP - 1];
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

// fine phase theta of the acoustic branch at mu, or -1 when mu is past it
__device__ double dev_theta(const Ref1D &ref, int p, double mu) {
  if (mu <= 0.0) return 0.0;
  double F;
  if (!dev_condensed_F(ref, p, mu, F) || !(F >= -1.0 && F <= 1.0)) return -1.0;
  return acos(F);
}

// Re sqrt(1 + i shift): the real wavenumber factor of the damped medium
__device__ __forceinline__ double dev_eff(double shift) {
  return sqrt(0.5 * (1.0 + sqrt(1.0 + shift * shift)));
}

template <int DIM>
__global__ __launch_bounds__(256) void k_stencil_check(const double *__restrict__ samples,
                                                       const float *__restrict__ y, int n,
                                                       Ref1D ref, NetScale sc,
                                                       double *__restrict__ q_out,
                                                       double *__restrict__ mis) {
  constexpr int NO = DIM == 3 ? 3 : 2, NQ = DIM == 3 ? 4 : 3;
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const double eta_c = samples[3 * i], shift = samples[3 * i + 2];
  const int p = (int)lround(samples[3 * i + 1]);
  const double eta = eta_c * dev_eff(shift);
  double e[NO];
#pragma unroll
  for (int c = 0; c < NO; ++c) {
    const double yr = (double)y[NO * i + c] * sc.out_std[c] + sc.out_mean[c];
    e[c] = -(exp(yr) - sc.floor);
  }
  // stencil classes P (P0 fixed) whose symbol vanishes at eta (1 + e_m) along the fit directions
  double P[4];
  if (DIM == 2) {
    const double t1 = M_PI / 16.0, t2 = 3.0 * M_PI / 16.0;
    const double z1 = eta * (1.0 + e[0]), z2 = eta * (1.0 + e[1]);
    const double c1 = cos(z1 * cos(t1)), s1 = cos(z1 * sin(t1));
    const double c2 = cos(z2 * cos(t2)), s2 = cos(z2 * sin(t2));
    const double den = c2 * s2 * (c1 + s1) - c1 * s1 * (c2 + s2);
    P[0] = 4.0;
    P[1] = 2.0 * (c1 * s1 - c2 * s2) / den;
    P[2] = (c2 + s2 - c1 - s1) / den;
    const double Nn = -eta * eta / (P[0] + 4.0 * P[1] + 4.0 * P[2]);
    q_out[NQ * i + 0] = Nn * P[0] / 4.0;
    q_out[NQ * i + 1] = Nn * P[1] / 2.0;
    q_out[NQ * i + 2] = Nn * P[2];
  } else {
    const double raw[3][3] = {{1.0, 0.2, 0.1}, {1.0, 0.6, 0.3}, {1.0, 0.9, 0.7}};
    double A[3][4];
    for (int m = 0; m < 3; ++m) {
      const double nr = sqrt(raw[m][0] * raw[m][0] + raw[m][1] * raw[m][1] + raw[m][2] * raw[m][2]);
      const double z = eta * (1.0 + e[m]);
      const double c0 = cos(z * raw[m][0] / nr), c1 = cos(z * raw[m][1] / nr), c2 = cos(z * raw[m][2] / nr);
      A[m][0] = 2.0 * (c0 + c1 + c2);
      A[m][1] = 4.0 * (c0 * c1 + c0 * c2 + c1 * c2);
      A[m][2] = 8.0 * c0 * c1 * c2;
      A[m][3] = -8.0;
    }
    for (int k = 0; k < 3; ++k) {  // partial pivoting
      int piv = k;
      for (int r = k + 1; r < 3; ++r)
        if (fabs(A[r][k]) > fabs(A[piv][k])) piv = r;
      for (int j = 0; j < 4; ++j) {
        const double t = A[k][j];
        A[k][j] = A[piv][j];
        A[piv][j] = t;
      }
      for (int r = k + 1; r < 3; ++r) {
        const double f = A[r][k] / A[k][k];
        for (int j = k; j < 4; ++j) A[r][j] -= f * A[k][j];
      }
    }
    double X[3];
    for (int r = 2; r >= 0; --r) {
      double t = A[r][3];
      for (int j = r + 1; j < 3; ++j) t -= A[r][j] * X[j];
      X[r] = t / A[r][r];
    }
    P[0] = 8.0;
    P[1] = X[0];
    P[2] = X[1];
    P[3] = X[2];
    const double Nn = -eta * eta / (P[0] + 6.0 * P[1] + 12.0 * P[2] + 8.0 * P[3]);
    q_out[NQ * i + 0] = Nn * P[0] / 8.0;
    q_out[NQ * i + 1] = Nn * P[1] / 4.0;
    q_out[NQ * i + 2] = Nn * P[2] / 2.0;
    q_out[NQ * i + 3] = Nn * P[3];
  }
  // trace the fine curve (fine kh = eta p / 2, phases converted by h_c / h = 2 / p)
  const double kh = eta * p / 2.0, k2 = kh * kh, toc = 2.0 / p;
  double worst = 0.0;
  auto probe = [&](const double *mu) {
    double ph[3] = {0, 0, 0};
    for (int a = 0; a < DIM; ++a) {
      const double th = dev_theta(ref, p, mu[a]);
      if (th < 0.0) {
        worst = INFINITY;
        return;
      }
      ph[a] = th * toc;
    }
    double sig, g[3] = {0, 0, 0};
    if (DIM == 2) {
      const double cx_ = cos(ph[0]), cy_ = cos(ph[1]);
      sig = P[0] + 2.0 * P[1] * (cx_ + cy_) + 4.0 * P[2] * cx_ * cy_;
      g[0] = -sin(ph[0]) * (2.0 * P[1] + 4.0 * P[2] * cy_);
      g[1] = -sin(ph[1]) * (2.0 * P[1] + 4.0 * P[2] * cx_);
    } else {
      const double c0 = cos(ph[0]), c1 = cos(ph[1]), c2 = cos(ph[2]);
      sig = P[0] + 2.0 * P[1] * (c0 + c1 + c2) + 4.0 * P[2] * (c0 * c1 + c0 * c2 + c1 * c2) +
            8.0 * P[3] * c0 * c1 * c2;
      g[0] = -sin(ph[0]) * (2.0 * P[1] + 4.0 * P[2] * (c1 + c2) + 8.0 * P[3] * c1 * c2);
      g[1] = -sin(ph[1]) * (2.0 * P[1] + 4.0 * P[2] * (c0 + c2) + 8.0 * P[3] * c0 * c2);
      g[2] = -sin(ph[2]) * (2.0 * P[1] + 4.0 * P[2] * (c0 + c1) + 8.0 * P[3] * c0 * c1);
    }
    const double gr = g[0] * ph[0] + g[1] * ph[1] + g[2] * ph[2];
    const double r = sqrt(ph[0] * ph[0] + ph[1] * ph[1] + ph[2] * ph[2]);
    const double d = fabs(sig / gr) * r / eta;
    if (!(d <= worst)) worst = d;  // NaN propagates
  };
  if (DIM == 2) {
    for (int m = 0; m < kCheckPts2; ++m) {
      // mu_x from k2 / 2 (diagonal, t = pi/4) to k2 (axis, t = 0), both ends included
      const double w = 0.5 + 0.5 * m / (kCheckPts2 - 1);
      const double mu[2] = {w * k2, (1.0 - w) * k2};
      probe(mu);
    }
  } else {
    // sector mu_x >= mu_y >= mu_z: barycentric points of the triangle with
    // corners (1, 0, 0), (1/2, 1/2, 0), (1/3, 1/3, 1/3)
    const double V[3][3] = {{1.0, 0.0, 0.0}, {0.5, 0.5, 0.0}, {1.0 / 3, 1.0 / 3, 1.0 / 3}};
    for (int a = 0; a <= kCheckGrid3; ++a)
      for (int b = 0; a + b <= kCheckGrid3; ++b) {
        const int c = kCheckGrid3 - a - b;
        const double wa = (double)a / kCheckGrid3, wb = (double)b / kCheckGrid3,
                     wc = (double)c / kCheckGrid3;
        double mu[3];
        for (int k = 0; k < 3; ++k) mu[k] = k2 * (wa * V[0][k] + wb * V[1][k] + wc * V[2][k]);
        probe(mu);
      }
  }
  mis[i] = worst;
}

int stencil_check_launch(int dim, int p, const double *d_samples, const float *d_y, int n,
                         const double out_mean[3], const double out_std[3], double floor_,
                         double *d_q, double *d_mis, hipStream_t s) {
  Ref1D ref;
  make_ref1d(p, ref);
  NetScale sc;
  for (int c = 0; c < 3; ++c) {
    sc.out_mean[c] = out_mean[c];
    sc.out_std[c] = out_std[c];
  }
  sc.floor = floor_;
  if (dim == 3)
    hipLaunchKernelGGL(k_stencil_check<3>, dim3(ceil_div(n, 256)), dim3(256), 0, s, d_samples, d_y,
                       n, ref, sc, d_q, d_mis);
  else
    hipLaunchKernelGGL(k_stencil_check<2>, dim3(ceil_div(n, 256)), dim3(256), 0, s, d_samples, d_y,
                       n, ref, sc, d_q, d_mis);
  TH_HIP_CHECK_RET(hipGetLastError());
  return 0;
}

}  // namespace th
