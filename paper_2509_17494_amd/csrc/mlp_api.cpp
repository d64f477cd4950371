// C ABI of the dispersion-matched coarse stencils: plain fit (host) and the
// surrogate network (device training and inference), and the per-cell weights
// used by th_setup_coarse for TH_COARSE_PLAINFIT / TH_COARSE_MLP.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "ctx.hpp"

namespace th {
void plain_fit_batch(const double *x, int n, double *e_out, double *q_out);
int stencil_check_launch(int dim, int p, const double *d_samples, const float *d_y, int n,
                         const double out_mean[3], const double out_std[3], double floor_,
                         double *d_q, double *d_mis, hipStream_t s);
void fit_from_errors(double eta, const double e[2], double qw[3]);
double effective_eta(double eta_c, double shift);
int mlp_num_params(int n_out);
int mlp_step_launch(int n_out, const float *master, const unsigned short *wbf, bool bf16,
                    const float *x, const float *t, int n, int off, int count, float inv_norm,
                    float *gpart, float *lpart, hipStream_t s);
int mlp_adam_launch(int n_out, float *master, unsigned short *wbf, float *m1, float *m2,
                    const float *gpart, const float *lpart, int nblk, int step, float lr,
                    float *grad_out, float *loss_out, hipStream_t s);
int mlp_infer_launch(int n_out, const float *master, const unsigned short *wbf, bool bf16,
                     const float *x, float *y, int n, hipStream_t s);
int mlp_refresh_bf16(int n_out, const float *master, unsigned short *wbf, hipStream_t s);

// fine dispersion errors of a stencil family: 2 per sample (9-point) or 3 (27-point)
static void family_errors(int n_out, const double *x, int n, double *e_out) {
  if (n_out == 3)
    plain_fit27_batch(x, n, e_out, nullptr);
  else
    plain_fit_batch(x, n, e_out, nullptr);
}
}  // namespace th

using namespace th;

constexpr double kEFloor = 1e-13;

struct th_mlp {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  float *d_master = nullptr, *d_m1 = nullptr, *d_m2 = nullptr;
  unsigned short *d_bf = nullptr;
  double in_mean[3] = {0, 0, 0}, in_std[3] = {1, 1, 1};
  double out_mean[3] = {0, 0, 0}, out_std[3] = {1, 1, 1};
  int n_out = 2;               // 2: 9-point family (2-D), 3: 27-point family (3-D)
  bool has_weights = false;
};

static th_status mfail(th_mlp *m, th_status st, const std::string &msg) {
  if (m) m->err = msg;
  return st;
}

static th_status check_samples(const double *x, int n, std::string &msg) {
  if (!x || n < 1) {
    msg = "samples must be a non-empty host array";
    return TH_EINVAL;
  }
  for (int i = 0; i < n; ++i) {
    const double eta = x[3 * i], pp = x[3 * i + 1], sh = x[3 * i + 2];
    const long p = std::lround(pp);
    if (!(eta > 0.0) || !std::isfinite(eta) || p < 1 || p > kMaxP || std::fabs(pp - p) > 1e-12 ||
        !(sh >= 0.0) || !std::isfinite(sh)) {
      msg = "sample " + std::to_string(i) + ": need eta_c > 0, integer p in [1, 8], shift >= 0";
      return TH_EINVAL;
    }
    if (!(effective_eta(eta, sh) * p / 2.0 < M_PI)) {
      msg = "sample " + std::to_string(i) + ": fine kh = eta_c p / 2 must be below pi";
      return TH_EINVAL;
    }
  }
  return TH_OK;
}

// Device buffers of one training / inference call (freed on scope exit).
struct DevBuf {
  std::vector<void *> ptrs;
  ~DevBuf() {
    for (void *p : ptrs) (void)hipFree(p);
  }
  template <typename T>
  T *alloc(size_t count) {
    void *p = nullptr;
    if (hipMalloc(&p, std::max<size_t>(count, 1) * sizeof(T)) != hipSuccess) return nullptr;
    ptrs.push_back(p);
    return (T *)p;
  }
};

extern "C" {

th_status th_plain_fit(const double *samples, int n, double *e_out, double *q_out) {
  std::string msg;
  if (check_samples(samples, n, msg) != TH_OK) return TH_EINVAL;
  plain_fit_batch(samples, n, e_out, q_out);
  return TH_OK;
}

th_status th_plain_fit3d(const double *samples, int n, double *e_out, double *q_out) {
  std::string msg;
  if (check_samples(samples, n, msg) != TH_OK) return TH_EINVAL;
  plain_fit27_batch(samples, n, e_out, q_out);
  return TH_OK;
}

th_status th_mlp_num_params(int *n_params) {
  if (!n_params) return TH_EINVAL;
  *n_params = mlp_num_params(2);
  return TH_OK;
}

th_status th_mlp_info(const th_mlp *m, int *dim, int *n_params) {
  if (!m || !dim || !n_params) return TH_EINVAL;
  *dim = m->n_out == 3 ? 3 : 2;
  *n_params = mlp_num_params(m->n_out);
  return TH_OK;
}

th_status th_mlp_create(th_mlp **out, int hip_device, void *hip_stream) {
  return th_mlp_create_family(out, hip_device, hip_stream, 2);
}

th_status th_mlp_create_family(th_mlp **out, int hip_device, void *hip_stream, int dim) {
  if (!out) return TH_EINVAL;
  *out = nullptr;
  if (dim != 2 && dim != 3) return TH_EINVAL;
  if (hipSetDevice(hip_device) != hipSuccess) return TH_EHIP;
  th_mlp *m = new (std::nothrow) th_mlp();
  if (!m) return TH_ENOMEM;
  m->device = hip_device;
  m->stream = (hipStream_t)hip_stream;
  m->n_out = dim == 3 ? 3 : 2;
  const int P = mlp_num_params(m->n_out);
  if (hipMalloc(&m->d_master, P * sizeof(float)) != hipSuccess ||
      hipMalloc(&m->d_m1, P * sizeof(float)) != hipSuccess ||
      hipMalloc(&m->d_m2, P * sizeof(float)) != hipSuccess ||
      hipMalloc(&m->d_bf, P * sizeof(unsigned short)) != hipSuccess) {
    th_mlp_destroy(m);
    return TH_ENOMEM;
  }
  *out = m;
  return TH_OK;
}

void th_mlp_destroy(th_mlp *m) {
  if (!m) return;
  (void)hipSetDevice(m->device);
  if (m->stream) (void)hipStreamSynchronize(m->stream);
  void *ptrs[] = {m->d_master, m->d_m1, m->d_m2, m->d_bf};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  delete m;
}

const char *th_mlp_last_error(const th_mlp *m) { return m ? m->err.c_str() : "null network"; }

th_status th_mlp_set_weights(th_mlp *m, const float *theta, int n_params) {
  if (!m) return TH_EINVAL;
  const int P = mlp_num_params(m->n_out);
  if (!theta || n_params != P) return mfail(m, TH_EINVAL, "weights must hold n_params floats");
  for (int i = 0; i < P; ++i)
    if (!std::isfinite(theta[i])) return mfail(m, TH_EINVAL, "non-finite weight");
  if (hipSetDevice(m->device) != hipSuccess) return mfail(m, TH_EHIP, "hipSetDevice failed");
  if (hipMemcpyAsync(m->d_master, theta, P * sizeof(float), hipMemcpyHostToDevice, m->stream) ||
      hipMemsetAsync(m->d_m1, 0, P * sizeof(float), m->stream) ||
      hipMemsetAsync(m->d_m2, 0, P * sizeof(float), m->stream))
    return mfail(m, TH_EHIP, "upload failed");
  int rc = mlp_refresh_bf16(m->n_out, m->d_master, m->d_bf, m->stream);
  if (rc) return mfail(m, (th_status)rc, get_error());
  if (hipStreamSynchronize(m->stream) != hipSuccess) return mfail(m, TH_EHIP, "synchronisation failed");
  m->has_weights = true;
  return TH_OK;
}

th_status th_mlp_get_weights(const th_mlp *m, float *theta, int n_params) {
  if (!m || !theta || n_params != mlp_num_params(m->n_out)) return TH_EINVAL;
  if (hipSetDevice(m->device) != hipSuccess) return TH_EHIP;
  if (hipMemcpyAsync(theta, m->d_master, n_params * sizeof(float), hipMemcpyDeviceToHost,
                     m->stream) != hipSuccess ||
      hipStreamSynchronize(m->stream) != hipSuccess)
    return TH_EHIP;
  return TH_OK;
}

th_status th_mlp_set_scaling(th_mlp *m, const double *in_mean, const double *in_std,
                             const double *out_mean, const double *out_std) {
  if (!m || !in_mean || !in_std || !out_mean || !out_std) return TH_EINVAL;
  for (int i = 0; i < 3; ++i)
    if (!(in_std[i] > 0.0)) return mfail(m, TH_EINVAL, "scales must be positive");
  for (int i = 0; i < m->n_out; ++i)
    if (!(out_std[i] > 0.0)) return mfail(m, TH_EINVAL, "scales must be positive");
  std::memcpy(m->in_mean, in_mean, sizeof(m->in_mean));
  std::memcpy(m->in_std, in_std, sizeof(m->in_std));
  std::memcpy(m->out_mean, out_mean, m->n_out * sizeof(double));
  std::memcpy(m->out_std, out_std, m->n_out * sizeof(double));
  return TH_OK;
}

th_status th_mlp_get_scaling(const th_mlp *m, double *in_mean, double *in_std, double *out_mean,
                             double *out_std) {
  if (!m || !in_mean || !in_std || !out_mean || !out_std) return TH_EINVAL;
  std::memcpy(in_mean, m->in_mean, sizeof(m->in_mean));
  std::memcpy(in_std, m->in_std, sizeof(m->in_std));
  std::memcpy(out_mean, m->out_mean, m->n_out * sizeof(double));
  std::memcpy(out_std, m->out_std, m->n_out * sizeof(double));
  return TH_OK;
}

th_status th_mlp_loss_grad(th_mlp *m, const float *x_std, const float *y_std, int n, int bf16,
                           double *loss, float *grad) {
  if (!m) return TH_EINVAL;
  if (!x_std || !y_std || n < 1 || !loss || !grad) return mfail(m, TH_EINVAL, "bad arguments");
  if (!m->has_weights) return mfail(m, TH_ESTATE, "weights not set");
  if (hipSetDevice(m->device) != hipSuccess) return mfail(m, TH_EHIP, "hipSetDevice failed");
  const int P = mlp_num_params(m->n_out);
  const int nblk = (n + 63) / 64;
  const int no = m->n_out;
  DevBuf b;
  float *dx = b.alloc<float>((size_t)n * 3), *dy = b.alloc<float>((size_t)n * no);
  float *gp = b.alloc<float>((size_t)nblk * P), *lp = b.alloc<float>(nblk);
  float *gd = b.alloc<float>(P), *ld = b.alloc<float>(1);
  if (!dx || !dy || !gp || !lp || !gd || !ld) return mfail(m, TH_ENOMEM, "device allocation failed");
  hipStream_t s = m->stream;
  if (hipMemcpyAsync(dx, x_std, (size_t)n * 3 * sizeof(float), hipMemcpyHostToDevice, s) ||
      hipMemcpyAsync(dy, y_std, (size_t)n * no * sizeof(float), hipMemcpyHostToDevice, s))
    return mfail(m, TH_EHIP, "upload failed");
  int rc = mlp_step_launch(no, m->d_master, m->d_bf, bf16 != 0, dx, dy, n, 0, n,
                           1.0f / ((float)no * n), gp, lp, s);
  if (!rc)
    rc = mlp_adam_launch(no, m->d_master, m->d_bf, m->d_m1, m->d_m2, gp, lp, nblk, 0, 0.0f, gd, ld,
                         s);
  if (rc) return mfail(m, (th_status)rc, get_error());
  float lh = 0.0f;
  if (hipMemcpyAsync(grad, gd, P * sizeof(float), hipMemcpyDeviceToHost, s) ||
      hipMemcpyAsync(&lh, ld, sizeof(float), hipMemcpyDeviceToHost, s) ||
      hipStreamSynchronize(s))
    return mfail(m, TH_EHIP, "download failed");
  *loss = lh / ((double)no * n);
  return TH_OK;
}

th_status th_mlp_train(th_mlp *m, const double *samples, int n, const th_mlp_train_opts *o,
                       th_mlp_train_stats *stats) {
  if (!m) return TH_EINVAL;
  if (!o || o->epochs < 1 || o->batch < 64 || o->batch % 64 || !(o->lr > 0.0))
    return mfail(m, TH_EINVAL, "need epochs >= 1, batch a positive multiple of 64, lr > 0");
  std::string msg;
  if (check_samples(samples, n, msg) != TH_OK) return mfail(m, TH_EINVAL, msg);
  if (!m->has_weights) return mfail(m, TH_ESTATE, "initial weights not set");
  if (hipSetDevice(m->device) != hipSuccess) return mfail(m, TH_EHIP, "hipSetDevice failed");
  auto t0 = std::chrono::steady_clock::now();
  const int no = m->n_out;
  std::vector<double> e((size_t)n * no);
  family_errors(no, samples, n, e.data());
  std::vector<double> y((size_t)n * no);
  for (size_t i = 0; i < y.size(); ++i) y[i] = std::log(std::max(-e[i], 0.0) + kEFloor);
  auto t1 = std::chrono::steady_clock::now();
  // standardisation from the samples
  for (int c = 0; c < 3; ++c) {
    double s = 0, s2 = 0;
    for (int i = 0; i < n; ++i) s += samples[3 * i + c];
    const double mu = s / n;
    for (int i = 0; i < n; ++i) s2 += (samples[3 * i + c] - mu) * (samples[3 * i + c] - mu);
    const double sd = std::sqrt(s2 / n);
    m->in_mean[c] = mu;
    m->in_std[c] = sd > 1e-12 ? sd : 1.0;
  }
  for (int c = 0; c < no; ++c) {
    double s = 0, s2 = 0;
    for (int i = 0; i < n; ++i) s += y[(size_t)no * i + c];
    const double mu = s / n;
    for (int i = 0; i < n; ++i) s2 += (y[(size_t)no * i + c] - mu) * (y[(size_t)no * i + c] - mu);
    const double sd = std::sqrt(s2 / n);
    m->out_mean[c] = mu;
    m->out_std[c] = sd > 1e-12 ? sd : 1.0;
  }
  std::vector<float> xs((size_t)n * 3), ys((size_t)n * no);
  for (int i = 0; i < n; ++i) {
    for (int c = 0; c < 3; ++c)
      xs[3 * i + c] = (float)((samples[3 * i + c] - m->in_mean[c]) / m->in_std[c]);
    for (int c = 0; c < no; ++c)
      ys[(size_t)no * i + c] = (float)((y[(size_t)no * i + c] - m->out_mean[c]) / m->out_std[c]);
  }
  const int P = mlp_num_params(m->n_out);
  const int B = std::min(o->batch, (n + 63) / 64 * 64);
  const int nblk = B / 64;
  DevBuf b;
  float *dx = b.alloc<float>((size_t)n * 3), *dy = b.alloc<float>((size_t)n * no);
  float *gp = b.alloc<float>((size_t)nblk * P), *lp = b.alloc<float>(nblk), *ld = b.alloc<float>(1);
  if (!dx || !dy || !gp || !lp || !ld) return mfail(m, TH_ENOMEM, "device allocation failed");
  hipStream_t s = m->stream;
  if (hipMemcpyAsync(dx, xs.data(), xs.size() * sizeof(float), hipMemcpyHostToDevice, s) ||
      hipMemcpyAsync(dy, ys.data(), ys.size() * sizeof(float), hipMemcpyHostToDevice, s) ||
      hipMemsetAsync(m->d_m1, 0, P * sizeof(float), s) || hipMemsetAsync(m->d_m2, 0, P * sizeof(float), s))
    return mfail(m, TH_EHIP, "upload failed");
  const int steps_per_epoch = std::max(1, n / B);
  int step = 0;
  float lfirst = 0.0f, llast = 0.0f;
  const float inv_norm = 1.0f / ((float)no * B);
  for (int ep = 0; ep < o->epochs; ++ep)
    for (int bi = 0; bi < steps_per_epoch; ++bi) {
      const int off = (int)(((long long)bi * B + (long long)ep * 7919) % n);
      int rc = mlp_step_launch(no, m->d_master, m->d_bf, o->bf16 != 0, dx, dy, n, off, B, inv_norm,
                               gp, lp, s);
      if (!rc)
        rc = mlp_adam_launch(no, m->d_master, m->d_bf, m->d_m1, m->d_m2, gp, lp, nblk, ++step,
                             (float)o->lr, nullptr, ld, s);
      if (rc) return mfail(m, (th_status)rc, get_error());
      if (step == 1) {
        if (hipMemcpyAsync(&lfirst, ld, sizeof(float), hipMemcpyDeviceToHost, s) ||
            hipStreamSynchronize(s))
          return mfail(m, TH_EHIP, "download failed");
      }
    }
  if (hipMemcpyAsync(&llast, ld, sizeof(float), hipMemcpyDeviceToHost, s) || hipStreamSynchronize(s))
    return mfail(m, TH_EHIP, "download failed");
  auto t2 = std::chrono::steady_clock::now();
  if (stats) {
    stats->loss_first = lfirst / ((double)no * B);
    stats->loss_last = llast / ((double)no * B);
    stats->steps = step;
    stats->t_targets_s = std::chrono::duration<double>(t1 - t0).count();
    stats->t_train_s = std::chrono::duration<double>(t2 - t1).count();
  }
  return TH_OK;
}

}  // extern "C"

namespace th {

// Device inference: e_out (n x n_out) from raw samples.
int mlp_predict_impl(const th_mlp *m, const double *samples, int n, bool bf16, double *e_out) {
  const int no = m->n_out;
  std::vector<float> xs((size_t)n * 3), ys((size_t)n * no);
  for (int i = 0; i < n; ++i)
    for (int c = 0; c < 3; ++c)
      xs[3 * i + c] = (float)((samples[3 * i + c] - m->in_mean[c]) / m->in_std[c]);
  DevBuf b;
  float *dx = b.alloc<float>((size_t)n * 3), *dy = b.alloc<float>((size_t)n * no);
  if (!dx || !dy) {
    set_error("device allocation failed");
    return TH_ENOMEM;
  }
  hipStream_t s = m->stream;
  TH_HIP_CHECK_RET(hipMemcpyAsync(dx, xs.data(), xs.size() * sizeof(float), hipMemcpyHostToDevice, s));
  int rc = mlp_infer_launch(no, m->d_master, m->d_bf, bf16, dx, dy, n, s);
  if (rc) return rc;
  TH_HIP_CHECK_RET(hipMemcpyAsync(ys.data(), dy, ys.size() * sizeof(float), hipMemcpyDeviceToHost, s));
  TH_HIP_CHECK_RET(hipStreamSynchronize(s));
  for (int i = 0; i < n; ++i)
    for (int c = 0; c < no; ++c) {
      const double yr = ys[(size_t)no * i + c] * m->out_std[c] + m->out_mean[c];
      e_out[(size_t)no * i + c] = -(std::exp(yr) - kEFloor);
    }
  return 0;
}

// Device: network inference, the stencil weights from the predicted errors
// and each stencil's dispersion mismatch (k_stencil.hip); all cells of one
// call share the order p.  q_out: n x 3 (2-D) or n x 4 (3-D), mis: n.
int mlp_stencils_impl(const th_mlp *m, int dim, const double *samples, int n, double *q_out,
                      double *mis) {
  const int no = m->n_out, nq = dim == 3 ? 4 : 3;
  const int p = (int)std::lround(samples[1]);
  for (int i = 0; i < n; ++i)
    if ((int)std::lround(samples[3 * i + 1]) != p) {
      set_error("cells of one problem must share the order");
      return TH_EINVAL;
    }
  std::vector<float> xs((size_t)n * 3);
  for (int i = 0; i < n; ++i)
    for (int c = 0; c < 3; ++c)
      xs[3 * i + c] = (float)((samples[3 * i + c] - m->in_mean[c]) / m->in_std[c]);
  DevBuf b;
  float *dx = b.alloc<float>((size_t)n * 3), *dy = b.alloc<float>((size_t)n * no);
  double *ds = b.alloc<double>((size_t)n * 3), *dq = b.alloc<double>((size_t)n * nq);
  double *dm = b.alloc<double>(n);
  if (!dx || !dy || !ds || !dq || !dm) {
    set_error("device allocation failed");
    return TH_ENOMEM;
  }
  hipStream_t s = m->stream;
  TH_HIP_CHECK_RET(hipMemcpyAsync(dx, xs.data(), xs.size() * sizeof(float), hipMemcpyHostToDevice, s));
  TH_HIP_CHECK_RET(hipMemcpyAsync(ds, samples, (size_t)n * 3 * sizeof(double), hipMemcpyHostToDevice, s));
  int rc = mlp_infer_launch(no, m->d_master, m->d_bf, true, dx, dy, n, s);
  if (!rc) rc = stencil_check_launch(dim, p, ds, dy, n, m->out_mean, m->out_std, kEFloor, dq, dm, s);
  if (rc) return rc;
  TH_HIP_CHECK_RET(hipMemcpyAsync(q_out, dq, (size_t)n * nq * sizeof(double), hipMemcpyDeviceToHost, s));
  TH_HIP_CHECK_RET(hipMemcpyAsync(mis, dm, (size_t)n * sizeof(double), hipMemcpyDeviceToHost, s));
  TH_HIP_CHECK_RET(hipStreamSynchronize(s));
  return 0;
}

// Per-cell weights for the coarse schemes PLAINFIT / MLP of a dim-dimensional
// problem.  samples: n x 3 (eta_c, p, shift); q_out: n x 3 (2-D) or n x 4
// (3-D).  For MLP, the network's stencils are computed and checked on the
// device: a cell whose zero-set mismatch against the fine dispersion curve
// exceeds tau (or is not finite) gets the exact plain fit.
int coarse_weights(int dim, int scheme, const th_mlp *m, double tau, const double *samples, int n,
                   double *q_out, int *n_fallback) {
  *n_fallback = 0;
  const int no = dim == 3 ? 3 : 2, nq = dim == 3 ? 4 : 3;
  auto weights_from = [&](int i, double eta, const double *e) {
    if (dim == 3) {
      const double z[3] = {eta * (1.0 + e[0]), eta * (1.0 + e[1]), eta * (1.0 + e[2])};
      fit27_from_radii(eta, z, q_out + (size_t)nq * i);
    } else {
      fit_from_errors(eta, e, q_out + (size_t)nq * i);
    }
  };
  if (scheme == TH_COARSE_PLAINFIT) {
    if (dim == 3)
      plain_fit27_batch(samples, n, nullptr, q_out);
    else
      plain_fit_batch(samples, n, nullptr, q_out);
    return 0;
  }
  if (!m || m->n_out != no) {
    set_error("the surrogate network's stencil family does not match the problem dimension");
    return TH_EINVAL;
  }
  std::vector<double> mis(n);
  int rc = mlp_stencils_impl(m, dim, samples, n, q_out, mis.data());
  if (rc) return rc;
  std::vector<int> bad;
  for (int i = 0; i < n; ++i)
    if (!(mis[i] <= tau)) bad.push_back(i);
  // exact plain fit for the flagged cells
  if (!bad.empty()) {
    std::vector<double> sb(bad.size() * 3), eb(bad.size() * no);
    for (size_t k = 0; k < bad.size(); ++k)
      for (int c = 0; c < 3; ++c) sb[3 * k + c] = samples[3 * bad[k] + c];
    family_errors(no, sb.data(), (int)bad.size(), eb.data());
    for (size_t k = 0; k < bad.size(); ++k)
      weights_from(bad[k], effective_eta(samples[3 * bad[k]], samples[3 * bad[k] + 2]),
                   &eb[(size_t)no * k]);
  }
  *n_fallback = (int)bad.size();
  return 0;
}

}  // namespace th

extern "C" th_status th_mlp_predict(th_mlp *m, const double *samples, int n, int bf16,
                                    double *e_out) {
  if (!m) return TH_EINVAL;
  std::string msg;
  if (check_samples(samples, n, msg) != TH_OK) return mfail(m, TH_EINVAL, msg);
  if (!e_out) return mfail(m, TH_EINVAL, "e_out is NULL");
  if (!m->has_weights) return mfail(m, TH_ESTATE, "weights not set");
  if (hipSetDevice(m->device) != hipSuccess) return mfail(m, TH_EHIP, "hipSetDevice failed");
  int rc = mlp_predict_impl(m, samples, n, bf16 != 0, e_out);
  if (rc) return mfail(m, (th_status)rc, get_error());
  return TH_OK;
}

extern "C" th_status th_mlp_stencils(th_mlp *m, const double *samples, int n, double *q_out,
                                     double *mismatch_out) {
  if (!m) return TH_EINVAL;
  std::string msg;
  if (check_samples(samples, n, msg) != TH_OK) return mfail(m, TH_EINVAL, msg);
  if (!q_out || !mismatch_out) return mfail(m, TH_EINVAL, "output array is NULL");
  if (!m->has_weights) return mfail(m, TH_ESTATE, "weights not set");
  if (hipSetDevice(m->device) != hipSuccess) return mfail(m, TH_EHIP, "hipSetDevice failed");
  int rc = mlp_stencils_impl(m, m->n_out == 3 ? 3 : 2, samples, n, q_out, mismatch_out);
  if (rc) return mfail(m, (th_status)rc, get_error());
  return TH_OK;
}
