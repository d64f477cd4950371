// Vector kernels of the outer FP64 Krylov method and precision conversions.
// Reductions are two-pass with a fixed tree, so every result is bitwise
// reproducible (no atomics).
#include "ctx.hpp"

namespace th {

constexpr int RED_BLOCKS = 256;

__device__ __forceinline__ void block_reduce(c64 *sh, c64 v) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] = sh[threadIdx.x] + sh[threadIdx.x + w];
    __syncthreads();
  }
}

// partial[rhs][block] = sum over the block's slice of conj(x) y
__global__ __launch_bounds__(256) void k_dot_partial(const c64 *__restrict__ x,
                                                     const c64 *__restrict__ y, long long n,
                                                     long long ldx, long long ldy,
                                                     c64 *__restrict__ partial) {
  __shared__ c64 sh[256];
  const long long rhs = blockIdx.y;
  x += rhs * ldx;
  y += rhs * ldy;
  c64 acc = {0, 0};
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
    const c64 a = x[i], b = y[i];
    acc.re = fma(a.re, b.re, acc.re);
    acc.re = fma(a.im, b.im, acc.re);
    acc.im = fma(a.re, b.im, acc.im);
    acc.im = fma(-a.im, b.re, acc.im);
  }
  block_reduce(sh, acc);
  if (threadIdx.x == 0) partial[rhs * RED_BLOCKS + blockIdx.x] = sh[0];
}

// out[rhs] = the sum of the rhs's nb partials (fixed order)
__global__ __launch_bounds__(256) void k_dot_final(const c64 *__restrict__ partial, int nb,
                                                   c64 *__restrict__ out) {
  __shared__ c64 sh[256];
  block_reduce(sh, (int)threadIdx.x < nb ? partial[blockIdx.x * RED_BLOCKS + threadIdx.x]
                                         : c64{0, 0});
  if (threadIdx.x == 0) out[blockIdx.x] = sh[0];
}

// Partial blocks per right-hand side: enough for 8 entries per thread, at most
// RED_BLOCKS (short vectors with many right-hand sides, such as 64 of 16,641
// entries, would otherwise launch mostly idle blocks)
static int dot_blocks(long long n) {
  return (int)std::max<long long>(1, std::min<long long>(RED_BLOCKS, ceil_div_ll(n, 256 * 8)));
}

int launch_dot(const c64 *x, const c64 *y, long long n, int nrhs, long long ldx, long long ldy,
               c64 *out, c64 *partial, hipStream_t s) {
  const int nb = dot_blocks(n);
  hipLaunchKernelGGL(k_dot_partial, dim3(nb, nrhs), dim3(256), 0, s, x, y, n, ldx, ldy, partial);
  hipLaunchKernelGGL(k_dot_final, dim3(nrhs), dim3(RED_BLOCKS), 0, s, (const c64 *)partial, nb, out);
  TH_HIP_CHECK_RET(hipGetLastError());
  return 0;
}

int launch_dot_partial(const c64 *x, const c64 *y, long long n, int nrhs, long long ldx,
                       long long ldy, c64 *partial, hipStream_t s) {
  hipLaunchKernelGGL(k_dot_partial, dim3(dot_blocks(n), nrhs), dim3(256), 0, s, x, y, n, ldx, ldy,
                     partial);
  TH_HIP_CHECK_RET(hipGetLastError());
  return 0;
}

// The dot product of right-hand side r from its partials, in the same fixed
// order as k_dot_final (every block of the caller computes it)
__device__ __forceinline__ c64 dot_from_partials(const c64 *__restrict__ partial, int nb, int r,
                                                 c64 *sh) {
  block_reduce(sh, (int)threadIdx.x < nb ? partial[r * RED_BLOCKS + threadIdx.x] : c64{0, 0});
  return sh[0];
}

// y[rhs] += sign * a x[rhs] with a = conj(x_i) . y from the partials of
// k_dot_partial; block 0 stores a in coef[rhs]
__global__ __launch_bounds__(256) void k_axpy_partials(c64 *__restrict__ y,
                                                       const c64 *__restrict__ x,
                                                       const c64 *__restrict__ partial, int nb,
                                                       c64 *__restrict__ coef, double sign,
                                                       long long n, long long ldy, long long ldx) {
  __shared__ c64 sh[256];
  const long long rhs = blockIdx.y;
  const c64 a = dot_from_partials(partial, nb, (int)rhs, sh);
  if (blockIdx.x == 0 && threadIdx.x == 0) coef[rhs] = a;
  const c64 sa = {sign * a.re, sign * a.im};
  y += rhs * ldy;
  x += rhs * ldx;
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
    c64 v = y[i];
    cmac(v, sa, x[i]);
    y[i] = v;
  }
}

int launch_axpy_partials(c64 *y, const c64 *x, const c64 *partial, c64 *coef, double sign,
                         long long n, int nrhs, long long ldy, long long ldx, hipStream_t s) {
  const int blocks = (int)std::min<long long>(ceil_div_ll(n, 256), 4096);
  hipLaunchKernelGGL(k_axpy_partials, dim3(blocks, nrhs), dim3(256), 0, s, y, x, partial,
                     dot_blocks(n), coef, sign, n, ldy, ldx);
  TH_HIP_CHECK_RET(hipGetLastError());
  return 0;
}

// y[rhs] += sign * a x[rhs] as k_axpy_partials, then the partial dot products
// conj(z) . y of the updated y for the next projection (z = y: its squared
// norm), over k_dot_partial's block partition (grid dot_blocks(n) x nrhs) and
// in its element order, so the partials are the bits a separate k_dot_partial
// would give: one launch and one vector pass fewer per projection.
__global__ __launch_bounds__(256) void k_axpy_dot_partials(c64 *__restrict__ y,
                                                           const c64 *__restrict__ x,
                                                           const c64 *z, int z_is_y,
                                                           const c64 *__restrict__ pin, int nb,
                                                           c64 *__restrict__ coef, double sign,
                                                           long long n, long long ld,
                                                           c64 *__restrict__ pout) {
  __shared__ c64 sh[256];
  const long long rhs = blockIdx.y;
  const c64 a = dot_from_partials(pin, nb, (int)rhs, sh);
  __syncthreads();  // every thread holds a before sh is reused
  if (blockIdx.x == 0 && threadIdx.x == 0) coef[rhs] = a;
  const c64 sa = {sign * a.re, sign * a.im};
  y += rhs * ld;
  x += rhs * ld;
  z += rhs * ld;
  c64 acc = {0, 0};
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
    c64 v = y[i];
    cmac(v, sa, x[i]);
    y[i] = v;
    const c64 q = z_is_y ? v : z[i];
    acc.re = fma(q.re, v.re, acc.re);
    acc.re = fma(q.im, v.im, acc.re);
    acc.im = fma(q.re, v.im, acc.im);
    acc.im = fma(-q.im, v.re, acc.im);
  }
  block_reduce(sh, acc);
  if (threadIdx.x == 0) pout[rhs * RED_BLOCKS + blockIdx.x] = sh[0];
}

int launch_axpy_dot_partials(c64 *y, const c64 *x, const c64 *z, const c64 *pin, c64 *coef,
                             double sign, long long n, int nrhs, long long ld, c64 *pout,
                             hipStream_t s) {
  const int nb = dot_blocks(n);
  hipLaunchKernelGGL(k_axpy_dot_partials, dim3(nb, nrhs), dim3(256), 0, s, y, x, z,
                     z == y ? 1 : 0, pin, nb, coef, sign, n, ld, pout);
  TH_HIP_CHECK_RET(hipGetLastError());
  return 0;
}

// v[rhs] /= ||v[rhs]|| with ||v||^2 from the partials of k_dot_partial (0 when
// the norm is zero or not finite, as k_inv_norm); block 0 stores ||v||^2 in
// dot[rhs]
__global__ __launch_bounds__(256) void k_scale_partials(c64 *__restrict__ v,
                                                        const c64 *__restrict__ partial, int nb,
                                                        c64 *__restrict__ dot, long long n,
                                                        long long ld) {
  __shared__ c64 sh[256];
  const long long rhs = blockIdx.y;
  const c64 a = dot_from_partials(partial, nb, (int)rhs, sh);
  if (blockIdx.x == 0 && threadIdx.x == 0) dot[rhs] = a;
  const double nrm = sqrt(a.re > 0.0 ? a.re : 0.0);
  const double inv = (nrm > 0.0 && isfinite(nrm)) ? 1.0 / nrm : 0.0;
  v += rhs * ld;
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
    const c64 e = v[i];
    v[i] = c64{inv * e.re, inv * e.im};
  }
}

int launch_scale_partials(c64 *v, const c64 *partial, c64 *dot, long long n, int nrhs,
                          long long ld, hipStream_t s) {
  const int blocks = (int)std::min<long long>(ceil_div_ll(n, 256), 4096);
  hipLaunchKernelGGL(k_scale_partials, dim3(blocks, nrhs), dim3(256), 0, s, v, partial,
                     dot_blocks(n), dot, n, ld);
  TH_HIP_CHECK_RET(hipGetLastError());
  return 0;
}

// One whole modified Gram-Schmidt step of the Arnoldi process for vectors of
// at most 1024 K entries: one workgroup per right-hand side keeps its new
// vector w in registers (K entries per thread) and, for i = 0 .. nv - 1 in
// order, forms h_i = conj(V_i) . w (a fixed-order workgroup sum), stores it in
// hcol[i][rhs] and subtracts h_i V_i (V_i read a second time, from L2); then
// ||w||^2 goes to hcol[nv][rhs] and w / ||w|| (0 when the norm is zero or
// not finite, as k_scale_partials) back to w.  Every step is deterministic;
// the vectors pass through memory about half as often as with a launch per
// projection, and the step is one launch instead of 2 nv + 2.
constexpr int kMgsThreads = 1024;

__device__ __forceinline__ c64 mgs_block_sum(c64 v, c64 *red, c64 *out) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    v.re += __shfl_xor(v.re, o, 64);
    v.im += __shfl_xor(v.im, o, 64);
  }
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) red[wave] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    c64 t = red[0];
    for (int q = 1; q < kMgsThreads / 64; ++q) t = t + red[q];
    *out = t;
  }
  __syncthreads();
  return *out;
}

template <int K>
__global__ __launch_bounds__(kMgsThreads) void k_mgs_step(MgsBasis B, int nv,
                                                          c64 *__restrict__ w,
                                                          c64 *__restrict__ hcol, long long n,
                                                          long long ld, int nrhs) {
  __shared__ c64 red[kMgsThreads / 64];
  __shared__ c64 bc;
  const int rhs = blockIdx.x;
  const long long off = (long long)rhs * ld;
  c64 x[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const long long i = threadIdx.x + (long long)k * kMgsThreads;
    x[k] = i < n ? w[off + i] : c64{0, 0};
  }
  for (int p = 0; p < nv; ++p) {
    const c64 *__restrict__ v = B.v[p] + off;
    c64 acc = {0, 0};
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const long long i = threadIdx.x + (long long)k * kMgsThreads;
      if (i < n) {
        const c64 a = v[i], b = x[k];
        acc.re = fma(a.re, b.re, acc.re);
        acc.re = fma(a.im, b.im, acc.re);
        acc.im = fma(a.re, b.im, acc.im);
        acc.im = fma(-a.im, b.re, acc.im);
      }
    }
    const c64 h = mgs_block_sum(acc, red, &bc);
    if (threadIdx.x == 0) hcol[(long long)p * nrhs + rhs] = h;
    const c64 sa = {-h.re, -h.im};
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const long long i = threadIdx.x + (long long)k * kMgsThreads;
      if (i < n) cmac(x[k], sa, v[i]);
    }
  }
  c64 acc = {0, 0};
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const c64 b = x[k];
    acc.re = fma(b.re, b.re, acc.re);
    acc.re = fma(b.im, b.im, acc.re);
    acc.im = fma(b.re, b.im, acc.im);
    acc.im = fma(-b.im, b.re, acc.im);
  }
  const c64 a = mgs_block_sum(acc, red, &bc);
  if (threadIdx.x == 0) hcol[(long long)nv * nrhs + rhs] = a;
  const double nrm = sqrt(a.re > 0.0 ? a.re : 0.0);
  const double inv = (nrm > 0.0 && isfinite(nrm)) ? 1.0 / nrm : 0.0;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const long long i = threadIdx.x + (long long)k * kMgsThreads;
    if (i < n) w[off + i] = c64{inv * x[k].re, inv * x[k].im};
  }
}

bool mgs_step_fits(long long n, int nrhs, int nv) {
  return nrhs >= kMgsMinRhs && nv <= kMgsMax && n <= (long long)kMgsThreads * 18;
}

int launch_mgs_step(const MgsBasis &B, int nv, c64 *w, c64 *hcol, long long n, int nrhs,
                     long long ld, hipStream_t s) {
  if (!mgs_step_fits(n, nrhs, nv)) {
    set_error("launch_mgs_step: vector too long, too few right-hand sides or too many projections");
    return TH_EINVAL;
  }
  const int K = (int)ceil_div_ll(n, kMgsThreads);
  const dim3 g(nrhs), b(kMgsThreads);
  if (K <= 4)
    hipLaunchKernelGGL(k_mgs_step<4>, g, b, 0, s, B, nv, w, hcol, n, ld, nrhs);
  else if (K <= 8)
    hipLaunchKernelGGL(k_mgs_step<8>, g, b, 0, s, B, nv, w, hcol, n, ld, nrhs);
  else if (K <= 12)
    hipLaunchKernelGGL(k_mgs_step<12>, g, b, 0, s, B, nv, w, hcol, n, ld, nrhs);
  else if (K <= 16)
    hipLaunchKernelGGL(k_mgs_step<16>, g, b, 0, s, B, nv, w, hcol, n, ld, nrhs);
  else
    hipLaunchKernelGGL(k_mgs_step<18>, g, b, 0, s, B, nv, w, hcol, n, ld, nrhs);
  TH_HIP_CHECK_RET(hipGetLastError());
  return 0;
}

// y[rhs] += sign * coef[rhs] * x[rhs]
__global__ __launch_bounds__(256) void k_axpy_dev(c64 *__restrict__ y, const c64 *__restrict__ x,
                                                  const c64 *__restrict__ coef, double sign,
                                                  long long n, long long ldy, long long ldx) {
  const long long rhs = blockIdx.y;
  const c64 a = coef[rhs];
  const c64 sa = {sign * a.re, sign * a.im};
  y += rhs * ldy;
  x += rhs * ldx;
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
    c64 v = y[i];
    cmac(v, sa, x[i]);
    y[i] = v;
  }
}

int launch_axpy_dev(c64 *y, const c64 *x, const c64 *coef, double sign, long long n, int nrhs,
                    long long ldy, long long ldx, hipStream_t s) {
  int blocks = (int)std::min<long long>(ceil_div_ll(n, 256), 4096);
  hipLaunchKernelGGL(k_axpy_dev, dim3(blocks, nrhs), dim3(256), 0, s, y, x, coef, sign, n, ldy,
                     ldx);
  TH_HIP_CHECK_RET(hipGetLastError());
  return 0;
}

// y[rhs] = x[rhs] * s[rhs]  (s real, from a device array)
__global__ __launch_bounds__(256) void k_scale_dev(c64 *__restrict__ y, const c64 *__restrict__ x,
                                                   const double *__restrict__ sc, long long n,
                                                   long long ldy, long long ldx) {
  const long long rhs = blockIdx.y;
  const double a = sc[rhs];
  y += rhs * ldy;
  x += rhs * ldx;
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
    const c64 v = x[i];
    y[i] = c64{a * v.re, a * v.im};
  }
}

int launch_scale_dev(c64 *y, const c64 *x, const double *inv_norm, long long n, int nrhs,
                     long long ldy, long long ldx, hipStream_t s) {
  int blocks = (int)std::min<long long>(ceil_div_ll(n, 256), 4096);
  hipLaunchKernelGGL(k_scale_dev, dim3(blocks, nrhs), dim3(256), 0, s, y, x, inv_norm, n, ldy, ldx);
  TH_HIP_CHECK_RET(hipGetLastError());
  return 0;
}

// x[rhs] += sum_j coef[rhs][j] Z[j][rhs]   (Z block j at Z + j*ldz_j + rhs*ldz_r)
__global__ __launch_bounds__(256) void k_lincomb(c64 *__restrict__ x, const c64 *__restrict__ Z,
                                                 const c64 *__restrict__ coef, int m, int cstride,
                                                 long long n, long long ldz_j, long long ldz_r) {
  const long long rhs = blockIdx.y;
  x += rhs * n;
  const c64 *cf = coef + rhs * cstride;
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
    c64 acc = x[i];
    for (int j = 0; j < m; ++j) cmac(acc, cf[j], Z[j * ldz_j + rhs * ldz_r + i]);
    x[i] = acc;
  }
}

int launch_lincomb(c64 *x, const c64 *Z, const c64 *coef, int mcount, int cstride, long long n,
                   int nrhs, long long ldz_j, long long ldz_r, hipStream_t s) {
  int blocks = (int)std::min<long long>(ceil_div_ll(n, 256), 4096);
  hipLaunchKernelGGL(k_lincomb, dim3(blocks, nrhs), dim3(256), 0, s, x, Z, coef, mcount, cstride,
                     n, ldz_j, ldz_r);
  TH_HIP_CHECK_RET(hipGetLastError());
  return 0;
}

template <typename Ti, typename To>
__global__ __launch_bounds__(256) void k_convert(const Ti *__restrict__ in, To *__restrict__ out,
                                                 long long n) {
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += (long long)gridDim.x * 256)
    out[i] = (To)in[i];
}

int launch_convert(const void *in, void *out, long long n_complex, bool in_f32, bool out_f32,
                   hipStream_t s) {
  const long long n = 2 * n_complex;
  int blocks = (int)std::min<long long>(ceil_div_ll(n, 256), 8192);
  if (in_f32 && !out_f32)
    hipLaunchKernelGGL((k_convert<float, double>), dim3(blocks), dim3(256), 0, s,
                       (const float *)in, (double *)out, n);
  else if (!in_f32 && out_f32)
    hipLaunchKernelGGL((k_convert<double, float>), dim3(blocks), dim3(256), 0, s,
                       (const double *)in, (float *)out, n);
  else if (in_f32)
    hipLaunchKernelGGL((k_convert<float, float>), dim3(blocks), dim3(256), 0, s,
                       (const float *)in, (float *)out, n);
  else
    hipLaunchKernelGGL((k_convert<double, double>), dim3(blocks), dim3(256), 0, s,
                       (const double *)in, (double *)out, n);
  TH_HIP_CHECK_RET(hipGetLastError());
  return 0;
}

// u += v (complex, either precision)
template <typename T>
__global__ __launch_bounds__(256) void k_add(T *__restrict__ u, const T *__restrict__ v,
                                             long long n) {
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += (long long)gridDim.x * 256)
    u[i] += v[i];
}

int launch_add(void *u, const void *v, long long n_complex, bool f32, hipStream_t s) {
  const long long n = 2 * n_complex;
  int blocks = (int)std::min<long long>(ceil_div_ll(n, 256), 8192);
  if (f32)
    hipLaunchKernelGGL((k_add<float>), dim3(blocks), dim3(256), 0, s, (float *)u,
                       (const float *)v, n);
  else
    hipLaunchKernelGGL((k_add<double>), dim3(blocks), dim3(256), 0, s, (double *)u,
                       (const double *)v, n);
  TH_HIP_CHECK_RET(hipGetLastError());
  return 0;
}

// inv[r] = 1 / sqrt(Re dots[r]) (0 when the norm is zero or not finite)
__global__ void k_inv_norm(const c64 *__restrict__ dots, double *__restrict__ inv, int n) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n) {
    const double v = dots[r].re;
    const double nrm = sqrt(v > 0.0 ? v : 0.0);
    inv[r] = (nrm > 0.0 && isfinite(nrm)) ? 1.0 / nrm : 0.0;
  }
}

int launch_inv_norm(const c64 *dots, double *inv, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_inv_norm, dim3(ceil_div(n, 64)), dim3(64), 0, s, dots, inv, n);
  TH_HIP_CHECK_RET(hipGetLastError());
  return 0;
}

// flag = 1 if any entry is not finite
__global__ __launch_bounds__(256) void k_nan_check(const c64 *__restrict__ x, long long n,
                                                   int *flag) {
  bool bad = false;
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
    const c64 v = x[i];
    bad |= !isfinite(v.re) || !isfinite(v.im);
  }
  if (bad) flag[0] = 1;
}

int launch_nan_check(const c64 *x, long long n, int *flag, hipStream_t s) {
  int blocks = (int)std::min<long long>(ceil_div_ll(n, 256), 1024);
  hipLaunchKernelGGL(k_nan_check, dim3(blocks), dim3(256), 0, s, x, n, flag);
  TH_HIP_CHECK_RET(hipGetLastError());
  return 0;
}

}  // namespace th
