// Coarse-stencil surrogate network on the device: 3 -> 64 -> 64 -> NOUT MLP
// with SiLU activations (a project addition that replaces the per-cell
// dispersion root finding of the plain fit by inference); NOUT = 2 for the
// 9-point family, 3 for the 27-point family.
//
// Training step (k_mlp_step): a workgroup takes 64 samples, keeps the weights
// (FP32, or the BF16 copy widened to FP32) and every activation in LDS, runs
// the forward pass, the mean-squared-error loss and the backward pass as small
// LDS GEMMs, and writes its gradient partial sum; k_mlp_adam sums the
// partials in a fixed order (deterministic), applies Adam to the FP32 master
// weights and refreshes the BF16 copy.  Inference (k_mlp_infer) runs one
// sample per thread with the weights in LDS.  Accumulation is FP32 throughout.
#include "ctx.hpp"

namespace th {

constexpr int MLP_IN = 3, MLP_W = 64, MLP_S = 64;
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + MLP_W * MLP_IN, OFF_W2 = OFF_B1 + MLP_W,
              OFF_B2 = OFF_W2 + MLP_W * MLP_W, OFF_W3 = OFF_B2 + MLP_W;
template <int NOUT> struct MlpShape {
  static constexpr int B3 = OFF_W3 + NOUT * MLP_W, P = B3 + NOUT;
};

int mlp_num_params(int n_out) { return OFF_W3 + n_out * (MLP_W + 1); }

__device__ __forceinline__ float bf2f(unsigned short b) {
  return __uint_as_float(((unsigned int)b) << 16);
}
__device__ __forceinline__ unsigned short f2bf_rne(float x) {
  unsigned int u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float sigm(float a) { return 1.0f / (1.0f + expf(-a)); }

template <int MLP_OUT>
__global__ __launch_bounds__(256) void k_mlp_step(const float *__restrict__ master,
                                                  const unsigned short *__restrict__ wbf, int use_bf16,
                                                  const float *__restrict__ x,
                                                  const float *__restrict__ t, int n, int off,
                                                  int count, float inv_norm,
                                                  float *__restrict__ gpart,
                                                  float *__restrict__ lpart) {
  constexpr int MLP_P = MlpShape<MLP_OUT>::P, OFF_B3 = MlpShape<MLP_OUT>::B3;
  __shared__ float W[MLP_P];
  __shared__ float X[MLP_S][MLP_IN];
  __shared__ float A1[MLP_S][MLP_W], H1[MLP_S][MLP_W], A2[MLP_S][MLP_W], H2[MLP_S][MLP_W];
  __shared__ float D[MLP_S][MLP_OUT];
  __shared__ float G[MLP_S][MLP_W];  // reused: dA2, then dA1
  __shared__ float red[256];
  const int tid = threadIdx.x;
  const int s0 = blockIdx.x * MLP_S;
  for (int i = tid; i < MLP_P; i += 256) W[i] = use_bf16 ? bf2f(wbf[i]) : master[i];
  for (int i = tid; i < MLP_S * MLP_IN; i += 256) {
    const int s = i / MLP_IN, c = i % MLP_IN;
    const int g = s0 + s;
    X[s][c] = (g < count) ? x[(long long)((off + g) % n) * MLP_IN + c] : 0.0f;
  }
  __syncthreads();
  // layer 1
  for (int i = tid; i < MLP_S * MLP_W; i += 256) {
    const int s = i / MLP_W, j = i % MLP_W;
    float a = W[OFF_B1 + j];
    for (int c = 0; c < MLP_IN; ++c) a = fmaf(W[OFF_W1 + j * MLP_IN + c], X[s][c], a);
    A1[s][j] = a;
    H1[s][j] = a * sigm(a);
  }
  __syncthreads();
  // layer 2
  for (int i = tid; i < MLP_S * MLP_W; i += 256) {
    const int s = i / MLP_W, j = i % MLP_W;
    float a = W[OFF_B2 + j];
    for (int k = 0; k < MLP_W; ++k) a = fmaf(W[OFF_W2 + j * MLP_W + k], H1[s][k], a);
    A2[s][j] = a;
    H2[s][j] = a * sigm(a);
  }
  __syncthreads();
  // output layer, loss and dL/dy
  float lsum = 0.0f;
  if (tid < MLP_S * MLP_OUT) {
    const int s = tid / MLP_OUT, o = tid % MLP_OUT;
    float y = W[OFF_B3 + o];
    for (int k = 0; k < MLP_W; ++k) y = fmaf(W[OFF_W3 + o * MLP_W + k], H2[s][k], y);
    const int g = s0 + s;
    float d = 0.0f;
    if (g < count) d = y - t[(long long)((off + g) % n) * MLP_OUT + o];
    lsum = d * d;
    D[s][o] = 2.0f * d * inv_norm;
  }
  red[tid] = lsum;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  float *gp = gpart + (long long)blockIdx.x * MLP_P;
  if (tid == 0) lpart[blockIdx.x] = red[0];
  // grads of the output layer
  for (int i = tid; i < MLP_OUT * MLP_W + MLP_OUT; i += 256) {
    if (i < MLP_OUT * MLP_W) {
      const int o = i / MLP_W, k = i % MLP_W;
      float g = 0.0f;
      for (int s = 0; s < MLP_S; ++s) g = fmaf(D[s][o], H2[s][k], g);
      gp[OFF_W3 + i] = g;
    } else {
      const int o = i - MLP_OUT * MLP_W;
      float g = 0.0f;
      for (int s = 0; s < MLP_S; ++s) g += D[s][o];
      gp[OFF_B3 + o] = g;
    }
  }
  // dA2 = (W3^T D) * silu'(A2)
  for (int i = tid; i < MLP_S * MLP_W; i += 256) {
    const int s = i / MLP_W, k = i % MLP_W;
    float d = 0.0f;
    for (int o = 0; o < MLP_OUT; ++o) d = fmaf(W[OFF_W3 + o * MLP_W + k], D[s][o], d);
    const float a = A2[s][k], sg = sigm(a);
    G[s][k] = d * sg * (1.0f + a * (1.0f - sg));
  }
  __syncthreads();
  for (int i = tid; i < MLP_W * MLP_W + MLP_W; i += 256) {
    if (i < MLP_W * MLP_W) {
      const int j = i / MLP_W, k = i % MLP_W;
      float g = 0.0f;
      for (int s = 0; s < MLP_S; ++s) g = fmaf(G[s][j], H1[s][k], g);
      gp[OFF_W2 + i] = g;
    } else {
      const int j = i - MLP_W * MLP_W;
      float g = 0.0f;
      for (int s = 0; s < MLP_S; ++s) g += G[s][j];
      gp[OFF_B2 + j] = g;
    }
  }
  // dA1 = (W2^T dA2) * silu'(A1), written to H2 (no longer needed)
  for (int i = tid; i < MLP_S * MLP_W; i += 256) {
    const int s = i / MLP_W, k = i % MLP_W;
    float d = 0.0f;
    for (int j = 0; j < MLP_W; ++j) d = fmaf(W[OFF_W2 + j * MLP_W + k], G[s][j], d);
    const float a = A1[s][k], sg = sigm(a);
    H2[s][k] = d * sg * (1.0f + a * (1.0f - sg));
  }
  __syncthreads();
  for (int i = tid; i < MLP_W * MLP_IN + MLP_W; i += 256) {
    if (i < MLP_W * MLP_IN) {
      const int j = i / MLP_IN, c = i % MLP_IN;
      float g = 0.0f;
      for (int s = 0; s < MLP_S; ++s) g = fmaf(H2[s][j], X[s][c], g);
      gp[OFF_W1 + i] = g;
    } else {
      const int j = i - MLP_W * MLP_IN;
      float g = 0.0f;
      for (int s = 0; s < MLP_S; ++s) g += H2[s][j];
      gp[OFF_B1 + j] = g;
    }
  }
}

// Fixed-order reduction of the partials; Adam on the FP32 master weights
// (step >= 1), or only the reduced gradient (step == 0).
template <int MLP_OUT>
__global__ __launch_bounds__(256) void k_mlp_adam(float *__restrict__ master,
                                                  unsigned short *__restrict__ wbf,
                                                  float *__restrict__ m1, float *__restrict__ m2,
                                                  const float *__restrict__ gpart,
                                                  const float *__restrict__ lpart, int nblk,
                                                  int step, float lr, float *__restrict__ grad_out,
                                                  float *__restrict__ loss_out) {
  constexpr int MLP_P = MlpShape<MLP_OUT>::P;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) {
    float l = 0.0f;
    for (int b = 0; b < nblk; ++b) l += lpart[b];
    loss_out[0] = l;
  }
  if (i >= MLP_P) return;
  float g = 0.0f;
  for (int b = 0; b < nblk; ++b) g += gpart[(long long)b * MLP_P + i];
  if (grad_out) grad_out[i] = g;
  if (step <= 0) return;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float a = b1 * m1[i] + (1.0f - b1) * g;
  const float v = b2 * m2[i] + (1.0f - b2) * g * g;
  m1[i] = a;
  m2[i] = v;
  const float mh = a / (1.0f - powf(b1, (float)step));
  const float vh = v / (1.0f - powf(b2, (float)step));
  const float w = master[i] - lr * mh / (sqrtf(vh) + eps);
  master[i] = w;
  wbf[i] = f2bf_rne(w);
}

template <int MLP_OUT>
__global__ __launch_bounds__(256) void k_mlp_infer(const float *__restrict__ master,
                                                   const unsigned short *__restrict__ wbf,
                                                   int use_bf16, const float *__restrict__ x,
                                                   float *__restrict__ y, int n) {
  constexpr int MLP_P = MlpShape<MLP_OUT>::P, OFF_B3 = MlpShape<MLP_OUT>::B3;
  __shared__ float W[MLP_P];
  for (int i = threadIdx.x; i < MLP_P; i += blockDim.x) W[i] = use_bf16 ? bf2f(wbf[i]) : master[i];
  __syncthreads();
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  float xi[MLP_IN], h1[MLP_W];
  for (int c = 0; c < MLP_IN; ++c) xi[c] = x[(long long)s * MLP_IN + c];
#pragma unroll 8
  for (int j = 0; j < MLP_W; ++j) {
    float a = W[OFF_B1 + j];
    for (int c = 0; c < MLP_IN; ++c) a = fmaf(W[OFF_W1 + j * MLP_IN + c], xi[c], a);
    h1[j] = a * sigm(a);
  }
  float out[MLP_OUT];
  for (int o = 0; o < MLP_OUT; ++o) out[o] = W[OFF_B3 + o];
  for (int j = 0; j < MLP_W; ++j) {
    float a = W[OFF_B2 + j];
#pragma unroll 16
    for (int k = 0; k < MLP_W; ++k) a = fmaf(W[OFF_W2 + j * MLP_W + k], h1[k], a);
    const float h = a * sigm(a);
    for (int o = 0; o < MLP_OUT; ++o) out[o] = fmaf(W[OFF_W3 + o * MLP_W + j], h, out[o]);
  }
  for (int o = 0; o < MLP_OUT; ++o) y[(long long)s * MLP_OUT + o] = out[o];
}

// --------------------------------------------------------------------------
int mlp_step_launch(int n_out, const float *master, const unsigned short *wbf, bool bf16,
                    const float *x, const float *t, int n, int off, int count, float inv_norm,
                    float *gpart, float *lpart, hipStream_t s) {
  const int nblk = ceil_div(count, MLP_S);
  if (n_out == 3)
    hipLaunchKernelGGL(k_mlp_step<3>, dim3(nblk), dim3(256), 0, s, master, wbf, bf16 ? 1 : 0, x,
                       t, n, off, count, inv_norm, gpart, lpart);
  else
    hipLaunchKernelGGL(k_mlp_step<2>, dim3(nblk), dim3(256), 0, s, master, wbf, bf16 ? 1 : 0, x,
                       t, n, off, count, inv_norm, gpart, lpart);
  TH_HIP_CHECK_RET(hipGetLastError());
  return 0;
}

int mlp_adam_launch(int n_out, float *master, unsigned short *wbf, float *m1, float *m2,
                    const float *gpart, const float *lpart, int nblk, int step, float lr,
                    float *grad_out, float *loss_out, hipStream_t s) {
  const unsigned g = (unsigned)ceil_div(mlp_num_params(n_out), 256);
  if (n_out == 3)
    hipLaunchKernelGGL(k_mlp_adam<3>, dim3(g), dim3(256), 0, s, master, wbf, m1, m2, gpart, lpart,
                       nblk, step, lr, grad_out, loss_out);
  else
    hipLaunchKernelGGL(k_mlp_adam<2>, dim3(g), dim3(256), 0, s, master, wbf, m1, m2, gpart, lpart,
                       nblk, step, lr, grad_out, loss_out);
  TH_HIP_CHECK_RET(hipGetLastError());
  return 0;
}

int mlp_infer_launch(int n_out, const float *master, const unsigned short *wbf, bool bf16,
                     const float *x, float *y, int n, hipStream_t s) {
  if (n_out == 3)
    hipLaunchKernelGGL(k_mlp_infer<3>, dim3(ceil_div(n, 256)), dim3(256), 0, s, master, wbf,
                       bf16 ? 1 : 0, x, y, n);
  else
    hipLaunchKernelGGL(k_mlp_infer<2>, dim3(ceil_div(n, 256)), dim3(256), 0, s, master, wbf,
                       bf16 ? 1 : 0, x, y, n);
  TH_HIP_CHECK_RET(hipGetLastError());
  return 0;
}

__global__ void k_f2bf(const float *__restrict__ a, unsigned short *__restrict__ b, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = f2bf_rne(a[i]);
}

int mlp_refresh_bf16(int n_out, const float *master, unsigned short *wbf, hipStream_t s) {
  const int P = mlp_num_params(n_out);
  hipLaunchKernelGGL(k_f2bf, dim3(ceil_div(P, 256)), dim3(256), 0, s, master, wbf, P);
  TH_HIP_CHECK_RET(hipGetLastError());
  return 0;
}

}  // namespace th
