// Complex-shifted domain-decomposition smoother, apply phase (Alg. 2).
//
// With n_dd = 1 and v = 0 the DD step gives w_i = (A_s^(i))^{-1} R_i r for every
// subdomain, and the averaged update (eq. RAS_like_update) sets
//   v_j = (1/L_j) sum_{i : j in Dofs(U^(i))} (w_i)_j .
// Setup stores B_i = diag(1/L_j) R_{U_i} (A_s^(i))^{-1} (n_U x n_Omega; the
// weights 1/L_j in {1, 1/2, 1/4, 1/8} are exact powers of two), so the apply is
//   gather  X_i = R_{Omega_i} r            (structured box, no index maps)
//   GEMV    Y_i = B_i X_i                  (k_dd_apply: streams B_i once)
//   gather  v_j = sum_i (Y_i)_j            (k_dd_accumulate: fixed order)
// B_i is stored in blocks of 64 rows (n_U padded to ldb, a multiple of 64):
// block rb holds, for k = 0 .. n_Omega - 1, the 64 entries B_i[64 rb + l][k]
// contiguously, so lane l of a wavefront owns output row 64 rb + l, every load
// of a wavefront is 1 KiB (FP64) of consecutive entries, and one wavefront
// streams one contiguous n_Omega x 64 region.  The gathered X chunk sits in LDS
// and is read as a broadcast.  No atomics: results are bitwise reproducible.
#include "ctx.hpp"

namespace th {

template <typename TB, typename T, int NR>
__global__ __launch_bounds__(256) void k_dd_apply(const Sub *__restrict__ subs,
                                                  const cx<TB> *__restrict__ B,
                                                  const cx<T> *__restrict__ r,
                                                  cx<T> *__restrict__ Y, int P, int n1, long long nf,
                                                  long long yrows, int nrhs) {
  constexpr int KC = 1024 / NR;
  __shared__ cx<T> Xs[KC * NR];
  const Sub s = subs[blockIdx.y];
  const int jb = blockIdx.x * 256;
  if (jb >= s.ldb) return;  // uniform over the block
  const int j = jb + threadIdx.x;
  const bool live = j < s.ldb;  // uniform per wavefront (ldb is a multiple of 64)
  const cx<TB> *Bi = B + s.boff;
  for (int r0 = 0; r0 < nrhs; r0 += NR) {
    cx<T> acc[NR];
#pragma unroll
    for (int q = 0; q < NR; ++q) acc[q] = {0, 0};
    for (int k0 = 0; k0 < s.nOm; k0 += KC) {
      const int kc = min(KC, s.nOm - k0);
      __syncthreads();
      for (int t = threadIdx.x; t < kc * NR; t += 256) {
        const int kk = t / NR, q = t - kk * NR;
        const int k = k0 + kk;
        const long long g = om_node(s, k, P, n1);
        Xs[t] = (r0 + q < nrhs) ? r[(long long)(r0 + q) * nf + g] : cx<T>{0, 0};
      }
      __syncthreads();
      if (live) {
        const cx<TB> *bp = Bi + ((long long)(j / 64) * s.nOm + k0) * 64 + (j % 64);
#pragma unroll 16
        for (int kk = 0; kk < kc; ++kk) {
          const cx<T> b = ccast<T>(ld_stream(bp + (long long)kk * 64));
#pragma unroll
          for (int q = 0; q < NR; ++q) cmac(acc[q], b, Xs[kk * NR + q]);
        }
      }
    }
    if (j < s.nU) {
#pragma unroll
      for (int q = 0; q < NR; ++q)
        if (r0 + q < nrhs) Y[(long long)(r0 + q) * yrows + s.yoff + j] = acc[q];
    }
  }
}

// v_j (assign) or u_j += sum over the closed U^(i) containing node j of (Y_i)_j,
// subdomains in ascending order.
template <typename T>
__global__ __launch_bounds__(256) void k_dd_accumulate(const Sub *__restrict__ subs,
                                                       const int *__restrict__ nblk,
                                                       const cx<T> *__restrict__ Y,
                                                       cx<T> *__restrict__ u, int M, int P, int n1,
                                                       long long nf, long long yrows, int assign) {
  const long long rhs = blockIdx.y;
  Y += rhs * yrows;
  u += rhs * nf;
  for (long long g = blockIdx.x * (long long)blockDim.x + threadIdx.x; g < nf;
       g += (long long)gridDim.x * blockDim.x) {
    const int ix = (int)(g % n1);
    const long long t = g / n1;
    const int iy = (int)(t % n1), iz = (int)(t / n1);  // iz = 0 in 2-D
    const int bx0 = nblk[2 * ix], nbx = nblk[2 * ix + 1];
    const int by0 = nblk[2 * iy], nby = nblk[2 * iy + 1];
    const int bz0 = nblk[2 * iz], nbz = nblk[2 * iz + 1];
    cx<T> acc = {0, 0};
    for (int bz = bz0; bz < bz0 + nbz; ++bz)
      for (int by = by0; by < by0 + nby; ++by)
        for (int bx = bx0; bx < bx0 + nbx; ++bx) {
          const Sub &s = subs[(bz * M + by) * M + bx];
          const int lx = ix - s.u0x * P, ly = iy - s.u0y * P, lz = iz - s.u0z * P;
          acc = acc + Y[s.yoff + ((long long)lz * s.nuy + ly) * s.nux + lx];
        }
    u[g] = assign ? acc : u[g] + acc;
  }
}

template <typename TB, typename T>
static int dd_apply_t(const th_ctx *c, const void *r, void *y, int nrhs, hipStream_t s) {
  dim3 grid(c->max_rowblocks, (unsigned)c->subs.size());
  const Sub *ds = c->d_subs;
  const cx<TB> *B = (const cx<TB> *)c->d_B;
  if (nrhs >= 4) {
    hipLaunchKernelGGL((k_dd_apply<TB, T, 4>), grid, dim3(256), 0, s, ds, B, (const cx<T> *)r,
                       (cx<T> *)y, c->P, c->n1, c->nf, c->y_rows, nrhs);
  } else if (nrhs == 2) {
    hipLaunchKernelGGL((k_dd_apply<TB, T, 2>), grid, dim3(256), 0, s, ds, B, (const cx<T> *)r,
                       (cx<T> *)y, c->P, c->n1, c->nf, c->y_rows, nrhs);
  } else if (nrhs == 3) {
    hipLaunchKernelGGL((k_dd_apply<TB, T, 3>), grid, dim3(256), 0, s, ds, B, (const cx<T> *)r,
                       (cx<T> *)y, c->P, c->n1, c->nf, c->y_rows, nrhs);
  } else {
    hipLaunchKernelGGL((k_dd_apply<TB, T, 1>), grid, dim3(256), 0, s, ds, B, (const cx<T> *)r,
                       (cx<T> *)y, c->P, c->n1, c->nf, c->y_rows, nrhs);
  }
  TH_HIP_CHECK_RET(hipGetLastError());
  return 0;
}

int launch_dd_apply(const th_ctx *c, const void *r, void *y, int nrhs, bool f32, hipStream_t s) {
  switch (c->desc.gemm) {
    case TH_GEMM_BF16:
      return launch_dd_mfma(c, r, y, nrhs, f32, c->mfma_cfg, c->mfma_grid, s);
    case TH_GEMM_F64:
      return f32 ? dd_apply_t<double, float>(c, r, y, nrhs, s)
                 : dd_apply_t<double, double>(c, r, y, nrhs, s);
    case TH_GEMM_F32:
      return f32 ? dd_apply_t<float, float>(c, r, y, nrhs, s)
                 : dd_apply_t<float, double>(c, r, y, nrhs, s);
    default:
      break;
  }
  set_error("subdomain operator storage not supported by this apply path");
  return TH_EUNSUPPORTED;
}

int launch_dd_accumulate(const th_ctx *c, const void *y, void *u, int nrhs, bool f32, bool assign,
                         hipStream_t s) {
  int blocks = (int)std::min<long long>(ceil_div_ll(c->nf, 256), 65535);
  if (f32)
    hipLaunchKernelGGL((k_dd_accumulate<float>), dim3(blocks, nrhs), dim3(256), 0, s, c->d_subs,
                       c->d_nblk, (const cx<float> *)y, (cx<float> *)u, c->M, c->P, c->n1, c->nf,
                       c->y_rows, assign ? 1 : 0);
  else
    hipLaunchKernelGGL((k_dd_accumulate<double>), dim3(blocks, nrhs), dim3(256), 0, s, c->d_subs,
                       c->d_nblk, (const cx<double> *)y, (cx<double> *)u, c->M, c->P, c->n1,
                       c->nf, c->y_rows, assign ? 1 : 0);
  TH_HIP_CHECK_RET(hipGetLastError());
  return 0;
}

}  // namespace th
