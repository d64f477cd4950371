// Coarse-level direct solve in FP64 (Alg. 1, "solve A_c u_c = r_c"; the paper
// uses a direct solver and notes that approximate ones may be used).
//
// The quasi-FE QSFEM matrix (Sec. 3.3) is a 9-point stencil on the coarse
// vertex grid.  Grouping K consecutive grid lines (constant y) into a
// super-block makes it block tridiagonal, and the coupling between
// super-blocks J-1 and J only links the last line of J-1 with the first line
// of J (tridiagonal in x).  Setup (once, timed separately) runs the block
// elimination in natural order
//   S_0 = T_0,   S_J = T_J - L_J S_{J-1}^{-1} U_{J-1},   G_J = S_J^{-1},
// where L_J S_{J-1}^{-1} U_{J-1} only touches the first-line block of S_J and
// only needs the last-line block of G_{J-1}.  Every S_J is inverted by the
// same Gauss-Jordan kernels as the subdomain operators (no pivoting: natural
// order elimination of these matrices is stable, checked against pivoted
// sparse LU).  The solve is
//   forward   y_J = G_J (r_J - L_J y_{J-1})
//   backward  x_J = y_J - G_J[:, last line] (U_J x_{J+1}[first line]),
// two launches per super-block, each a bandwidth-bound GEMV with one
// wavefront per output row (coalesced row reads of G_J, the right-hand side
// staged in LDS, fixed-order wavefront reductions).  K trades the bytes of G
// (proportional to K) against the number of sequential launches (~2 ny / K).
#include <algorithm>
#include <cmath>
#include <vector>

#include "ctx.hpp"

namespace th {

constexpr int CW = 8;  // wavefronts (rows) per workgroup in the sweeps

// S_J (ld x ld, identity padding) written over the G_J slot.
__global__ __launch_bounds__(256) void k_build_s(c64 *__restrict__ S, int ld, int nb, int nx,
                                                 int line0, const c64 *__restrict__ st9,
                                                 const c64 *__restrict__ Gp, int ldp, int kp) {
  const long long t = blockIdx.x * 256LL + threadIdx.x;
  if (t >= (long long)ld * ld) return;
  const int a = (int)(t / ld), b = (int)(t % ld);
  c64 v = {0, 0};
  if (a >= nb || b >= nb) {
    v = (a == b) ? c64{1.0, 0.0} : c64{0, 0};
  } else {
    const int la = a / nx, ca = a - la * nx, lb = b / nx, cb = b - lb * nx;
    const int dy = lb - la, dx = cb - ca;
    const long long ga = (long long)(line0 + la) * nx + ca;
    if (dy >= -1 && dy <= 1 && dx >= -1 && dx <= 1) v = st9[9 * ga + (dy + 1) * 3 + dx + 1];
    if (Gp && la == 0 && lb == 0) {
      // - sum_{c,d} L[ca][c] G_{J-1}[last c][last d] U[d][cb]
      const long long off = (long long)(kp - 1) * nx;
      for (int c = max(ca - 1, 0); c <= min(ca + 1, nx - 1); ++c) {
        const c64 l = st9[9 * ga + 0 * 3 + (c - ca) + 1];
        c64 s = {0, 0};
        for (int d = max(cb - 1, 0); d <= min(cb + 1, nx - 1); ++d) {
          const long long gd = (long long)(line0 - 1) * nx + d;
          const c64 u = st9[9 * gd + 2 * 3 + (cb - d) + 1];
          cmac(s, Gp[(off + c) * ldp + off + d], u);
        }
        v = v - l * s;
      }
    }
  }
  S[t] = v;
}

__device__ __forceinline__ c64 wave_sum(c64 v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    v.re += __shfl_xor(v.re, o, 64);
    v.im += __shfl_xor(v.im, o, 64);
  }
  return v;
}

// forward step of super-block J: y_J = G_J (r_J - L_J y_{J-1})
template <int RC>
__global__ __launch_bounds__(64 * CW) void k_cfwd(const c64 *__restrict__ G, int ld, int nb,
                                                  int nx, int line0, const c64 *__restrict__ st9,
                                                  const c64 *__restrict__ rc, c64 *__restrict__ uc,
                                                  int nrhs, long long ncn, int has_prev) {
  extern __shared__ c64 tsh[];  // RC x nb
  const int r0 = blockIdx.y * RC;
  for (int i = threadIdx.x; i < nb * RC; i += blockDim.x) {
    const int q = i / nb, a = i - q * nb;
    const int r = r0 + q;
    c64 v = {0, 0};
    if (r < nrhs) {
      const long long g = (long long)line0 * nx + a;
      v = rc[r * ncn + g];
      if (has_prev && a < nx) {
        const c64 *s = st9 + 9 * g;
        for (int c = max(a - 1, 0); c <= min(a + 1, nx - 1); ++c)
          v = v - s[(c - a) + 1] * uc[r * ncn + (long long)(line0 - 1) * nx + c];
      }
    }
    tsh[q * nb + a] = v;
  }
  __syncthreads();
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int a = blockIdx.x * CW + wave;
  if (a >= nb) return;
  const c64 *row = G + (long long)a * ld;
  c64 acc[RC];
#pragma unroll
  for (int q = 0; q < RC; ++q) acc[q] = {0, 0};
#pragma unroll 4
  for (int b = lane; b < nb; b += 64) {
    const c64 g = row[b];
#pragma unroll
    for (int q = 0; q < RC; ++q) cmac(acc[q], g, tsh[q * nb + b]);
  }
#pragma unroll
  for (int q = 0; q < RC; ++q) {
    const c64 s = wave_sum(acc[q]);
    if (lane == 0 && r0 + q < nrhs) uc[(r0 + q) * ncn + (long long)line0 * nx + a] = s;
  }
}

// backward step of super-block J (not the last): x_J = y_J - G_J[:, last] w,
// w = U_J x_{J+1}[first line]
template <int RC>
__global__ __launch_bounds__(64 * CW) void k_cbwd(const c64 *__restrict__ G, int ld, int nb,
                                                  int nx, int line0, int kJ,
                                                  const c64 *__restrict__ st9,
                                                  c64 *__restrict__ uc, int nrhs, long long ncn) {
  extern __shared__ c64 wsh[];  // RC x nx
  const int r0 = blockIdx.y * RC;
  const int lend = line0 + kJ;  // first line of J+1
  for (int i = threadIdx.x; i < nx * RC; i += blockDim.x) {
    const int q = i / nx, c = i - q * nx;
    const int r = r0 + q;
    c64 v = {0, 0};
    if (r < nrhs) {
      const long long gc = (long long)(lend - 1) * nx + c;
      const c64 *s = st9 + 9 * gc + 6;
      for (int d = max(c - 1, 0); d <= min(c + 1, nx - 1); ++d)
        cmac(v, s[(d - c) + 1], uc[r * ncn + (long long)lend * nx + d]);
    }
    wsh[q * nx + c] = v;
  }
  __syncthreads();
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int a = blockIdx.x * CW + wave;
  if (a >= nb) return;
  const c64 *row = G + (long long)a * ld + (long long)(kJ - 1) * nx;
  c64 acc[RC];
#pragma unroll
  for (int q = 0; q < RC; ++q) acc[q] = {0, 0};
  for (int c = lane; c < nx; c += 64) {
    const c64 g = row[c];
#pragma unroll
    for (int q = 0; q < RC; ++q) cmac(acc[q], g, wsh[q * nx + c]);
  }
#pragma unroll
  for (int q = 0; q < RC; ++q) {
    const c64 s = wave_sum(acc[q]);
    if (lane == 0 && r0 + q < nrhs) {
      c64 *p = uc + (r0 + q) * ncn + (long long)line0 * nx + a;
      *p = *p - s;
    }
  }
}

// Number of lines per super-block: minimise the modelled solve time
// (K + 1) ny nx^2 16 B / BW  +  2 ceil(ny / K) launches x latency, with the
// staged right-hand side within 64 KiB of LDS and G within a memory budget.
static int choose_lines(int nx, int ny, int rc_chunk, int passes) {
  const double bw = 4.0e12, lat = 8.0e-6;
  const int nb_max = std::min(4096, 65536 / (16 * rc_chunk));
  const int kmax = std::max(1, std::min(ny, nb_max / nx));
  int best = 1;
  double best_t = 1e300;
  for (int K = 1; K <= kmax; ++K) {
    const double bytes = (double)(K + 1) * ny * nx * (double)nx * 16.0 * passes;
    if ((double)ny * K * nx * (double)nx * 16.0 > 24e9) break;
    const double t = bytes / bw + 2.0 * std::ceil((double)ny / K) * lat;
    if (t < best_t) {
      best_t = t;
      best = K;
    }
  }
  return best;
}

int setup_coarse_factors(th_ctx *c, const std::vector<c64> &st) {
  hipStream_t s = c->stream;
  CoarseData &cd = c->coarse;
  const int nx = c->nc1, ny = c->nc1;
  cd.nx = nx;
  cd.ny = ny;
  const int R = c->desc.max_rhs;
  cd.rc_chunk = (R >= 4) ? 4 : (R >= 2 ? 2 : 1);
  const int passes = (R + cd.rc_chunk - 1) / cd.rc_chunk;
  const int K = choose_lines(nx, ny, cd.rc_chunk, passes);
  // balanced super-blocks of about K lines
  const int nblk = (ny + K - 1) / K;
  cd.nblk = nblk;
  cd.line0.assign(nblk + 1, 0);
  {
    const int base = ny / nblk, rem = ny % nblk;
    for (int J = 0; J < nblk; ++J) cd.line0[J + 1] = cd.line0[J] + base + (J < rem ? 1 : 0);
  }
  cd.ld.resize(nblk);
  cd.goff.resize(nblk + 1);
  cd.goff[0] = 0;
  for (int J = 0; J < nblk; ++J) {
    const int nb = (cd.line0[J + 1] - cd.line0[J]) * nx;
    cd.ld[J] = ceil_div(nb, 32) * 32;
    cd.goff[J + 1] = cd.goff[J] + (long long)cd.ld[J] * cd.ld[J];
  }
  const size_t st_bytes = (size_t)nx * ny * 9 * sizeof(c64);
  cd.bytes = cd.goff[nblk] * (long long)sizeof(c64) + (long long)st_bytes;
  c64 *pws = nullptr;
  if (hipMalloc(&cd.G, (size_t)cd.goff[nblk] * sizeof(c64)) != hipSuccess ||
      hipMalloc(&cd.st9, st_bytes) != hipSuccess ||
      hipMalloc(&pws, 32 * 32 * sizeof(c64) + 64) != hipSuccess) {
    if (pws) (void)hipFree(pws);
    set_error("cannot allocate the coarse factors");
    return TH_ENOMEM;
  }
  TH_HIP_CHECK_RET(hipMemcpyAsync(cd.st9, st.data(), st_bytes, hipMemcpyHostToDevice, s));
  int *flag = (int *)(pws + 32 * 32);
  TH_HIP_CHECK_RET(hipMemsetAsync(flag, 0, sizeof(int), s));
  int rc = 0;
  for (int J = 0; J < nblk && rc == 0; ++J) {
    const int ld = cd.ld[J], nb = (cd.line0[J + 1] - cd.line0[J]) * nx;
    c64 *GJ = cd.G + cd.goff[J];
    const c64 *Gp = J > 0 ? cd.G + cd.goff[J - 1] : nullptr;
    const int ldp = J > 0 ? cd.ld[J - 1] : 0;
    const int kp = J > 0 ? cd.line0[J] - cd.line0[J - 1] : 0;
    const long long tot = (long long)ld * ld;
    hipLaunchKernelGGL(k_build_s, dim3((unsigned)ceil_div_ll(tot, 256)), dim3(256), 0, s, GJ, ld,
                       nb, nx, cd.line0[J], (const c64 *)cd.st9, Gp, ldp, kp);
    TH_HIP_CHECK_RET(hipGetLastError());
    rc = gj_invert_batched(GJ, ld, ld, tot, 1, s, pws);
  }
  int hflag = 0;
  TH_HIP_CHECK_RET(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, s));
  TH_HIP_CHECK_RET(hipStreamSynchronize(s));
  (void)hipFree(pws);
  if (rc) return rc;
  if (hflag) {
    set_error("zero or non-finite pivot in the coarse factorisation");
    return TH_ENUMERIC;
  }
  return 0;
}

template <int RC>
static int sweep_t(th_ctx *c, const c64 *rcv, c64 *uc, int nrhs, hipStream_t s) {
  const CoarseData &cd = c->coarse;
  const long long ncn = (long long)cd.nx * cd.ny;
  const unsigned ychunks = (unsigned)ceil_div(nrhs, RC);
  for (int J = 0; J < cd.nblk; ++J) {
    const int nb = (cd.line0[J + 1] - cd.line0[J]) * cd.nx;
    const size_t shm = (size_t)nb * RC * sizeof(c64);
    hipLaunchKernelGGL((k_cfwd<RC>), dim3(ceil_div(nb, CW), ychunks), dim3(64 * CW), shm, s,
                       (const c64 *)(cd.G + cd.goff[J]), cd.ld[J], nb, cd.nx, cd.line0[J],
                       (const c64 *)cd.st9, rcv, uc, nrhs, ncn, J > 0 ? 1 : 0);
  }
  for (int J = cd.nblk - 2; J >= 0; --J) {
    const int kJ = cd.line0[J + 1] - cd.line0[J];
    const int nb = kJ * cd.nx;
    const size_t shm = (size_t)cd.nx * RC * sizeof(c64);
    hipLaunchKernelGGL((k_cbwd<RC>), dim3(ceil_div(nb, CW), ychunks), dim3(64 * CW), shm, s,
                       (const c64 *)(cd.G + cd.goff[J]), cd.ld[J], nb, cd.nx, cd.line0[J], kJ,
                       (const c64 *)cd.st9, uc, nrhs, ncn);
  }
  TH_HIP_CHECK_RET(hipGetLastError());
  return 0;
}

int launch_coarse_solve(th_ctx *c, const c64 *rcv, c64 *uc, int nrhs, hipStream_t s) {
  switch (c->coarse.rc_chunk) {
    case 4: return sweep_t<4>(c, rcv, uc, nrhs, s);
    case 2: return sweep_t<2>(c, rcv, uc, nrhs, s);
    default: return sweep_t<1>(c, rcv, uc, nrhs, s);
  }
}

}  // namespace th
