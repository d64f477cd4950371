// Setup of the smoother's subdomain operators on the device (FP64).
//
// For every subdomain (Sec. 4.1): assemble the dense Galerkin matrix
// A_s^(i) of a(u, v; Omega^(i), Gamma) with the shifted coefficient
// k^2 (1 + i alpha_s) + i eps and the absorbing term -i k on the sides of
// Omega^(i) that are internal or inherit an absorbing boundary; invert it by
// blocked Gauss-Jordan elimination; store B_i = diag(1/L_j) R_{U_i} A^{-1} in
// blocks of 64 rows (the apply kernel's streaming order) in the working
// precision.
//
// Gauss-Jordan runs without pivoting.  A_s^(i) = H - i S with S = alpha_s k^2 M
// + k M_Gamma (plus eps M) symmetric positive definite, so i A_s^(i) has a
// positive definite Hermitian part; that property passes to every leading
// block and every Schur complement, so all pivots are nonzero.  The blocked
// in-place sweep over 64-wide block columns k is
//   P = A_kk^{-1};  A_kj <- P A_kj (j != k);  A_ij <- A_ij - A_ik A_kj;
//   A_ik <- -A_ik P (i != k);  A_kk <- P,
// and after the last block A holds A^{-1}.  Matrices are padded with an
// identity block to a multiple of 64, which leaves the inverse unchanged on
// the leading block.
//
// Guards (every batched inversion): a pivot that is zero or not finite, or
// smaller than kPivotRel times the largest entry of its 64 x 64 diagonal block
// at the time it is eliminated, sets a flag; and every inverse is checked on
// one vector: b = A x is formed before the elimination for a fixed probe x of
// unit-modulus entries, and max_i |(A^{-1} b)_i - x_i| after it must stay
// below kCheckTol.  Either failure makes the setup return TH_ENUMERIC.
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "ctx.hpp"

namespace th {

constexpr int GJ_BS = kGJBlock;  // block width of the elimination (64)
constexpr int GJ_T = 64;         // tile edge of the update kernel
constexpr int GJ_KH = 32;        // k-slice of the update staged in LDS at a time
constexpr int GJ_PT = 32;        // tile width of the panel kernels
constexpr double kPivotRel = 1e-12;  // smallest accepted |pivot| / largest |entry| of its block
constexpr double kCheckTol = 1e-6;   // largest accepted error of the one-vector inverse check

// ---------------------------------------------------------------------------
// Gauss-Jordan kernels.  Matrix b of the batch starts at A + b * stride and is
// row-major with leading dimension ld; n is a multiple of GJ_BS.  A rank-64
// update per block column reads and writes the trailing matrix once per 64
// columns of elimination.

__global__ __launch_bounds__(256) void k_gj_diag(c64 *A, int ld, long long stride, int kb,
                                                 c64 *pbuf, int *flag) {
  __shared__ c64 a[GJ_BS][GJ_BS + 1];
  __shared__ double red[256];
  c64 *Ab = A + blockIdx.x * stride + (long long)kb * GJ_BS * ld + kb * GJ_BS;
  double mx = 0.0;
  for (int t = threadIdx.x; t < GJ_BS * GJ_BS; t += blockDim.x) {
    int i = t / GJ_BS, j = t % GJ_BS;
    const c64 v = Ab[(long long)i * ld + j];
    a[i][j] = v;
    mx = fmax(mx, v.re * v.re + v.im * v.im);
  }
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  const double small2 = kPivotRel * kPivotRel * red[0];  // squared threshold
  for (int kk = 0; kk < GJ_BS; ++kk) {
    const c64 d = a[kk][kk];
    const double den = d.re * d.re + d.im * d.im;
    if (!(den > 0.0) || !isfinite(den)) {
      if (threadIdx.x == 0) flag[0] |= 1;
    } else if (den < small2) {
      if (threadIdx.x == 0) flag[0] |= 2;
    }
    const c64 piv = {d.re / den, -d.im / den};
    __syncthreads();
    // scale pivot row
    for (int j = threadIdx.x; j < GJ_BS; j += blockDim.x)
      if (j != kk) a[kk][j] = piv * a[kk][j];
    __syncthreads();
    // eliminate other rows (pivot column still holds the old values)
    for (int t = threadIdx.x; t < GJ_BS * GJ_BS; t += blockDim.x) {
      int i = t / GJ_BS, j = t % GJ_BS;
      if (i != kk && j != kk) a[i][j] = a[i][j] - a[i][kk] * a[kk][j];
    }
    __syncthreads();
    for (int i = threadIdx.x; i < GJ_BS; i += blockDim.x)
      if (i != kk) a[i][kk] = cx<double>{0, 0} - a[i][kk] * piv;
    if (threadIdx.x == 0) a[kk][kk] = piv;
    __syncthreads();
  }
  c64 *pb = pbuf + (long long)blockIdx.x * GJ_BS * GJ_BS;
  for (int t = threadIdx.x; t < GJ_BS * GJ_BS; t += blockDim.x) {
    int i = t / GJ_BS, j = t % GJ_BS;
    Ab[(long long)i * ld + j] = a[i][j];
    pb[t] = a[i][j];
  }
}

// Probe vector of the inverse check: unit-modulus entries with no structure
// that a subdomain or coarse block could share.
__device__ inline c64 gj_probe(int j) {
  double sn, cs;
  sincos(0.7548776662466927 * (double)j + 0.25 * (double)(j % 7), &sn, &cs);
  return c64{cs, sn};
}

// b = A x (before the elimination; before == 1) or the check of A^{-1} b
// against x (after it; A then holds the inverse): one wavefront per row,
// lanes over the columns, fixed-order reductions.  Grid (ceil(n / 4), batch).
__global__ __launch_bounds__(256) void k_gj_probe(const c64 *A, int ld, long long stride, int n,
                                                  c64 *chk, int before,
                                                  unsigned long long *errbits) {
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= n) return;  // wavefront-uniform
  const c64 *Ar = A + blockIdx.y * stride + (long long)row * ld;
  c64 *cb = chk + (long long)blockIdx.y * n;
  c64 acc = {0, 0};
  for (int j = lane; j < n; j += 64) cmac(acc, Ar[j], before ? gj_probe(j) : cb[j]);
  for (int o = 32; o > 0; o >>= 1) {
    acc.re += __shfl_xor(acc.re, o);
    acc.im += __shfl_xor(acc.im, o);
  }
  if (lane != 0) return;
  if (before) {
    cb[row] = acc;
    return;
  }
  const c64 x = gj_probe(row);
  const double dr = acc.re - x.re, di = acc.im - x.im;
  const double e = sqrt(dr * dr + di * di);
  // non-negative doubles order like their bit patterns; NaN sorts above them
  atomicMax(errbits, (unsigned long long)__double_as_longlong(isnan(e) ? __longlong_as_double(0x7ff8000000000000LL) : e));
}

size_t gj_ws_bytes(int batch, int n) {
  return 256 + (size_t)batch * GJ_BS * GJ_BS * sizeof(c64) + (size_t)batch * n * sizeof(c64);
}

int gj_ws_reset(c64 *ws, hipStream_t s) {
  TH_HIP_CHECK_RET(hipMemsetAsync(ws, 0, 16, s));
  return 0;
}

int gj_ws_status(const c64 *ws, hipStream_t s, const char *what) {
  unsigned long long h[2] = {0, 0};
  TH_HIP_CHECK_RET(hipMemcpyAsync(h, ws, 16, hipMemcpyDeviceToHost, s));
  TH_HIP_CHECK_RET(hipStreamSynchronize(s));
  const int flag = (int)(h[0] & 0xffffffffu);
  double err;
  std::memcpy(&err, &h[1], sizeof(err));
  char msg[256];
  if (flag & 1) {
    std::snprintf(msg, sizeof msg, "zero or non-finite pivot in %s", what);
  } else if (flag & 2) {
    std::snprintf(msg, sizeof msg, "pivot below %.0e of its block's largest entry in %s", kPivotRel,
                  what);
  } else if (!(err <= kCheckTol)) {
    std::snprintf(msg, sizeof msg, "inverse check failed in %s: |A^-1 (A x) - x| = %.3e > %.0e",
                  what, err, kCheckTol);
  } else {
    return 0;
  }
  set_error(msg);
  return TH_ENUMERIC;
}

// A_kj <- P A_kj for the GJ_PT-column tile blockIdx.x (columns of block k skipped)
__global__ __launch_bounds__(256) void k_gj_rowpanel(c64 *A, int ld, long long stride, int n, int kb,
                                                     const c64 *pbuf) {
  __shared__ c64 Ps[GJ_BS][GJ_BS + 1];
  __shared__ c64 Ts[GJ_BS][GJ_PT + 1];
  const int j0 = blockIdx.x * GJ_PT;
  if (j0 / GJ_BS == kb) return;  // the whole tile lies in block column k (uniform)
  c64 *Ab = A + blockIdx.y * stride + (long long)kb * GJ_BS * ld;
  const c64 *pb = pbuf + (long long)blockIdx.y * GJ_BS * GJ_BS;
  for (int t = threadIdx.x; t < GJ_BS * GJ_BS; t += blockDim.x) Ps[t / GJ_BS][t % GJ_BS] = pb[t];
  for (int t = threadIdx.x; t < GJ_BS * GJ_PT; t += blockDim.x) {
    int i = t / GJ_PT, j = t % GJ_PT;
    Ts[i][j] = (j0 + j < n) ? Ab[(long long)i * ld + j0 + j] : c64{0, 0};
  }
  __syncthreads();
  for (int t = threadIdx.x; t < GJ_BS * GJ_PT; t += blockDim.x) {
    int i = t / GJ_PT, j = t % GJ_PT;
    int col = j0 + j;
    if (col >= n) continue;
    c64 acc = {0, 0};
#pragma unroll 8
    for (int q = 0; q < GJ_BS; ++q) cmac(acc, Ps[i][q], Ts[q][j]);
    Ab[(long long)i * ld + col] = acc;
  }
}

// A_ik <- -A_ik P for the GJ_PT-row tile blockIdx.x (rows of block k skipped)
__global__ __launch_bounds__(256) void k_gj_colpanel(c64 *A, int ld, long long stride, int n, int kb,
                                                     const c64 *pbuf) {
  __shared__ c64 Ps[GJ_BS][GJ_BS + 1];
  __shared__ c64 Ts[GJ_PT][GJ_BS + 1];
  const int i0 = blockIdx.x * GJ_PT;
  if (i0 / GJ_BS == kb) return;  // uniform
  c64 *Ab = A + blockIdx.y * stride + kb * GJ_BS;
  const c64 *pb = pbuf + (long long)blockIdx.y * GJ_BS * GJ_BS;
  for (int t = threadIdx.x; t < GJ_BS * GJ_BS; t += blockDim.x) Ps[t / GJ_BS][t % GJ_BS] = pb[t];
  for (int t = threadIdx.x; t < GJ_PT * GJ_BS; t += blockDim.x) {
    int i = t / GJ_BS, j = t % GJ_BS;
    Ts[i][j] = (i0 + i < n) ? Ab[(long long)(i0 + i) * ld + j] : c64{0, 0};
  }
  __syncthreads();
  for (int t = threadIdx.x; t < GJ_PT * GJ_BS; t += blockDim.x) {
    int i = t / GJ_BS, j = t % GJ_BS;
    int row = i0 + i;
    if (row >= n) continue;
    c64 acc = {0, 0};
#pragma unroll 8
    for (int q = 0; q < GJ_BS; ++q) cmac(acc, Ts[i][q], Ps[q][j]);
    Ab[(long long)row * ld + j] = c64{-acc.re, -acc.im};
  }
}

// A_ij <- A_ij - A_ik A_kj on the 64x64 tile (blockIdx.x, blockIdx.y), entries
// in block row k or block column k left untouched; the 64-wide k range is
// staged through LDS in two slices.
__global__ __launch_bounds__(256) void k_gj_update(c64 *A, int ld, long long stride, int n, int kb) {
  __shared__ c64 As[GJ_T][GJ_KH + 1];
  __shared__ c64 Bs[GJ_KH][GJ_T + 1];
  const int j0 = blockIdx.x * GJ_T, i0 = blockIdx.y * GJ_T;
  // tiles wholly inside block row or block column k have nothing to update (uniform)
  if (i0 / GJ_BS == kb || j0 / GJ_BS == kb) return;
  c64 *Ab = A + blockIdx.z * stride;
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  c64 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = {0, 0};
  for (int h = 0; h < GJ_BS / GJ_KH; ++h) {
    const int k0 = kb * GJ_BS + h * GJ_KH;
    if (h) __syncthreads();
    for (int t = threadIdx.x; t < GJ_T * GJ_KH; t += blockDim.x) {
      int i = t / GJ_KH, q = t % GJ_KH;
      As[i][q] = (i0 + i < n) ? Ab[(long long)(i0 + i) * ld + k0 + q] : c64{0, 0};
    }
    for (int t = threadIdx.x; t < GJ_KH * GJ_T; t += blockDim.x) {
      int q = t / GJ_T, j = t % GJ_T;
      Bs[q][j] = (j0 + j < n) ? Ab[(long long)(k0 + q) * ld + j0 + j] : c64{0, 0};
    }
    __syncthreads();
#pragma unroll 4
    for (int q = 0; q < GJ_KH; ++q) {
      c64 av[4], bv[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) av[a] = As[ty + 16 * a][q];
#pragma unroll
      for (int b = 0; b < 4; ++b) bv[b] = Bs[q][tx + 16 * b];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) cmac(acc[a][b], av[a], bv[b]);
    }
  }
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int row = i0 + ty + 16 * a;
    if (row >= n) continue;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int col = j0 + tx + 16 * b;
      if (col >= n) continue;
      c64 *p = Ab + (long long)row * ld + col;
      *p = *p - acc[a][b];
    }
  }
}

int gj_invert_batched(c64 *A, int n, int ld, long long stride, int batch, hipStream_t s,
                      c64 *ws) {
  // ws: gj_ws_bytes(batch, >= n) bytes, status words cleared by gj_ws_reset
  if (n % GJ_BS) {
    set_error("gauss-jordan size must be a multiple of the block width");
    return TH_EINVAL;
  }
  int *flag = (int *)ws;
  unsigned long long *errbits = (unsigned long long *)((char *)ws + 8);
  c64 *pbuf = (c64 *)((char *)ws + 256);
  c64 *chk = pbuf + (long long)batch * GJ_BS * GJ_BS;
  const int nbk = n / GJ_BS;
  const int nt = ceil_div(n, GJ_T), np = ceil_div(n, GJ_PT);
  const dim3 gprobe(ceil_div(n, 4), batch);
  hipLaunchKernelGGL(k_gj_probe, gprobe, dim3(256), 0, s, (const c64 *)A, ld, stride, n, chk, 1,
                     errbits);
  for (int kb = 0; kb < nbk; ++kb) {
    hipLaunchKernelGGL(k_gj_diag, dim3(batch), dim3(256), 0, s, A, ld, stride, kb, pbuf, flag);
    hipLaunchKernelGGL(k_gj_rowpanel, dim3(np, batch), dim3(256), 0, s, A, ld, stride, n, kb,
                       (const c64 *)pbuf);
    hipLaunchKernelGGL(k_gj_update, dim3(nt, nt, batch), dim3(256), 0, s, A, ld, stride, n, kb);
    hipLaunchKernelGGL(k_gj_colpanel, dim3(np, batch), dim3(256), 0, s, A, ld, stride, n, kb,
                       (const c64 *)pbuf);
    TH_HIP_CHECK_RET(hipGetLastError());
  }
  hipLaunchKernelGGL(k_gj_probe, gprobe, dim3(256), 0, s, (const c64 *)A, ld, stride, n, chk, 0,
                     errbits);
  TH_HIP_CHECK_RET(hipGetLastError());
  return 0;
}

// ---------------------------------------------------------------------------
// Dense subdomain assembly: one thread per row (local Omega node); every
// thread writes only its own row, summing its cells in a fixed order.  Nodes
// on a Dirichlet side of the domain get a unit row and column (the buffer is
// zero on entry).

template <int P>
__global__ __launch_bounds__(256) void k_assemble_sub(const Sub *__restrict__ subs, int s0,
                                                      c64 *A, int ld, long long stride,
                                                      const c64 *__restrict__ kaps,
                                                      const double *__restrict__ kr, Ref1D ref,
                                                      double h, int N) {
  constexpr int NP = P + 1;
  const Sub s = subs[s0 + blockIdx.y];
  c64 *Ab = A + blockIdx.y * stride;
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= ld) return;
  c64 *row = Ab + (long long)a * ld;
  if (a >= s.nOm) {
    row[a] = c64{1.0, 0.0};
    return;
  }
  const int ncx = s.o1x - s.o0x, ncy = s.o1y - s.o0y;
  const int ax = a % s.nox, ay = a / s.nox;
  if (on_dir(s.dir, 0, ax, ncx * P) || on_dir(s.dir, 1, ay, ncy * P)) {
    row[a] = c64{1.0, 0.0};
    return;
  }
  const int chx = min(ax / P, ncx - 1), chy = min(ay / P, ncy - 1);
  const int nxc = (ax % P == 0 && ax > 0 && ax < ncx * P) ? 2 : 1;
  const int nyc = (ay % P == 0 && ay > 0 && ay < ncy * P) ? 2 : 1;
  const double h2 = h * h;
  for (int qy = nyc - 1; qy >= 0; --qy) {
    const int lcy = chy - qy, ly = ay - lcy * P;
    for (int qx = nxc - 1; qx >= 0; --qx) {
      const int lcx = chx - qx, lx = ax - lcx * P;
      const long long gc = (long long)(s.o0y + lcy) * N + (s.o0x + lcx);
      const c64 kap = kaps[gc];
      const double kk = kr[gc];
      const bool rxl = (s.robin & 1) && lcx == 0 && lx == 0;
      const bool rxh = (s.robin & 2) && lcx == ncx - 1 && lx == P;
      const bool ryl = (s.robin & 4) && lcy == 0 && ly == 0;
      const bool ryh = (s.robin & 8) && lcy == ncy - 1 && ly == P;
      for (int by = 0; by < NP; ++by) {
        const double Ky = ref.K[ly * NP + by], My = ref.M[ly * NP + by];
        if (on_dir(s.dir, 1, lcy * P + by, ncy * P)) continue;
        for (int bx = 0; bx < NP; ++bx) {
          if (on_dir(s.dir, 0, lcx * P + bx, ncx * P)) continue;
          const double Kx = ref.K[lx * NP + bx], Mx = ref.M[lx * NP + bx];
          const double mm = h2 * My * Mx;
          c64 v = {Ky * Mx + My * Kx - kap.re * mm, -kap.im * mm};
          if ((rxl && bx == 0) || (rxh && bx == P)) v.im -= kk * h * My;
          if ((ryl && by == 0) || (ryh && by == P)) v.im -= kk * h * Mx;
          const int col = (lcy * P + by) * s.nox + lcx * P + bx;
          row[col] = row[col] + v;
        }
      }
    }
  }
}

// 3-D: per cell h (Kz My Mx + Mz Ky Mx + Mz My Kx) - kappa h^3 Mz My Mx, and
// -i k h^2 (M (x) M over the face) on faces of Omega carrying the absorbing term.
template <int P>
__global__ __launch_bounds__(256) void k_assemble_sub3(const Sub *__restrict__ subs, int s0,
                                                       c64 *A, int ld, long long stride,
                                                       const c64 *__restrict__ kaps,
                                                       const double *__restrict__ kr, Ref1D ref,
                                                       double h, int N) {
  constexpr int NP = P + 1;
  const Sub s = subs[s0 + blockIdx.y];
  c64 *Ab = A + blockIdx.y * stride;
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= ld) return;
  c64 *row = Ab + (long long)a * ld;
  if (a >= s.nOm) {
    row[a] = c64{1.0, 0.0};
    return;
  }
  const int nc[3] = {s.o1x - s.o0x, s.o1y - s.o0y, s.o1z - s.o0z};
  const int al[3] = {a % s.nox, (a / s.nox) % s.noy, a / (s.nox * s.noy)};
  if (on_dir(s.dir, 0, al[0], nc[0] * P) || on_dir(s.dir, 1, al[1], nc[1] * P) ||
      on_dir(s.dir, 2, al[2], nc[2] * P)) {
    row[a] = c64{1.0, 0.0};
    return;
  }
  int ch[3], nq[3];
  for (int d = 0; d < 3; ++d) {
    ch[d] = min(al[d] / P, nc[d] - 1);
    nq[d] = (al[d] % P == 0 && al[d] > 0 && al[d] < nc[d] * P) ? 2 : 1;
  }
  const double h2 = h * h, h3 = h2 * h;
  for (int qz = nq[2] - 1; qz >= 0; --qz) {
    const int lcz = ch[2] - qz, lz = al[2] - lcz * P;
    for (int qy = nq[1] - 1; qy >= 0; --qy) {
      const int lcy = ch[1] - qy, ly = al[1] - lcy * P;
      for (int qx = nq[0] - 1; qx >= 0; --qx) {
        const int lcx = ch[0] - qx, lx = al[0] - lcx * P;
        const long long gc = ((long long)(s.o0z + lcz) * N + (s.o0y + lcy)) * N + (s.o0x + lcx);
        const c64 kap = kaps[gc];
        const double kk = kr[gc];
        const bool rxl = (s.robin & 1) && lcx == 0 && lx == 0;
        const bool rxh = (s.robin & 2) && lcx == nc[0] - 1 && lx == P;
        const bool ryl = (s.robin & 4) && lcy == 0 && ly == 0;
        const bool ryh = (s.robin & 8) && lcy == nc[1] - 1 && ly == P;
        const bool rzl = (s.robin & 16) && lcz == 0 && lz == 0;
        const bool rzh = (s.robin & 32) && lcz == nc[2] - 1 && lz == P;
        for (int bz = 0; bz < NP; ++bz) {
          const double Kz = ref.K[lz * NP + bz], Mz = ref.M[lz * NP + bz];
          if (on_dir(s.dir, 2, lcz * P + bz, nc[2] * P)) continue;
          for (int by = 0; by < NP; ++by) {
            const double Ky = ref.K[ly * NP + by], My = ref.M[ly * NP + by];
            if (on_dir(s.dir, 1, lcy * P + by, nc[1] * P)) continue;
            for (int bx = 0; bx < NP; ++bx) {
              if (on_dir(s.dir, 0, lcx * P + bx, nc[0] * P)) continue;
              const double Kx = ref.K[lx * NP + bx], Mx = ref.M[lx * NP + bx];
              const double mmm = h3 * Mz * My * Mx;
              c64 v = {h * (Kz * My * Mx + Mz * Ky * Mx + Mz * My * Kx) - kap.re * mmm,
                       -kap.im * mmm};
              if ((rxl && bx == 0) || (rxh && bx == P)) v.im -= kk * h2 * Mz * My;
              if ((ryl && by == 0) || (ryh && by == P)) v.im -= kk * h2 * Mz * Mx;
              if ((rzl && bz == 0) || (rzh && bz == P)) v.im -= kk * h2 * My * Mx;
              const int col = ((lcz * P + bz) * s.noy + lcy * P + by) * s.nox + lcx * P + bx;
              row[col] = row[col] + v;
            }
          }
        }
      }
    }
  }
}

// B_i[j][k] = (A^{-1})[u_j][k] / L_{u_j} in the storage precision, in blocks of
// 64 rows: entry (j, k) at ((j / 64) n_Omega + k) 64 + j % 64.
template <typename TB>
__global__ __launch_bounds__(256) void k_extract_b(const Sub *__restrict__ subs, int s0,
                                                   const c64 *__restrict__ A, int ld,
                                                   long long stride, const int *__restrict__ nblk,
                                                   cx<TB> *__restrict__ B, int P) {
  const Sub s = subs[s0 + blockIdx.z];
  const c64 *Ab = A + blockIdx.z * stride;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= s.nU) return;
  int gn[3], uj;
  u_node(s, j, P, gn, uj);
  const double invL =
      1.0 / (double)(nblk[2 * gn[0] + 1] * nblk[2 * gn[1] + 1] * nblk[2 * gn[2] + 1]);
  const c64 *arow = Ab + (long long)uj * ld;
  for (int k = blockIdx.y; k < s.nOm; k += gridDim.y) {
    const c64 v = arow[k];
    B[s.boff + ((long long)(j / 64) * s.nOm + k) * 64 + (j % 64)] =
        cx<TB>{(TB)(v.re * invL), (TB)(v.im * invL)};
  }
}

// Symmetric-tile layout (see the apply kernel): workgroup = one tile of one
// subdomain; entries (l, c) row-major.  Upper tile (a, b): rows 64 a + l and
// columns 64 b + c of the U x U block of A^{-1}; ring tile (a, e): rows
// 64 a + l of U, ring columns 64 e + c.  No weights (applied after the sum).
template <typename TB>
__global__ __launch_bounds__(256) void k_extract_sym(const Sub *__restrict__ subs, int s0,
                                                     const c64 *__restrict__ A, int ld,
                                                     long long stride,
                                                     const int *__restrict__ eidx,
                                                     cx<TB> *__restrict__ B, int P) {
  constexpr int ST = kSymTile;
  const Sub s = subs[s0 + blockIdx.y];
  const c64 *Ab = A + blockIdx.y * stride;
  const int nrb = s.nrb, neb = s.neb;
  const int nS = nrb * (nrb + 1) / 2, nE = s.nOm - s.nU;
  const int t = blockIdx.x;
  if (t >= nS + nrb * neb) return;  // uniform
  int a, b = -1, e = -1;
  if (t < nS) {
    a = 0;
    while (a + 1 < nrb && sym_tile(a + 1, a + 1, nrb) <= t) ++a;
    b = a + (t - sym_tile(a, a, nrb));
  } else {
    a = (t - nS) / neb;
    e = (t - nS) - a * neb;
  }
  cx<TB> *tile = B + s.boff + (long long)t * (ST * ST);
  for (int q = threadIdx.x; q < ST * ST; q += blockDim.x) {
    const int l = q / ST, cc = q % ST;
    const int i = a * ST + l;
    c64 v = {0, 0};
    if (i < s.nU) {
      int g[3], ui;
      u_node(s, i, P, g, ui);
      int col = -1;
      if (b >= 0) {
        const int j = b * ST + cc;
        if (j < s.nU) u_node(s, j, P, g, col);
      } else {
        const int k = e * ST + cc;
        if (k < nE) col = eidx[s.eoff + k];
      }
      if (col >= 0) v = Ab[(long long)ui * ld + col];
    }
    tile[q] = cx<TB>{(TB)v.re, (TB)v.im};
  }
}

int setup_subdomain_operators(th_ctx *c) {
  hipStream_t s = c->stream;
  const int nsub = (int)c->subs.size();
  const int npad = ceil_div(c->max_nom, GJ_BS) * GJ_BS;
  const long long mat = (long long)npad * npad;
  // slab layout: three slab work matrices and the Schur product per subdomain
  const bool slab = c->layout == 3;
  int max_lsz = 0;
  for (const Sub &sb : c->subs) max_lsz = std::max(max_lsz, sb.lsz);
  const int ldw = slab ? ceil_div(c->max_slab_rows, GJ_BS) * GJ_BS : 0;
  const long long per_sub = mat + (slab ? 3LL * ldw * ldw + (long long)ldw * max_lsz : 0);
  // batch: bounded by ~8 GiB of work space and by free memory
  size_t free_b = 0, total_b = 0;
  TH_HIP_CHECK_RET(hipMemGetInfo(&free_b, &total_b));
  long long budget = std::min<long long>(8LL << 30, (long long)(free_b / 3));
  int batch = (int)std::max<long long>(1, std::min<long long>(nsub, budget / (per_sub * 16)));
  c64 *work = nullptr, *pws = nullptr;
  if (hipMalloc(&work, (size_t)batch * per_sub * sizeof(c64)) != hipSuccess) {
    set_error("cannot allocate the subdomain work space");
    return TH_ENOMEM;
  }
  c64 *const W[3] = {work + (long long)batch * mat, work + (long long)batch * (mat + ldw * ldw),
                     work + (long long)batch * (mat + 2LL * ldw * ldw)};
  c64 *T1 = work + (long long)batch * (mat + 3LL * ldw * ldw);
  if (hipMalloc(&pws, gj_ws_bytes(batch, npad)) != hipSuccess) {
    (void)hipFree(work);
    set_error("cannot allocate the pivot work space");
    return TH_ENOMEM;
  }
  int rc = gj_ws_reset(pws, s);
  // optional progress lines on stderr for long setups (environment TH_PROGRESS
  // set): the stream is synchronised after a batch at most every 10 s
  const bool progress = std::getenv("TH_PROGRESS") != nullptr;
  auto t_last = std::chrono::steady_clock::now();
  const auto t_begin = t_last;
  for (int s0 = 0; s0 < nsub && rc == 0; s0 += batch) {
    if (progress && s0 > 0 &&
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t_last).count() > 10.0) {
      TH_HIP_CHECK_RET(hipStreamSynchronize(s));
      t_last = std::chrono::steady_clock::now();
      std::fprintf(stderr, "setup: %d / %d subdomain operators, %.1f s\n", s0, nsub,
                   std::chrono::duration<double>(t_last - t_begin).count());
      std::fflush(stderr);
    }
    const int nb = std::min(batch, nsub - s0);
    TH_HIP_CHECK_RET(hipMemsetAsync(work, 0, (size_t)nb * mat * sizeof(c64), s));
    dim3 ga(ceil_div(npad, 256), nb);
    if (c->dim == 3) {
      if (c->P == 2)
        hipLaunchKernelGGL((k_assemble_sub3<2>), ga, dim3(256), 0, s, c->d_subs, s0, work, npad,
                           mat, (const c64 *)c->d_kaps, (const double *)c->d_k, c->ref, c->h, c->N);
      else
        hipLaunchKernelGGL((k_assemble_sub3<4>), ga, dim3(256), 0, s, c->d_subs, s0, work, npad,
                           mat, (const c64 *)c->d_kaps, (const double *)c->d_k, c->ref, c->h, c->N);
    } else switch (c->P) {
#define TH_ASM(PP)                                                                              \
  case PP:                                                                                      \
    hipLaunchKernelGGL((k_assemble_sub<PP>), ga, dim3(256), 0, s, c->d_subs, s0, work, npad,    \
                       mat, (const c64 *)c->d_kaps, (const double *)c->d_k, c->ref, c->h, c->N); \
    break;
      TH_ASM(2) TH_ASM(4) TH_ASM(6) TH_ASM(8)
#undef TH_ASM
    }
    TH_HIP_CHECK_RET(hipGetLastError());
    if (slab) {
      rc = setup_slab_factors(c, s0, nb, work, npad, mat, W, T1, ldw, max_lsz, pws, s);
      continue;
    }
    rc = gj_invert_batched(work, npad, npad, mat, nb, s, pws);
    if (rc) break;
    dim3 ge(ceil_div(c->max_ldb, 256), 64, nb);
    int max_tiles = 0;
    for (const Sub &sb : c->subs)
      max_tiles = std::max(max_tiles, sb.nrb * (sb.nrb + 1) / 2 + sb.nrb * sb.neb);
    if (c->desc.gemm == TH_GEMM_BF16) {
      rc = launch_extract_b_mfma(c, s0, nb, work, npad, mat, s);
      if (rc) break;
    } else if (c->layout == 1 && c->desc.gemm == TH_GEMM_F32) {
      hipLaunchKernelGGL((k_extract_sym<float>), dim3(max_tiles, nb), dim3(256), 0, s, c->d_subs,
                         s0, (const c64 *)work, npad, mat, (const int *)c->d_eidx,
                         (cx<float> *)c->d_B, c->P);
    } else if (c->layout == 1) {
      hipLaunchKernelGGL((k_extract_sym<double>), dim3(max_tiles, nb), dim3(256), 0, s, c->d_subs,
                         s0, (const c64 *)work, npad, mat, (const int *)c->d_eidx,
                         (cx<double> *)c->d_B, c->P);
    } else if (c->desc.gemm == TH_GEMM_F32)
      hipLaunchKernelGGL((k_extract_b<float>), ge, dim3(256), 0, s, c->d_subs, s0,
                         (const c64 *)work, npad, mat, c->d_nblk, (cx<float> *)c->d_B, c->P);
    else
      hipLaunchKernelGGL((k_extract_b<double>), ge, dim3(256), 0, s, c->d_subs, s0,
                         (const c64 *)work, npad, mat, c->d_nblk, (cx<double> *)c->d_B, c->P);
    TH_HIP_CHECK_RET(hipGetLastError());
  }
  if (rc == 0) rc = gj_ws_status(pws, s, slab ? "a subdomain slab factor" : "a subdomain inverse");
  (void)hipStreamSynchronize(s);
  (void)hipFree(work);
  (void)hipFree(pws);
  return rc;
}

}  // namespace th
