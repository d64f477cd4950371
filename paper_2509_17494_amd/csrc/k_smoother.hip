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
#include <algorithm>
#include <type_traits>

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

// ---------------------------------------------------------------------------
// Symmetric-tile layout.  A_s^(i) is complex symmetric (a symmetric bilinear
// form, no conjugation), hence so is its inverse, and the U x U block of
// R_U (A_s^(i))^{-1} is stored once: upper 64 x 64 tiles (a, b), a <= b, then
// the 64 x 64 tiles (a, e) of the U x ring block (ring = Omega \ U, in
// Omega-local order), every tile row-major; no weights folded in.  A
// workgroup owns the row blocks w and nrb - 1 - w of one subdomain (equal
// work for all pairs) and reads each of their tiles once: a tile (a, b)
// contributes S_ab x_b to the rows of block a (accumulated in registers) and,
// for a < b, S_ab^T x_a to the rows of block b, written as a partial vector
// that k_dd_symred adds in a fixed order.  Thread (tx, ty) owns rows 4 ty + i
// and columns tx + 16 j of a tile, so a wavefront streams 16 consecutive rows
// (16 KiB, FP64) of every tile.  The patch X_i is gathered once per launch into a
// contiguous buffer (U nodes, then ring nodes) by k_dd_gather.
template <typename T>
__global__ __launch_bounds__(256) void k_dd_gather(const Sub *__restrict__ subs,
                                                   const int *__restrict__ eidx,
                                                   const cx<T> *__restrict__ r,
                                                   cx<T> *__restrict__ X, int P, int n1,
                                                   long long nf, long long xrows) {
  const Sub s = subs[blockIdx.y];
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= s.nOm) return;
  const long long q = blockIdx.z;
  const long long g = i < s.nU ? u_global(s, i, P, n1) : om_node(s, eidx[s.eoff + i - s.nU], P, n1);
  X[q * xrows + s.xoff + i] = r[q * nf + g];
}

template <typename TB, typename T>
__global__ __launch_bounds__(256) void k_dd_sym(const Sub *__restrict__ subs,
                                                const cx<TB> *__restrict__ B,
                                                const cx<T> *__restrict__ X, cx<T> *__restrict__ Y,
                                                cx<T> *__restrict__ Pp, long long xrows,
                                                long long yrows, long long prows, int nrhs) {
  constexpr int ST = kSymTile;
  // double-buffered: the partial of a tile is reduced from one buffer while the
  // next tile fills the other, one barrier per tile
  __shared__ cx<T> red[2][16][ST + 1];
  const Sub s = subs[blockIdx.y];
  const int nrb = s.nrb, neb = s.neb, w = blockIdx.x;
  if (w >= (nrb + 1) / 2) return;  // uniform
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  const int nS = nrb * (nrb + 1) / 2, nE = s.nOm - s.nU;
  const cx<TB> *Bs = B + s.boff;
  int buf = 0;
  for (int q = 0; q < nrhs; ++q) {
    const cx<T> *xq = X + (long long)q * xrows + s.xoff;  // U nodes, then ring nodes
    for (int pass = 0; pass < 2; ++pass) {
      const int a = pass == 0 ? w : nrb - 1 - w;
      if (pass == 1 && a == w) break;  // middle block of an odd count
      cx<T> xa[4], acc[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int j = a * ST + 4 * ty + i;
        xa[i] = j < s.nU ? xq[j] : cx<T>{0, 0};
        acc[i] = {0, 0};
      }
      for (int b = a; b < nrb; ++b) {
        const cx<TB> *tile = Bs + (long long)sym_tile(a, b, nrb) * (ST * ST);
        cx<T> xb[4], pb[4];
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
          const int j = b * ST + tx + 16 * jj;
          xb[jj] = j < s.nU ? xq[j] : cx<T>{0, 0};
          pb[jj] = {0, 0};
        }
        cx<T> v[4][4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int jj = 0; jj < 4; ++jj)
            v[i][jj] = ccast<T>(ld_stream(tile + (4 * ty + i) * ST + tx + 16 * jj));
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int jj = 0; jj < 4; ++jj) {
            cmac(acc[i], v[i][jj], xb[jj]);
            cmac(pb[jj], v[i][jj], xa[i]);
          }
        if (b > a) {  // uniform: transposed contribution to the rows of block b
#pragma unroll
          for (int jj = 0; jj < 4; ++jj) red[buf][ty][tx + 16 * jj] = pb[jj];
          __syncthreads();
          if (threadIdx.x < ST) {
            cx<T> sum = {0, 0};
            for (int t = 0; t < 16; ++t) sum = sum + red[buf][t][threadIdx.x];
            Pp[(long long)q * prows + s.poff + (long long)sym_tile(a, b, nrb) * ST + threadIdx.x] =
                sum;
          }
          buf ^= 1;
        }
      }
      for (int e = 0; e < neb; ++e) {
        const cx<TB> *tile = Bs + (long long)(nS + a * neb + e) * (ST * ST);
        cx<T> xe[4];
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
          const int k = e * ST + tx + 16 * jj;
          xe[jj] = k < nE ? xq[s.nU + k] : cx<T>{0, 0};
        }
        cx<T> v[4][4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int jj = 0; jj < 4; ++jj)
            v[i][jj] = ccast<T>(ld_stream(tile + (4 * ty + i) * ST + tx + 16 * jj));
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int jj = 0; jj < 4; ++jj) cmac(acc[i], v[i][jj], xe[jj]);
      }
      // sum the 16 column owners of each row (lanes 16 ty .. 16 ty + 15)
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int o = 8; o > 0; o >>= 1) {
          acc[i].re += __shfl_xor(acc[i].re, o, 64);
          acc[i].im += __shfl_xor(acc[i].im, o, 64);
        }
      if (tx == 0) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int j = a * ST + 4 * ty + i;
          if (j < s.nU) Y[(long long)q * yrows + s.yoff + j] = acc[i];
        }
      }
    }
  }
}

// Y_i[j] = (Y_i[j] + sum_{a < j / 64} partial(a, j / 64)[j % 64]) / L_j, the
// partials added in ascending a.
template <typename T>
__global__ __launch_bounds__(256) void k_dd_symred(const Sub *__restrict__ subs,
                                                   const int *__restrict__ nblk,
                                                   const cx<T> *__restrict__ Pp,
                                                   cx<T> *__restrict__ Y, int P, long long yrows,
                                                   long long prows) {
  constexpr int ST = kSymTile;
  const Sub s = subs[blockIdx.y];
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= s.nU) return;
  const long long q = blockIdx.z;
  const int b = j / ST, c = j % ST;
  cx<T> *y = Y + q * yrows + s.yoff + j;
  cx<T> acc = *y;
  const cx<T> *pp = Pp + q * prows + s.poff + c;
  for (int a = 0; a < b; ++a) acc = acc + pp[(long long)sym_tile(a, b, s.nrb) * ST];
  int gn[3], uj;
  u_node(s, j, P, gn, uj);
  const T invL = (T)(1.0 / (double)(nblk[2 * gn[0] + 1] * nblk[2 * gn[1] + 1] * nblk[2 * gn[2] + 1]));
  *y = cx<T>{acc.re * invL, acc.im * invL};
}

template <typename TB, typename T>
static int dd_sym_t(const th_ctx *c, const void *r, void *y, int nrhs, hipStream_t s) {
  const unsigned nsub = (unsigned)c->subs.size();
  hipLaunchKernelGGL((k_dd_gather<T>), dim3(ceil_div(c->max_nom, 256), nsub, nrhs), dim3(256), 0,
                     s, c->d_subs, (const int *)c->d_eidx, (const cx<T> *)r, (cx<T> *)c->w_x, c->P,
                     c->n1, c->nf, c->x_rows);
  hipLaunchKernelGGL((k_dd_sym<TB, T>), dim3(c->max_pairs, nsub), dim3(256), 0, s, c->d_subs,
                     (const cx<TB> *)c->d_B, (const cx<T> *)c->w_x, (cx<T> *)y, (cx<T> *)c->w_p,
                     c->x_rows, c->y_rows, c->p_rows, nrhs);
  hipLaunchKernelGGL((k_dd_symred<T>), dim3(ceil_div(c->max_ldb, 256), nsub, nrhs), dim3(256), 0,
                     s, c->d_subs, (const int *)c->d_nblk, (const cx<T> *)c->w_p, (cx<T> *)y,
                     c->P, c->y_rows, c->p_rows);
  TH_HIP_CHECK_RET(hipGetLastError());
  return 0;
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

// ---------------------------------------------------------------------------
// FP64 operators with many right-hand sides: Y_i = B_i X_i as a complex GEMM
// on the FP64 matrix cores (v_mfma_f64_16x16x4f64, four real products per
// complex one).  The patches X_i are first gathered into [subdomain][k][Rp]
// (right-hand sides fastest, Rp a multiple of 16), so both MFMA operands are
// read straight from memory: the B_i fragment (16 rows x 4 columns) as four
// 256-byte row segments of the dense 64-row-block layout, the X fragment (4
// columns x 16 right-hand sides) as four 256-byte segments of the gathered
// patch.  A workgroup owns one 16-row block of one subdomain, its wavefronts
// one block of 16 right-hand sides each (the B_i fragment is shared through
// the cache); workgroups of one subdomain sit on one XCD so that its patch
// stays in one L2.
typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int kXgTileK = 64;  // patch rows per workgroup of the gather

__global__ __launch_bounds__(256) void k_dd_gatherx(const Sub *__restrict__ subs,
                                                    const c64 *__restrict__ r,
                                                    c64 *__restrict__ Xg, int P, int n1,
                                                    long long nf, int nrhs, int Rp) {
  __shared__ c64 T[16][kXgTileK + 1];
  const Sub s = subs[blockIdx.y];
  const int k0 = blockIdx.x * kXgTileK;
  if (k0 >= s.nOm) return;  // uniform
  c64 *xo = Xg + s.xoff * Rp;
  for (int q0 = 0; q0 < Rp; q0 += 16) {
    // read 16 right-hand sides x 64 patch nodes, coalesced along the nodes
    for (int t = threadIdx.x; t < 16 * kXgTileK; t += 256) {
      const int kk = t % kXgTileK, qq = t / kXgTileK;
      const int k = k0 + kk, q = q0 + qq;
      T[qq][kk] = (k < s.nOm && q < nrhs) ? r[(long long)q * nf + om_node(s, k, P, n1)] : c64{0, 0};
    }
    __syncthreads();
    // write them right-hand sides fastest
    for (int t = threadIdx.x; t < 16 * kXgTileK; t += 256) {
      const int qq = t % 16, kk = t / 16;
      if (k0 + kk < s.nOm) xo[(long long)(k0 + kk) * Rp + q0 + qq] = T[qq][kk];
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void k_dd_mfma64(const Sub *__restrict__ subs, int nsub,
                                                   int nrb, const c64 *__restrict__ B,
                                                   const c64 *__restrict__ Xg,
                                                   c64 *__restrict__ Y, long long yrows,
                                                   int nrhs, int Rp) {
  // XCD-aware mapping: workgroup b runs on XCD b % 8; subdomain si on XCD si % 8
  const int b = blockIdx.x;
  const int si = (b & 7) + 8 * ((b >> 3) / nrb), rb = (b >> 3) % nrb;
  if (si >= nsub) return;
  const Sub s = subs[si];
  if (rb * 16 >= s.nU) return;  // uniform
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int kl = lane >> 4, cl = lane & 15;
  const c64 *Ab = B + s.boff + (long long)(rb >> 2) * s.nOm * 64 + (rb & 3) * 16 + cl;
  const c64 *Xi = Xg + s.xoff * Rp;
  for (int cb = wave; cb * 16 < nrhs; cb += 4) {
    f64x4 cre = {0, 0, 0, 0}, cim = {0, 0, 0, 0};
    const c64 *Xb = Xi + cb * 16 + cl;
    // four k-steps per pass: their eight operand loads are issued before the
    // sixteen MFMAs that use them
    for (int k0 = 0; k0 < s.nOm; k0 += 16) {
      c64 a[4], x[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int k = k0 + 4 * u + kl;
        const bool ok = k < s.nOm;
        a[u] = ok ? Ab[(long long)k * 64] : c64{0, 0};
        x[u] = ok ? Xb[(long long)k * Rp] : c64{0, 0};
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        cre = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u].re, x[u].re, cre, 0, 0, 0);
        cre = __builtin_amdgcn_mfma_f64_16x16x4f64(-a[u].im, x[u].im, cre, 0, 0, 0);
        cim = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u].re, x[u].im, cim, 0, 0, 0);
        cim = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u].im, x[u].re, cim, 0, 0, 0);
      }
    }
    // lane: right-hand side cb * 16 + cl; its value i is row rb * 16 + 4 i + kl
    // (the FP64 16x16 result interleaves rows over the lane quarters)
    const int q = cb * 16 + cl;
    if (q < nrhs) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = rb * 16 + 4 * i + kl;
        if (row < s.nU) Y[(long long)q * yrows + s.yoff + row] = c64{cre[i], cim[i]};
      }
    }
  }
}

// right-hand sides from which the FP64 dense apply runs on the matrix cores
constexpr int kMfma64MinRhs = 16;

int dd_mfma64_rhs_pad(int max_rhs) { return max_rhs >= kMfma64MinRhs ? ceil_div(max_rhs, 16) * 16 : 0; }

static int dd_apply_mfma64(const th_ctx *c, const void *r, void *y, int nrhs, hipStream_t s) {
  const int nsub = (int)c->subs.size();
  const int Rp = dd_mfma64_rhs_pad(c->desc.max_rhs);
  int nrb = 0;
  for (const Sub &sb : c->subs) nrb = std::max(nrb, ceil_div(sb.nU, 16));
  hipLaunchKernelGGL(k_dd_gatherx, dim3(ceil_div(c->max_nom, kXgTileK), nsub), dim3(256), 0, s,
                     c->d_subs, (const c64 *)r, (c64 *)c->w_x, c->P, c->n1, c->nf, nrhs, Rp);
  const int groups = ceil_div(nsub, 8);
  hipLaunchKernelGGL(k_dd_mfma64, dim3(8 * groups * nrb), dim3(256), 0, s, c->d_subs, nsub, nrb,
                     (const c64 *)c->d_B, (const c64 *)c->w_x, (c64 *)y, c->y_rows, nrhs, Rp);
  TH_HIP_CHECK_RET(hipGetLastError());
  return 0;
}

template <typename TB, typename T>
static int dd_apply_t(const th_ctx *c, const void *r, void *y, int nrhs, hipStream_t s) {
  if (std::is_same<TB, double>::value && std::is_same<T, double>::value && c->layout == 0 &&
      nrhs >= kMfma64MinRhs && dd_mfma64_rhs_pad(c->desc.max_rhs) > 0)
    return dd_apply_mfma64(c, r, y, nrhs, s);
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
  if (c->layout == 3) return launch_dd_slab(c, r, y, nrhs, f32, s);
  switch (c->desc.gemm) {
    case TH_GEMM_BF16:
      return launch_dd_mfma(c, r, y, nrhs, f32, c->mfma_cfg, c->mfma_grid, s);
    case TH_GEMM_F64:
      if (c->layout == 1)
        return f32 ? dd_sym_t<double, float>(c, r, y, nrhs, s)
                   : dd_sym_t<double, double>(c, r, y, nrhs, s);
      return f32 ? dd_apply_t<double, float>(c, r, y, nrhs, s)
                 : dd_apply_t<double, double>(c, r, y, nrhs, s);
    case TH_GEMM_F32:
      if (c->layout == 1)
        return f32 ? dd_sym_t<float, float>(c, r, y, nrhs, s)
                   : dd_sym_t<float, double>(c, r, y, nrhs, s);
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
  // the staged matrix-core kernel leaves its results in the colour planes
  if (c->layout == 2 && mfma_cfg_staged(c->mfma_cfg))
    return launch_dd_accum_col(c, u, nrhs, f32, assign, s);
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
