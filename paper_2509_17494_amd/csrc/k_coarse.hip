// Coarse-level direct solve in FP64 (Alg. 1, "solve A_c u_c = r_c"; the paper
// uses a direct solver and notes that approximate ones may be used).
//
// The quasi-FE QSFEM matrix (Sec. 3.3) is a 9-point (2-D) or 27-point (3-D)
// stencil on the coarse vertex grid.  Grouping K consecutive slabs (grid
// lines of constant y in 2-D, planes of constant z in 3-D) into a super-block
// makes it block tridiagonal, and the coupling between super-blocks J-1 and J
// only links the last slab of J-1 with the first slab of J (3 or 9 in-slab
// neighbours per vertex).  Setup (once, timed separately) runs the block
// elimination in natural order
//   S_0 = T_0,   S_J = T_J - L_J S_{J-1}^{-1} U_{J-1},   G_J = S_J^{-1},
// where L_J S_{J-1}^{-1} U_{J-1} only touches the first-slab block of S_J and
// only needs the last-slab block of G_{J-1}.  When the right-hand sides of a
// slab fit in LDS the elimination is twisted: blocks above a middle block m
// are eliminated downwards as above, blocks below it upwards,
//   S_J = T_J - U_J S_{J+1}^{-1} L_{J+1}   (last-slab block only),
// and m takes both corrections, so the two chains run side by side and a
// solve needs about half the sequential launches.  Every S_J is inverted by the
// same Gauss-Jordan kernels as the subdomain operators (no pivoting: natural
// order elimination of these matrices is stable, checked against pivoted
// sparse LU).  The solve is
//   forward   y_J = G_J (r_J - L_J y_{J-1})   (upward chain: r_J - U_J y_{J+1})
//   backward  x_J = y_J - G_J[:, last slab] (U_J x_{J+1}[first slab])
//             (upward chain: y_J - G_J[:, first slab] (L_J x_{J-1}[last slab])),
// each a bandwidth-bound GEMV: for slabs whose right-hand sides fit in LDS one
// launch per step with one wavefront per output row (coalesced row reads of
// G_J, fixed-order wavefront reductions); for larger (3-D) slabs a GEMV that
// reads G_J through its symmetry with one thread per output row, over column
// chunks summed in a fixed order.  K trades the bytes of G (proportional to K)
// against the number of sequential launches (~2 ny / K).
#include <algorithm>
#include <cmath>
#include <vector>

#include "ctx.hpp"

namespace th {

// wavefronts (rows) per workgroup in the small-slab sweeps for RC right-hand
// sides per pass: every workgroup stages the block's right-hand side, and 16
// halve that redundancy against 8 (1.43 -> 1.35 ms per C2 coarse solve, one
// right-hand side); with 4 right-hand sides the larger register footprint
// makes 16 slower (C3: 1.81 -> 2.09 ms of coarse sweeps per solve)
__host__ __device__ constexpr int sweep_waves(int rc) { return rc == 1 ? 16 : 8; }
constexpr int kAhead = 8;  // row entries per lane loaded before the right-hand side is staged
constexpr int kCoarseChunk = 256;  // columns per partial sum of the large-slab GEMV

// In-slab neighbourhood: C = 3 codes dx + 1 along a line (2-D), C = 9 codes
// (dy + 1) 3 + dx + 1 in a plane (3-D).  The code from b back to a is C - 1 - code.
__device__ __forceinline__ int slab_nbr(int a, int code, int nx, int C) {
  if (C == 3) {
    const int x = a + code - 1;
    return (x >= 0 && x < nx) ? x : -1;
  }
  const int y = a / nx + code / 3 - 1, x = a % nx + code % 3 - 1;
  return (x >= 0 && x < nx && y >= 0 && y < nx) ? y * nx + x : -1;
}

__device__ __forceinline__ int slab_code(int a, int b, int nx, int C) {
  if (C == 3) {
    const int d = b - a;
    return (d >= -1 && d <= 1) ? d + 1 : -1;
  }
  const int dy = b / nx - a / nx, dx = b % nx - a % nx;
  return (dy >= -1 && dy <= 1 && dx >= -1 && dx <= 1) ? (dy + 1) * 3 + dx + 1 : -1;
}

// S_J (ld x ld, identity padding) written over the G_J slot; with rev its
// nb x nb part in reversed node order.
__global__ __launch_bounds__(256) void k_build_s(c64 *__restrict__ S, int ld, int nb, int nx,
                                                 int L, int C, int line0,
                                                 const c64 *__restrict__ st,
                                                 const c64 *__restrict__ Gp, int ldp, int kp,
                                                 const c64 *__restrict__ Gn, int ldn, int rev) {
  const long long t = blockIdx.x * 256LL + threadIdx.x;
  if (t >= (long long)ld * ld) return;
  int a = (int)(t / ld), b = (int)(t % ld);
  if (rev && a < nb && b < nb) {  // the block in reversed node order
    a = nb - 1 - a;
    b = nb - 1 - b;
  }
  const int SC = 3 * C;
  c64 v = {0, 0};
  if (a >= nb || b >= nb) {
    v = (a == b) ? c64{1.0, 0.0} : c64{0, 0};
  } else {
    const int la = a / L, ca = a - la * L, lb = b / L, cb = b - lb * L;
    const int ds = lb - la;
    const long long ga = (long long)(line0 + la) * L + ca;
    if (ds >= -1 && ds <= 1) {
      const int code = slab_code(ca, cb, nx, C);
      if (code >= 0) v = st[SC * ga + (ds + 1) * C + code];
    }
    if (Gp && la == 0 && lb == 0) {
      // - sum_{c,d} L[ca][c] G_{J-1}[last c][last d] U[d][cb]
      const long long off = (long long)(kp - 1) * L;
      for (int c1 = 0; c1 < C; ++c1) {
        const int c = slab_nbr(ca, c1, nx, C);
        if (c < 0) continue;
        const c64 l = st[SC * ga + c1];
        c64 sum = {0, 0};
        for (int c2 = 0; c2 < C; ++c2) {
          const int d = slab_nbr(cb, c2, nx, C);
          if (d < 0) continue;
          const long long gd = (long long)(line0 - 1) * L + d;
          const c64 u = st[SC * gd + 2 * C + (C - 1 - c2)];
          cmac(sum, Gp[(off + c) * ldp + off + d], u);
        }
        v = v - l * sum;
      }
    }
    const int kJ = nb / L;
    if (Gn && la == kJ - 1 && lb == kJ - 1) {
      // - sum_{c,d} U[ca][c] G_{J+1}[first c][first d] L[d][cb]  (L[d][cb] = U[cb][d])
      const long long gb = (long long)(line0 + lb) * L + cb;
      for (int c1 = 0; c1 < C; ++c1) {
        const int c = slab_nbr(ca, c1, nx, C);
        if (c < 0) continue;
        const c64 u = st[SC * ga + 2 * C + c1];
        c64 sum = {0, 0};
        for (int c2 = 0; c2 < C; ++c2) {
          const int d = slab_nbr(cb, c2, nx, C);
          if (d < 0) continue;
          cmac(sum, Gn[(long long)c * ldn + d], st[SC * gb + 2 * C + c2]);
        }
        v = v - u * sum;
      }
    }
  }
  S[t] = v;
}

// G[a][b] <-> G[nb-1-a][nb-1-b] for a, b < nb: back to natural order after the
// inversion of a block built in reversed order
__global__ __launch_bounds__(256) void k_reverse_block(c64 *__restrict__ G, int ld, int nb) {
  const long long t = blockIdx.x * 256LL + threadIdx.x;
  const long long n2 = (long long)nb * nb;
  if (t >= n2 / 2) return;
  const int a = (int)(t / nb), b = (int)(t % nb);
  c64 &x = G[(long long)a * ld + b];
  c64 &y = G[(long long)(nb - 1 - a) * ld + nb - 1 - b];
  const c64 v = x;
  x = y;
  y = v;
}

__device__ __forceinline__ c64 wave_sum(c64 v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    v.re += __shfl_xor(v.re, o, 64);
    v.im += __shfl_xor(v.im, o, 64);
  }
  return v;
}

// right-hand side of the forward step of super-block J: r_J - L_J y_{J-1}
__device__ __forceinline__ c64 fwd_rhs(int a, int r, int nx, int L, int C, int line0,
                                       const c64 *__restrict__ st, const c64 *__restrict__ rc,
                                       const c64 *__restrict__ uc, long long ncn, int has_prev) {
  const long long g = (long long)line0 * L + a;
  c64 v = rc[r * ncn + g];
  if (has_prev && a < L) {
    const c64 *s = st + 3 * C * g;
    for (int code = 0; code < C; ++code) {
      const int c = slab_nbr(a, code, nx, C);
      if (c >= 0) v = v - s[code] * uc[r * ncn + (long long)(line0 - 1) * L + c];
    }
  }
  return v;
}

// U_J x_{J+1}[first slab] at position c of the last slab of J (lend = first slab of J+1)
__device__ __forceinline__ c64 bwd_rhs(int c, int r, int nx, int L, int C, int lend,
                                       const c64 *__restrict__ st, const c64 *__restrict__ uc,
                                       long long ncn) {
  const long long gc = (long long)(lend - 1) * L + c;
  const c64 *s = st + 3 * C * gc + 2 * C;
  c64 v = {0, 0};
  for (int code = 0; code < C; ++code) {
    const int d = slab_nbr(c, code, nx, C);
    if (d >= 0) cmac(v, s[code], uc[r * ncn + (long long)lend * L + d]);
  }
  return v;
}

// Staging in global memory for slabs whose right-hand sides do not fit in
// LDS, interleaved by column: xg[i nrhs + r] for r < nrhs, i < n, n = nb
// (forward) or L (backward).
__global__ __launch_bounds__(256) void k_cstage(int fwd, int n, int nx, int L, int C, int slab,
                                                const c64 *__restrict__ st,
                                                const c64 *__restrict__ rc,
                                                const c64 *__restrict__ uc, c64 *__restrict__ xg,
                                                int nrhs, long long ncn, int has_prev) {
  const long long tot = (long long)n * nrhs;
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < tot; i += (long long)gridDim.x * 256) {
    const int a = (int)(i / nrhs), r = (int)(i - (long long)a * nrhs);
    xg[i] = fwd ? fwd_rhs(a, r, nx, L, C, slab, st, rc, uc, ncn, has_prev)
                : bwd_rhs(a, r, nx, L, C, slab, st, uc, ncn);
  }
}

// Sweep GEMV for large slabs, y_a = sum_b G[a][col0 + b] x_b for the rows a of
// one super-block and RC right-hand sides.  S_J is complex symmetric (A_c is,
// and the Schur complement keeps it), so G_J = S_J^{-1} is too and the product
// is formed as sum_b G[col0 + b][a] x_b: every thread owns one output row a,
// every load instruction of a wavefront reads 64 consecutive entries of one
// row of G (1 KiB), and x_b is the same for the whole wavefront (broadcast
// LDS reads of the chunk's right-hand sides, staged once per workgroup).  No
// cross-lane sums.  The columns are split in chunks of kCoarseChunk; chunk k
// writes its partial sums to part[(k nrhs + q) nrows + a], and k_cpartsum adds
// them in chunk order.
template <int RC>
__global__ __launch_bounds__(256) void k_cgemv_t(const c64 *__restrict__ G, int ld, int nrows,
                                                 int col0, int ncols,
                                                 const c64 *__restrict__ xg,
                                                 c64 *__restrict__ part, int nrhs) {
  constexpr int U = 8;  // rows of G in flight per thread
  __shared__ c64 xs[kCoarseChunk][RC];
  const int ch = blockIdx.y, r0 = blockIdx.z * RC;
  const int b0 = ch * kCoarseChunk, nbk = min(kCoarseChunk, ncols - b0);
  const int nq = min(RC, nrhs - r0);
  for (int t = threadIdx.x; t < kCoarseChunk * RC; t += 256) {
    const int b = t / RC, q = t - b * RC;
    xs[b][q] = (b < nbk && q < nq) ? xg[(long long)(b0 + b) * nrhs + r0 + q] : c64{0, 0};
  }
  __syncthreads();
  const int a = blockIdx.x * 256 + threadIdx.x;
  if (a >= nrows) return;
  c64 acc[RC];
#pragma unroll
  for (int q = 0; q < RC; ++q) acc[q] = {0, 0};
  const c64 *gp = G + (long long)(col0 + b0) * ld + a;
  for (int b = 0; b < nbk; b += U) {  // b + u < kCoarseChunk: xs beyond nbk holds zeros
    c64 g[U];
#pragma unroll
    for (int u = 0; u < U; ++u)
      g[u] = b + u < nbk ? ld_stream(gp + (long long)(b + u) * ld) : c64{0, 0};
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int q = 0; q < RC; ++q) cmac(acc[q], g[u], xs[b + u][q]);
  }
#pragma unroll
  for (int q = 0; q < RC; ++q)
    if (q < nq) part[((long long)ch * nrhs + r0 + q) * nrows + a] = acc[q];
}

// uc[row0 + a] = sum_k part[k][q][a] (sub = 0) or uc[row0 + a] -= that sum
// (sub = 1), the chunks added in ascending order.
__global__ __launch_bounds__(256) void k_cpartsum(const c64 *__restrict__ part, int nch, int nrows,
                                                  int nrhs, c64 *__restrict__ uc, long long row0,
                                                  long long ncn, int sub) {
  const long long t = blockIdx.x * 256LL + threadIdx.x;
  if (t >= (long long)nrows * nrhs) return;
  const int q = (int)(t / nrows), a = (int)(t - (long long)q * nrows);
  c64 sm = {0, 0};
  for (int k = 0; k < nch; ++k) sm = sm + part[((long long)k * nrhs + q) * nrows + a];
  c64 *p = uc + q * ncn + row0 + a;
  *p = sub ? *p - sm : sm;
}

// One super-block of a sweep step (small slabs).  Forward: the right-hand side
// r_J, minus L_J y_{J-1} on the first slab when prev, minus U_J y_{J+1} on the
// last slab when next.  Backward: x_J -= G_J[:, col slab] w with w = U_J
// x_{J+1}[first slab] (up = 0, col slab = last) or w = L_J x_{J-1}[last slab]
// (up = 1, col slab = first).
struct SweepBlk {
  const c64 *G;
  int ld, nb, line0, kJ;
  int prev, next, up;
};

// forward step of up to two super-blocks (blockIdx.z), one wavefront per row
// of G_J, the right-hand side staged in LDS
template <int RC>
__global__ __launch_bounds__(64 * sweep_waves(RC)) void k_cfwd(SweepBlk b0, SweepBlk b1, int nx, int L, int C,
                                                  const c64 *__restrict__ st,
                                                  const c64 *__restrict__ rc, c64 *__restrict__ uc,
                                                  int nrhs, long long ncn) {
  extern __shared__ c64 tsh[];  // RC x nb
  const SweepBlk B = blockIdx.z == 0 ? b0 : b1;
  const int nb = B.nb, line0 = B.line0;
  const int r0 = blockIdx.y * RC;
  const int SC = 3 * C;
  const c64 *xs = tsh;
  // the first kAhead entries of the wavefront's row are loaded before the
  // right-hand side is staged (they do not depend on it)
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int arow = blockIdx.x * sweep_waves(RC) + wave;
  const bool once = gridDim.y == 1;  // rows streamed once when one pass covers all RHS
  const c64 *row = B.G + (long long)min(arow, nb - 1) * B.ld;
  c64 gah[kAhead];
#pragma unroll
  for (int u = 0; u < kAhead; ++u) {
    const int b = lane + 64 * u;
    gah[u] = b < nb ? (once ? ld_stream(row + b) : row[b]) : c64{0, 0};
  }
  for (int i = threadIdx.x; i < nb * RC; i += blockDim.x) {
    const int q = i / nb, a = i - q * nb;
    const int r = r0 + q;
    c64 v = {0, 0};
    if (r < nrhs) {
      const long long g = (long long)line0 * L + a;
      v = rc[r * ncn + g];
      if (B.prev && a < L) {
        for (int code = 0; code < C; ++code) {
          const int c = slab_nbr(a, code, nx, C);
          if (c >= 0) v = v - st[SC * g + code] * uc[r * ncn + (long long)(line0 - 1) * L + c];
        }
      }
      const int al = a - (B.kJ - 1) * L;
      if (B.next && al >= 0) {
        for (int code = 0; code < C; ++code) {
          const int c = slab_nbr(al, code, nx, C);
          if (c >= 0)
            v = v - st[SC * g + 2 * C + code] * uc[r * ncn + (long long)(line0 + B.kJ) * L + c];
        }
      }
    }
    tsh[q * nb + a] = v;
  }
  __syncthreads();
  const int a = arow;
  if (a >= nb) return;
  c64 acc[RC];
#pragma unroll
  for (int q = 0; q < RC; ++q) acc[q] = {0, 0};
#pragma unroll
  for (int u = 0; u < kAhead; ++u) {
    const int b = lane + 64 * u;
    if (b < nb)
#pragma unroll
      for (int q = 0; q < RC; ++q) cmac(acc[q], gah[u], xs[q * nb + b]);
  }
  constexpr int UNR = RC == 1 ? 8 : 4;  // deeper unrolling only where registers allow
#pragma unroll UNR
  for (int b = lane + 64 * kAhead; b < nb; b += 64) {
    const c64 g = once ? ld_stream(row + b) : row[b];
#pragma unroll
    for (int q = 0; q < RC; ++q) cmac(acc[q], g, xs[q * nb + b]);
  }
#pragma unroll
  for (int q = 0; q < RC; ++q) {
    const c64 sm = wave_sum(acc[q]);
    if (lane == 0 && r0 + q < nrhs) uc[(r0 + q) * ncn + (long long)line0 * L + a] = sm;
  }
}

// backward step of up to two super-blocks (blockIdx.z)
template <int RC>
__global__ __launch_bounds__(64 * sweep_waves(RC)) void k_cbwd(SweepBlk b0, SweepBlk b1, int nx, int L, int C,
                                                  const c64 *__restrict__ st, c64 *__restrict__ uc,
                                                  int nrhs, long long ncn) {
  extern __shared__ c64 wsh[];  // RC x L
  const SweepBlk B = blockIdx.z == 0 ? b0 : b1;
  const int nb = B.nb, line0 = B.line0;
  const int r0 = blockIdx.y * RC;
  const int SC = 3 * C;
  const c64 *ws = wsh;
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int arow = blockIdx.x * sweep_waves(RC) + wave;
  const bool once = gridDim.y == 1;
  const c64 *row = B.G + (long long)min(arow, nb - 1) * B.ld + (B.up ? 0 : (long long)(B.kJ - 1) * L);
  c64 gah[kAhead];
#pragma unroll
  for (int u = 0; u < kAhead; ++u) {
    const int c = lane + 64 * u;
    gah[u] = c < L ? (once ? ld_stream(row + c) : row[c]) : c64{0, 0};
  }
  for (int i = threadIdx.x; i < L * RC; i += blockDim.x) {
    const int q = i / L, c = i - q * L;
    const int r = r0 + q;
    c64 v = {0, 0};
    if (r < nrhs) {
      if (B.up) {  // L_J x_{J-1}[last slab] at position c of the first slab of J
        const long long gc = (long long)line0 * L + c;
        for (int code = 0; code < C; ++code) {
          const int d = slab_nbr(c, code, nx, C);
          if (d >= 0) cmac(v, st[SC * gc + code], uc[r * ncn + (long long)(line0 - 1) * L + d]);
        }
      } else {
        v = bwd_rhs(c, r, nx, L, C, line0 + B.kJ, st, uc, ncn);
      }
    }
    wsh[q * L + c] = v;
  }
  __syncthreads();
  const int a = arow;
  if (a >= nb) return;
  c64 acc[RC];
#pragma unroll
  for (int q = 0; q < RC; ++q) acc[q] = {0, 0};
#pragma unroll
  for (int u = 0; u < kAhead; ++u) {
    const int c = lane + 64 * u;
    if (c < L)
#pragma unroll
      for (int q = 0; q < RC; ++q) cmac(acc[q], gah[u], ws[q * L + c]);
  }
#pragma unroll 4
  for (int c = lane + 64 * kAhead; c < L; c += 64) {
    const c64 g = once ? ld_stream(row + c) : row[c];
#pragma unroll
    for (int q = 0; q < RC; ++q) cmac(acc[q], g, ws[q * L + c]);
  }
#pragma unroll
  for (int q = 0; q < RC; ++q) {
    const c64 sm = wave_sum(acc[q]);
    if (lane == 0 && r0 + q < nrhs) {
      c64 *p = uc + (r0 + q) * ncn + (long long)line0 * L + a;
      *p = *p - sm;
    }
  }
}

// Number of slabs per super-block: minimise the modelled solve time
// (K + 1) ny L^2 16 B / BW  +  launches x latency, with G within a memory
// budget; slab right-hand sides up to 64 KiB are staged in LDS.  With at least
// three super-blocks the sweeps are twisted (ceil(ny / K) + 1 launches, else
// 2 ceil(ny / K) - 1).  BW and latency are a least-squares fit of measured
// coarse solves over K = 3..10 at ny = L = 401 (8 wavefronts per workgroup;
// with 16 the measured optimum stays at K = 4).
static int choose_lines(int L, int ny, int rc_chunk, int passes) {
  const double bw = 6.3e12, lat = 7.3e-6;
  const int nb_max = std::min(4096, 65536 / (16 * rc_chunk));
  const int kmax = std::max(1, std::min(ny, nb_max / L));
  int best = 1;
  double best_t = 1e300;
  for (int K = 1; K <= kmax; ++K) {
    const double bytes = (double)(K + 1) * ny * L * (double)L * 16.0 * passes;
    if (K > 1 && (double)ny * K * L * (double)L * 16.0 > 24e9) break;
    const double nblk = std::ceil((double)ny / K);
    const double launches = nblk >= 3 ? nblk + 1 : 2 * nblk - 1;
    const double t = bytes / bw + launches * lat;
    if (t < best_t) {
      best_t = t;
      best = K;
    }
  }
  return best;
}

// Modelled time of one coarse solve by the line elimination (the model above
// at the K it chooses).
double coarse_model_lines(const th_ctx *c) {
  const int dim = c->dim, nx = c->nc1;
  const int L = dim == 3 ? nx * nx : nx, ny = nx;
  const int R = c->desc.max_rhs;
  const int rc_chunk = (R >= 4) ? 4 : (R >= 2 ? 2 : 1);
  const int passes = (R + rc_chunk - 1) / rc_chunk;
  const int K = choose_lines(L, ny, rc_chunk, passes);
  const double nblk = std::ceil((double)ny / K);
  const double launches = nblk >= 3 ? nblk + 1 : 2 * nblk - 1;
  return (double)(K + 1) * ny * L * (double)L * 16.0 * passes / 6.3e12 + launches * 7.3e-6;
}

int setup_coarse_factors(th_ctx *c, const std::vector<c64> &st) {
  hipStream_t s = c->stream;
  CoarseData &cd = c->coarse;
  const int nx = c->nc1;
  cd.dim = c->dim;
  cd.nx = nx;
  cd.L = c->dim == 3 ? nx * nx : nx;
  cd.ny = nx;
  cd.C = c->dim == 3 ? 9 : 3;
  const int L = cd.L, ny = cd.ny, C = cd.C;
  const int R = c->desc.max_rhs;
  cd.rc_chunk = (R >= 4) ? 4 : (R >= 2 ? 2 : 1);
  const int passes = (R + cd.rc_chunk - 1) / cd.rc_chunk;
  const int K = choose_lines(L, ny, cd.rc_chunk, passes);
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
    const int nb = (cd.line0[J + 1] - cd.line0[J]) * L;
    cd.ld[J] = ceil_div(nb, kGJBlock) * kGJBlock;
    cd.goff[J + 1] = cd.goff[J] + (long long)cd.ld[J] * cd.ld[J];
  }
  const size_t st_bytes = (size_t)L * ny * 3 * C * sizeof(c64);
  if (st.size() * sizeof(c64) != st_bytes) {
    set_error("coarse stencil has the wrong size");
    return TH_EINVAL;
  }
  int max_nb = 0, max_ld = 0;
  for (int J = 0; J < nblk; ++J) {
    max_nb = std::max(max_nb, (cd.line0[J + 1] - cd.line0[J]) * L);
    max_ld = std::max(max_ld, cd.ld[J]);
  }
  const size_t t_bytes = (size_t)max_nb * R * sizeof(c64);
  const size_t p_bytes = (size_t)ceil_div(max_nb, kCoarseChunk) * t_bytes;
  cd.bytes = cd.goff[nblk] * (long long)sizeof(c64) + (long long)st_bytes;
  c64 *pws = nullptr;
  if (hipMalloc(&cd.G, (size_t)cd.goff[nblk] * sizeof(c64)) != hipSuccess ||
      hipMalloc(&cd.st, st_bytes) != hipSuccess ||
      hipMalloc(&cd.tbuf, t_bytes) != hipSuccess ||
      hipMalloc(&cd.pbuf, p_bytes) != hipSuccess ||
      hipMalloc(&pws, gj_ws_bytes(1, max_ld)) != hipSuccess) {
    if (pws) (void)hipFree(pws);
    set_error("cannot allocate the coarse factors");
    return TH_ENOMEM;
  }
  TH_HIP_CHECK_RET(hipMemcpyAsync(cd.st, st.data(), st_bytes, hipMemcpyHostToDevice, s));
  if (int e = gj_ws_reset(pws, s)) {
    (void)hipFree(pws);
    return e;
  }
  // twisted elimination where the small-slab sweeps apply (at least 3 blocks)
  cd.mid = (nblk >= 3 && max_nb * cd.rc_chunk * (long long)sizeof(c64) <= 64 * 1024) ? nblk / 2 : -1;
  // block J with the correction from the block above (prev) and/or below (next).
  // Gauss-Jordan without pivoting eliminates in node order; a block of the
  // upward chain (corrected on its last slab) is eliminated in reversed order,
  // so that, as in the downward chain, the corrected slab goes first (in
  // natural order its pivots can become small).
  auto build = [&](int J, bool prev, bool next) -> int {
    const bool rev = next && !prev;
    const int ld = cd.ld[J], nb = (cd.line0[J + 1] - cd.line0[J]) * L;
    c64 *GJ = cd.G + cd.goff[J];
    const c64 *Gp = prev ? cd.G + cd.goff[J - 1] : nullptr;
    const int ldp = prev ? cd.ld[J - 1] : 0;
    const int kp = prev ? cd.line0[J] - cd.line0[J - 1] : 0;
    const c64 *Gn = next ? cd.G + cd.goff[J + 1] : nullptr;
    const int ldn = next ? cd.ld[J + 1] : 0;
    const long long tot = (long long)ld * ld;
    hipLaunchKernelGGL(k_build_s, dim3((unsigned)ceil_div_ll(tot, 256)), dim3(256), 0, s, GJ, ld,
                       nb, nx, L, C, cd.line0[J], (const c64 *)cd.st, Gp, ldp, kp, Gn, ldn,
                       rev ? 1 : 0);
    TH_HIP_CHECK_RET(hipGetLastError());
    const int rc = gj_invert_batched(GJ, ld, ld, tot, 1, s, pws);
    if (rc == 0 && rev) {
      hipLaunchKernelGGL(k_reverse_block, dim3((unsigned)ceil_div_ll((long long)nb * nb / 2 + 1, 256)),
                         dim3(256), 0, s, GJ, ld, nb);
      TH_HIP_CHECK_RET(hipGetLastError());
    }
    return rc;
  };
  int rc = 0;
  if (cd.mid < 0) {
    for (int J = 0; J < nblk && rc == 0; ++J) rc = build(J, J > 0, false);
  } else {
    const int m = cd.mid;
    for (int J = 0; J < m && rc == 0; ++J) rc = build(J, J > 0, false);
    for (int J = nblk - 1; J > m && rc == 0; --J) rc = build(J, false, J < nblk - 1);
    if (rc == 0) rc = build(m, true, true);
  }
  if (rc == 0) rc = gj_ws_status(pws, s, "the coarse factorisation");
  (void)hipStreamSynchronize(s);
  (void)hipFree(pws);
  return rc;
}

// Large slabs: per step one staging launch, one GEMV over column chunks and one
// fixed-order sum of the chunk partials; G streamed once per RC right-hand sides.
template <int RC>
static void gemv_large(const CoarseData &cd, const c64 *G, int ld, int nb, int col0, int ncols,
                       c64 *uc, long long row0, long long ncn, int nrhs, int sub,
                       hipStream_t s) {
  const int nch = ceil_div(ncols, kCoarseChunk);
  hipLaunchKernelGGL((k_cgemv_t<RC>), dim3(ceil_div(nb, 256), nch, ceil_div(nrhs, RC)), dim3(256),
                     0, s, G, ld, nb, col0, ncols, (const c64 *)cd.tbuf, cd.pbuf, nrhs);
  hipLaunchKernelGGL(k_cpartsum, dim3((unsigned)ceil_div_ll((long long)nb * nrhs, 256)), dim3(256),
                     0, s, (const c64 *)cd.pbuf, nch, nb, nrhs, uc, row0, ncn, sub);
}

template <int RC>
static int sweep_large_t(th_ctx *c, const c64 *rcv, c64 *uc, int nrhs, hipStream_t s) {
  const CoarseData &cd = c->coarse;
  const int nx = cd.nx, L = cd.L, C = cd.C;
  const long long ncn = (long long)L * cd.ny;
  for (int J = 0; J < cd.nblk; ++J) {
    const int nb = (cd.line0[J + 1] - cd.line0[J]) * L;
    const unsigned sb = (unsigned)std::min<long long>(ceil_div_ll((long long)nb * nrhs, 256), 2048);
    hipLaunchKernelGGL(k_cstage, dim3(sb), dim3(256), 0, s, 1, nb, nx, L, C, cd.line0[J],
                       (const c64 *)cd.st, rcv, (const c64 *)uc, cd.tbuf, nrhs, ncn,
                       J > 0 ? 1 : 0);
    gemv_large<RC>(cd, cd.G + cd.goff[J], cd.ld[J], nb, 0, nb, uc, (long long)cd.line0[J] * L,
                   ncn, nrhs, 0, s);
  }
  for (int J = cd.nblk - 2; J >= 0; --J) {
    const int kJ = cd.line0[J + 1] - cd.line0[J];
    const int nb = kJ * L;
    const unsigned sb = (unsigned)std::min<long long>(ceil_div_ll((long long)L * nrhs, 256), 2048);
    hipLaunchKernelGGL(k_cstage, dim3(sb), dim3(256), 0, s, 0, L, nx, L, C, cd.line0[J] + kJ,
                       (const c64 *)cd.st, (const c64 *)nullptr, (const c64 *)uc, cd.tbuf, nrhs,
                       ncn, 0);
    gemv_large<RC>(cd, cd.G + cd.goff[J], cd.ld[J], nb, (kJ - 1) * L, L, uc,
                   (long long)cd.line0[J] * L, ncn, nrhs, 1, s);
  }
  TH_HIP_CHECK_RET(hipGetLastError());
  return 0;
}

// Small slabs: the right-hand side of a step is formed in LDS by the GEMV
// launch itself (one launch per step; with the twisted elimination each
// launch carries one super-block of each chain).
template <int RC>
static int sweep_t(th_ctx *c, const c64 *rcv, c64 *uc, int nrhs, hipStream_t s) {
  const CoarseData &cd = c->coarse;
  const int nx = cd.nx, L = cd.L, C = cd.C;
  const long long ncn = (long long)L * cd.ny;
  const unsigned ychunks = (unsigned)ceil_div(nrhs, RC);
  int max_nb = 0;
  for (int J = 0; J < cd.nblk; ++J) max_nb = std::max(max_nb, (cd.line0[J + 1] - cd.line0[J]) * L);
  auto blk = [&](int J, int prev, int next, int up) {
    SweepBlk b;
    b.G = cd.G + cd.goff[J];
    b.ld = cd.ld[J];
    b.kJ = cd.line0[J + 1] - cd.line0[J];
    b.nb = b.kJ * L;
    b.line0 = cd.line0[J];
    b.prev = prev;
    b.next = next;
    b.up = up;
    return b;
  };
  auto fwd = [&](const SweepBlk &b0, const SweepBlk &b1, int nchain) {
    const int nb = std::max(b0.nb, nchain > 1 ? b1.nb : 0);
    hipLaunchKernelGGL((k_cfwd<RC>), dim3(ceil_div(nb, sweep_waves(RC)), ychunks, nchain),
                       dim3(64 * sweep_waves(RC)),
                       (size_t)max_nb * RC * sizeof(c64), s, b0, b1, nx, L, C, (const c64 *)cd.st,
                       rcv, uc, nrhs, ncn);
  };
  auto bwd = [&](const SweepBlk &b0, const SweepBlk &b1, int nchain) {
    const int nb = std::max(b0.nb, nchain > 1 ? b1.nb : 0);
    hipLaunchKernelGGL((k_cbwd<RC>), dim3(ceil_div(nb, sweep_waves(RC)), ychunks, nchain),
                       dim3(64 * sweep_waves(RC)),
                       (size_t)L * RC * sizeof(c64), s, b0, b1, nx, L, C, (const c64 *)cd.st, uc,
                       nrhs, ncn);
  };
  const int n = cd.nblk, m = cd.mid;
  if (m < 0) {  // top-down
    for (int J = 0; J < n; ++J) fwd(blk(J, J > 0, 0, 0), blk(J, J > 0, 0, 0), 1);
    for (int J = n - 2; J >= 0; --J) bwd(blk(J, 0, 0, 0), blk(J, 0, 0, 0), 1);
  } else {      // twisted: chains 0..m-1 downwards and n-1..m+1 upwards, then m
    const int nup = n - 1 - m, steps = std::max(m, nup);
    for (int i = 0; i < steps; ++i) {
      if (i < m && i < nup)
        fwd(blk(i, i > 0, 0, 0), blk(n - 1 - i, 0, i > 0, 0), 2);
      else if (i < m)
        fwd(blk(i, i > 0, 0, 0), blk(i, i > 0, 0, 0), 1);
      else
        fwd(blk(n - 1 - i, 0, i > 0, 0), blk(n - 1 - i, 0, i > 0, 0), 1);
    }
    fwd(blk(m, m > 0, m < n - 1, 0), blk(m, m > 0, m < n - 1, 0), 1);
    for (int i = 0; i < steps; ++i) {
      const int Jd = m - 1 - i, Ju = m + 1 + i;
      if (Jd >= 0 && Ju < n)
        bwd(blk(Jd, 0, 0, 0), blk(Ju, 0, 0, 1), 2);
      else if (Jd >= 0)
        bwd(blk(Jd, 0, 0, 0), blk(Jd, 0, 0, 0), 1);
      else
        bwd(blk(Ju, 0, 0, 1), blk(Ju, 0, 0, 1), 1);
    }
  }
  TH_HIP_CHECK_RET(hipGetLastError());
  return 0;
}

// LDS bytes the small-slab path needs for RC right-hand sides
static bool small_slabs_fit(const CoarseData &cd, int RC) {
  int max_nb = 0;
  for (int J = 0; J < cd.nblk; ++J) max_nb = std::max(max_nb, (cd.line0[J + 1] - cd.line0[J]) * cd.L);
  return (size_t)max_nb * RC * sizeof(c64) <= 64 * 1024;
}

bool coarse_lines_need_staging(const th_ctx *c) {
  return !small_slabs_fit(c->coarse, c->coarse.rc_chunk);
}

int launch_coarse_solve(th_ctx *c, const c64 *rcv, c64 *uc, int nrhs, hipStream_t s, int accuracy,
                        const CoarseScratch *ws) {
  if (c->coarse.kind == 1) return launch_coarse_nd(c, rcv, uc, nrhs, s, accuracy, ws);
  if (!small_slabs_fit(c->coarse, c->coarse.rc_chunk)) {
    if (nrhs >= 8) return sweep_large_t<8>(c, rcv, uc, nrhs, s);
    if (nrhs >= 4) return sweep_large_t<4>(c, rcv, uc, nrhs, s);
    if (nrhs >= 2) return sweep_large_t<2>(c, rcv, uc, nrhs, s);
    return sweep_large_t<1>(c, rcv, uc, nrhs, s);
  }
  switch (c->coarse.rc_chunk) {
    case 4: return sweep_t<4>(c, rcv, uc, nrhs, s);
    case 2: return sweep_t<2>(c, rcv, uc, nrhs, s);
    default: return sweep_t<1>(c, rcv, uc, nrhs, s);
  }
}

}  // namespace th
