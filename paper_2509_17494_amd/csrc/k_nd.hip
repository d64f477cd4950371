// Coarse-level direct solve by nested dissection (FP64).
//
// Alg. 1 solves A_c u_c = r_c with a direct solver; the paper names the
// coarse solve as the second costly step and allows other (approximate)
// solvers.  The coarse QSFEM matrix (Sec. 3.3) is a 9-point (2-D) or 27-point
// (3-D) stencil on the structured coarse vertex grid, so a plane of vertices
// one vertex thick separates the grid into two halves that do not couple.
// Nested dissection splits the vertex box recursively at the middle plane of
// its longest axis until a box holds at most `leafmax` vertices; every tree
// node sigma owns the vertices I (its separator plane, or the whole leaf box)
// and sees the vertices B on the frame of its subtree's box (one vertex layer
// around the box, clipped to the grid), which all belong to separators of its
// ancestors.  Eliminating the tree bottom-up (multifrontal order) gives, per
// node, the frontal matrix over I u B
//   F = [A_II A_IB; A_BI 0] + sum over the children of their update matrices,
// and
//   G = F_II^{-1},  T = F_BI G,  W = G F_IB,  U = F_BB - F_BI W  (to the parent).
// The solve is a forward pass over the tree levels (leaves first)
//   w = [r_I; 0] + children's update vectors,  y_I = G w_I,  u = w_B - T w_I,
// and a backward pass (root first)
//   x_I = y_I - W x_B,
// where x_B are the already computed values at the ancestors' vertices.  Every
// step is a batched GEMV over all nodes of one tree level, so a solve takes two
// launches per level; with the 1e5-vertex grids here that is about 13 levels
// against ~100 sequential steps of a block elimination over grid lines, and
// the factors stream about 14 times fewer bytes (2-D: O(n log n) entries
// against the dense Schur blocks of the line elimination).
//
// Storage per node: [G; -T] column-major (column i of the node's matrix holds
// rows 0..nI+nB-1, so a wavefront reads 64 consecutive rows of one column as
// one contiguous 1 KiB segment) and -W column-major over B (column b holds
// rows i).  Setup runs on the device level by level: a frontal assembly
// kernel, the batched Gauss-Jordan of the subdomain setup on F_II (no
// pivoting; its pivot and one-vector guards apply), and a batched complex GEMM
// for T, W and U.  A solve of a probe vector against the stencil matrix checks
// the factorisation once at setup.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "ctx.hpp"

namespace th {

constexpr int kNDRows = 64;      // output rows per workgroup task (one per lane)
constexpr int kNDStage = 2048;   // staged input entries per pass (RC right-hand sides x columns)
constexpr int kGemmT = 64;       // GEMM output tile edge
constexpr int kGemmK = 16;       // GEMM k-slice staged in LDS

// ---------------------------------------------------------------------------
// Solve kernels.

// Forward step of one tree level.  Task (node, row0): rows row0 .. row0 + 63 of
// the node's [G; -T] (rows < nI give y_I, written to uc at I; rows nI.. give
// the node's update vector u = w_B - T w_I).  The W wavefronts split the
// columns; their partial sums are added in wavefront order.  A level is
// short, so the loads that do not depend on the staged w (the output row's
// extend-add sources and values, and the first kNDPre columns of every
// wavefront) are issued before the staging.
constexpr int kNDPre = 4;

template <int RC, int W>
__global__ __launch_bounds__(64 * W) void k_nd_fwd(const NDNode *__restrict__ nodes,
                                                   const int2 *__restrict__ tasks,
                                                   const int *__restrict__ idx,
                                                   const int *__restrict__ src,
                                                   const c64 *__restrict__ M,
                                                   const c64 *__restrict__ rc,
                                                   c64 *__restrict__ uc, c64 *__restrict__ uvec,
                                                   long long ncn, long long ulen, int nrhs) {
  constexpr int KC = kNDStage / RC;
  __shared__ c64 ws[RC * KC];
  __shared__ c64 red[(W > 1 ? W - 1 : 1) * 64 * RC];
  const int2 tk = tasks[blockIdx.x];
  const NDNode nd = nodes[tk.x];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r = tk.y + lane, rows = nd.nI + nd.nB;
  const int q0 = blockIdx.y * RC, nq = min(RC, nrhs - q0);
  const int *I = idx + nd.ioff;
  const int *S = src + nd.soff;
  const bool live = r < rows;
  // output side: the vertex of row r (r < nI) or its two extend-add values
  long long gout = 0;
  c64 e0[RC], e1[RC];
  if (wave == 0 && live) {
    if (r < nd.nI) {
      gout = I[r];
    } else {
      const int s0 = S[2 * r], s1 = S[2 * r + 1];
#pragma unroll
      for (int q = 0; q < RC; ++q) {
        const long long qq = q0 + min(q, nq - 1);
        e0[q] = s0 >= 0 ? uvec[qq * ulen + s0] : c64{0, 0};
        e1[q] = s1 >= 0 ? uvec[qq * ulen + s1] : c64{0, 0};
      }
    }
  }
  const c64 *Mr = M + nd.moff + r;
  c64 pre[kNDPre];
#pragma unroll
  for (int u = 0; u < kNDPre; ++u) {
    const int j = wave + u * W;
    pre[u] = (live && j < min(KC, nd.nI)) ? ld_stream(Mr + (long long)j * nd.ldm) : c64{0, 0};
  }
  c64 acc[RC];
#pragma unroll
  for (int q = 0; q < RC; ++q) acc[q] = c64{0, 0};
  for (int c0 = 0; c0 < nd.nI; c0 += KC) {
    const int kc = min(KC, nd.nI - c0);
    if (c0) __syncthreads();
    // w_I = r_I + the children's update vectors, for columns c0 .. c0 + kc - 1
    for (int t = threadIdx.x; t < kc * RC; t += 64 * W) {
      const int j = t % kc, q = t / kc;
      c64 v = {0, 0};
      if (q < nq) {
        const int p = c0 + j;
        const long long qq = q0 + q;
        v = rc[qq * ncn + I[p]];
        const int s0 = S[2 * p], s1 = S[2 * p + 1];
        if (s0 >= 0) v = v + uvec[qq * ulen + s0];
        if (s1 >= 0) v = v + uvec[qq * ulen + s1];
      }
      ws[q * KC + j] = v;
    }
    __syncthreads();
    if (live) {
      int j = wave;
      if (c0 == 0) {
#pragma unroll
        for (int u = 0; u < kNDPre; ++u, j += W)
          if (j < kc) {
#pragma unroll
            for (int q = 0; q < RC; ++q) cmac(acc[q], pre[u], ws[q * KC + j]);
          }
      }
#pragma unroll 4
      for (; j < kc; j += W) {
        const c64 g = ld_stream(Mr + (long long)(c0 + j) * nd.ldm);
#pragma unroll
        for (int q = 0; q < RC; ++q) cmac(acc[q], g, ws[q * KC + j]);
      }
    }
  }
  if (W > 1) {
    if (wave > 0) {
#pragma unroll
      for (int q = 0; q < RC; ++q) red[((wave - 1) * RC + q) * 64 + lane] = acc[q];
    }
    __syncthreads();
  }
  if (wave != 0 || !live) return;
  for (int w = 1; w < W; ++w) {
#pragma unroll
    for (int q = 0; q < RC; ++q) acc[q] = acc[q] + red[((w - 1) * RC + q) * 64 + lane];
  }
  if (r < nd.nI) {
#pragma unroll
    for (int q = 0; q < RC; ++q)
      if (q < nq) uc[(q0 + q) * ncn + gout] = acc[q];
  } else {
    const int j = r - nd.nI;
#pragma unroll
    for (int q = 0; q < RC; ++q)
      if (q < nq) uvec[(q0 + q) * ulen + nd.uoff + j] = acc[q] + e0[q] + e1[q];
  }
}

// Backward step of one tree level: x_I = y_I + (-W) x_B for rows row0 ..
// row0 + 63 of I; x_B read from uc at the node's B vertices (ancestors).  The
// row's y_I and the first columns of -W are loaded before x_B is staged.
template <int RC, int W>
__global__ __launch_bounds__(64 * W) void k_nd_bwd(const NDNode *__restrict__ nodes,
                                                   const int2 *__restrict__ tasks,
                                                   const int *__restrict__ idx,
                                                   const c64 *__restrict__ Wm,
                                                   c64 *__restrict__ uc, long long ncn, int nrhs) {
  constexpr int KC = kNDStage / RC;
  __shared__ c64 ws[RC * KC];
  __shared__ c64 red[(W > 1 ? W - 1 : 1) * 64 * RC];
  const int2 tk = tasks[blockIdx.x];
  const NDNode nd = nodes[tk.x];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i = tk.y + lane;
  const bool live = i < nd.nI;
  const int q0 = blockIdx.y * RC, nq = min(RC, nrhs - q0);
  const int *I = idx + nd.ioff;
  const int *B = I + nd.nI;
  long long g = 0;
  c64 yv[RC];
  if (wave == 0 && live) {
    g = I[i];
#pragma unroll
    for (int q = 0; q < RC; ++q) yv[q] = uc[(q0 + min(q, nq - 1)) * ncn + g];
  }
  const c64 *Wr = Wm + nd.woff + i;
  c64 pre[kNDPre];
#pragma unroll
  for (int u = 0; u < kNDPre; ++u) {
    const int j = wave + u * W;
    pre[u] = (live && j < min(KC, nd.nB)) ? ld_stream(Wr + (long long)j * nd.ldw) : c64{0, 0};
  }
  c64 acc[RC];
#pragma unroll
  for (int q = 0; q < RC; ++q) acc[q] = c64{0, 0};
  for (int c0 = 0; c0 < nd.nB; c0 += KC) {
    const int kc = min(KC, nd.nB - c0);
    if (c0) __syncthreads();
    for (int t = threadIdx.x; t < kc * RC; t += 64 * W) {
      const int j = t % kc, q = t / kc;
      ws[q * KC + j] = q < nq ? uc[(q0 + q) * ncn + B[c0 + j]] : c64{0, 0};
    }
    __syncthreads();
    if (live) {
      int j = wave;
      if (c0 == 0) {
#pragma unroll
        for (int u = 0; u < kNDPre; ++u, j += W)
          if (j < kc) {
#pragma unroll
            for (int q = 0; q < RC; ++q) cmac(acc[q], pre[u], ws[q * KC + j]);
          }
      }
#pragma unroll 4
      for (; j < kc; j += W) {
        const c64 gw = ld_stream(Wr + (long long)(c0 + j) * nd.ldw);
#pragma unroll
        for (int q = 0; q < RC; ++q) cmac(acc[q], gw, ws[q * KC + j]);
      }
    }
  }
  if (W > 1) {
    if (wave > 0) {
#pragma unroll
      for (int q = 0; q < RC; ++q) red[((wave - 1) * RC + q) * 64 + lane] = acc[q];
    }
    __syncthreads();
  }
  if (wave != 0 || !live) return;
  for (int w = 1; w < W; ++w) {
#pragma unroll
    for (int q = 0; q < RC; ++q) acc[q] = acc[q] + red[((w - 1) * RC + q) * 64 + lane];
  }
#pragma unroll
  for (int q = 0; q < RC; ++q)
    if (q < nq) uc[(q0 + q) * ncn + g] = yv[q] + acc[q];
}

// ---------------------------------------------------------------------------
// Setup kernels.

// Per node of a setup batch: the children's update matrices.
struct NDAsm {
  const c64 *U[2];      // child update matrix (row-major, ld ldu), or null
  int ldu[2];
  long long cuoff[2];   // child's update-vector offset (src entries minus it index the child's B)
};

// Frontal matrix of node n0 + blockIdx.y, F over [I (padded to nIp) | B], ld ldF:
// stencil entries A(v_p, v_q) where p or q lies in I, plus the children's
// update matrices; identity on the padding of the I block, zero elsewhere.
__global__ __launch_bounds__(256) void k_nd_assemble(const NDNode *__restrict__ nodes,
                                                     const NDAsm *__restrict__ asmd, int n0,
                                                     const int *__restrict__ idx,
                                                     const int *__restrict__ src,
                                                     const c64 *__restrict__ st, int dim, int nx,
                                                     c64 *__restrict__ F, int nIp, int ldF,
                                                     long long fstride) {
  const NDNode nd = nodes[n0 + blockIdx.y];
  const NDAsm as = asmd[blockIdx.y];
  c64 *Fb = F + blockIdx.y * fstride;
  const int *I = idx + nd.ioff;
  const int S = dim == 3 ? 27 : 9;
  const long long tot = (long long)ldF * ldF;
  for (long long t = blockIdx.x * 256LL + threadIdx.x; t < tot; t += (long long)gridDim.x * 256) {
    const int p = (int)(t / ldF), q = (int)(t % ldF);
    // front positions (I first, then B), -1 on padding
    const int fp = p < nIp ? (p < nd.nI ? p : -1) : (p - nIp < nd.nB ? nd.nI + p - nIp : -1);
    const int fq = q < nIp ? (q < nd.nI ? q : -1) : (q - nIp < nd.nB ? nd.nI + q - nIp : -1);
    c64 v = {0, 0};
    if (fp < 0 || fq < 0) {
      if (p == q && p < nIp) v = c64{1.0, 0.0};
      Fb[t] = v;
      continue;
    }
    if (fp < nd.nI || fq < nd.nI) {
      const int a = I[fp], b = I[fq];  // the B list follows the I list
      const int ax = a % nx, ay = (a / nx) % nx, az = a / (nx * nx);
      const int bx = b % nx, by = (b / nx) % nx, bz = b / (nx * nx);
      const int dx = bx - ax, dy = by - ay, dz = bz - az;
      if (dx >= -1 && dx <= 1 && dy >= -1 && dy <= 1 && dz >= -1 && dz <= 1) {
        const int code = dim == 3 ? ((dz + 1) * 3 + dy + 1) * 3 + dx + 1 : (dy + 1) * 3 + dx + 1;
        v = st[(long long)S * a + code];
      }
    }
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      if (!as.U[c]) continue;
      const int sp = src[nd.soff + 2 * fp + c], sq = src[nd.soff + 2 * fq + c];
      if (sp >= 0 && sq >= 0)
        v = v + as.U[c][(long long)(sp - as.cuoff[c]) * as.ldu[c] + (sq - as.cuoff[c])];
    }
    Fb[t] = v;
  }
}

// One job of the batched GEMM C = Cin + alpha A B (or a copy C = A when k == 0),
// operands addressed through row and column strides.
struct NDGemm {
  const c64 *A, *B, *Cin;
  c64 *C;
  int m, n, k;
  long long ars, acs, brs, bcs, cirs, cics, crs, ccs;
  double alpha;
};

// 64 x 64 output tile (blockIdx.x over columns, blockIdx.y over rows) of job
// blockIdx.z; k staged through LDS in slices of 16, 4 x 4 outputs per thread.
__global__ __launch_bounds__(256) void k_nd_gemm(const NDGemm *__restrict__ jobs) {
  __shared__ c64 As[kGemmT][kGemmK + 1];
  __shared__ c64 Bs[kGemmK][kGemmT + 1];
  const NDGemm J = jobs[blockIdx.z];
  const int i0 = blockIdx.y * kGemmT, j0 = blockIdx.x * kGemmT;
  if (i0 >= J.m || j0 >= J.n) return;  // uniform
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  c64 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = c64{0, 0};
  for (int k0 = 0; k0 < J.k; k0 += kGemmK) {
    if (k0) __syncthreads();
    for (int t = threadIdx.x; t < kGemmT * kGemmK; t += 256) {
      int i, q;
      if (J.acs == 1) { i = t / kGemmK; q = t % kGemmK; } else { i = t % kGemmT; q = t / kGemmT; }
      As[i][q] = (i0 + i < J.m && k0 + q < J.k) ? J.A[(i0 + i) * J.ars + (k0 + q) * J.acs] : c64{0, 0};
    }
    for (int t = threadIdx.x; t < kGemmK * kGemmT; t += 256) {
      int q, j;
      if (J.bcs == 1) { q = t / kGemmT; j = t % kGemmT; } else { q = t % kGemmK; j = t / kGemmK; }
      Bs[q][j] = (k0 + q < J.k && j0 + j < J.n) ? J.B[(k0 + q) * J.brs + (j0 + j) * J.bcs] : c64{0, 0};
    }
    __syncthreads();
#pragma unroll 4
    for (int q = 0; q < kGemmK; ++q) {
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
    const int i = i0 + ty + 16 * a;
    if (i >= J.m) continue;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int j = j0 + tx + 16 * b;
      if (j >= J.n) continue;
      c64 v = J.alpha * acc[a][b];
      if (J.Cin) v = v + J.Cin[i * J.cirs + j * J.cics];
      J.C[i * J.crs + j * J.ccs] = v;
    }
  }
}

// C = A for job blockIdx.y (m x n, strided), grid-stride over the entries.
__global__ __launch_bounds__(256) void k_nd_copy(const NDGemm *__restrict__ jobs) {
  const NDGemm J = jobs[blockIdx.y];
  const long long tot = (long long)J.m * J.n;
  for (long long t = blockIdx.x * 256LL + threadIdx.x; t < tot; t += (long long)gridDim.x * 256) {
    const long long i = t % J.m, j = t / J.m;
    J.C[i * J.crs + j * J.ccs] = J.A[i * J.ars + j * J.acs];
  }
}

// y = b - A_c x (b may be null: y = A_c x) with the stencil, for right-hand
// side blockIdx.y: the probe check of the factorisation and the residual of
// the iterative refinement.
__global__ __launch_bounds__(256) void k_cstencil_apply(const c64 *__restrict__ st, int dim, int nx,
                                                        const c64 *__restrict__ b,
                                                        const c64 *__restrict__ x,
                                                        c64 *__restrict__ y) {
  const long long n = dim == 3 ? (long long)nx * nx * nx : (long long)nx * nx;
  const int S = dim == 3 ? 27 : 9;
  const long long off = blockIdx.y * n;
  for (long long v = blockIdx.x * 256LL + threadIdx.x; v < n; v += (long long)gridDim.x * 256) {
    const int ax = (int)(v % nx), ay = (int)((v / nx) % nx), az = (int)(v / ((long long)nx * nx));
    c64 acc = {0, 0};
    for (int t = 0; t < S; ++t) {
      const int dx = t % 3 - 1, dy = (t / 3) % 3 - 1, dz = dim == 3 ? t / 9 - 1 : 0;
      const int bx = ax + dx, by = ay + dy, bz = az + dz;
      if (bx < 0 || bx >= nx || by < 0 || by >= nx || bz < 0 || bz >= (dim == 3 ? nx : 1)) continue;
      cmac(acc, st[S * v + t], x[off + ((long long)bz * nx + by) * nx + bx]);
    }
    y[off + v] = b ? b[off + v] - acc : acc;
  }
}

// ---------------------------------------------------------------------------
// Host: the dissection tree.

namespace {

struct NDTmp {
  int box[6];          // vertex box of the node's subtree, half-open per axis
  int child[2] = {-1, -1};
  int parent = -1;
  int height = 0;
  std::vector<int> I, B;
};

int nd_split(std::vector<NDTmp> &T, const int box[6], int dim, int nx, int leafmax) {
  int ext[3], vol = 1;
  for (int a = 0; a < 3; ++a) {
    ext[a] = box[2 * a + 1] - box[2 * a];
    vol *= ext[a];
  }
  if (vol <= 0) return -1;
  NDTmp nd;
  std::memcpy(nd.box, box, sizeof nd.box);
  auto gid = [&](int x, int y, int z) { return (z * nx + y) * nx + x; };
  // frame of the box: one vertex layer around it, clipped to the grid
  {
    int lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
      const int n_a = (a < dim) ? nx : 1;
      lo[a] = std::max(box[2 * a] - 1, 0);
      hi[a] = std::min(box[2 * a + 1] + 1, n_a);
    }
    for (int z = lo[2]; z < hi[2]; ++z)
      for (int y = lo[1]; y < hi[1]; ++y)
        for (int x = lo[0]; x < hi[0]; ++x) {
          const bool in = x >= box[0] && x < box[1] && y >= box[2] && y < box[3] &&
                          z >= box[4] && z < box[5];
          if (!in) nd.B.push_back(gid(x, y, z));
        }
  }
  if (vol <= leafmax) {
    for (int z = box[4]; z < box[5]; ++z)
      for (int y = box[2]; y < box[3]; ++y)
        for (int x = box[0]; x < box[1]; ++x) nd.I.push_back(gid(x, y, z));
    T.push_back(std::move(nd));
    return (int)T.size() - 1;
  }
  int ax = 0;
  for (int a = 1; a < dim; ++a)
    if (ext[a] >= ext[ax]) ax = a;  // longest axis, the slowest on ties
  const int m = (box[2 * ax] + box[2 * ax + 1]) / 2;
  int b0[6], b1[6];
  std::memcpy(b0, box, sizeof b0);
  std::memcpy(b1, box, sizeof b1);
  b0[2 * ax + 1] = m;
  b1[2 * ax] = m + 1;
  const int c0 = nd_split(T, b0, dim, nx, leafmax);
  const int c1 = nd_split(T, b1, dim, nx, leafmax);
  int sb[6];
  std::memcpy(sb, box, sizeof sb);
  sb[2 * ax] = m;
  sb[2 * ax + 1] = m + 1;
  for (int z = sb[4]; z < sb[5]; ++z)
    for (int y = sb[2]; y < sb[3]; ++y)
      for (int x = sb[0]; x < sb[1]; ++x) nd.I.push_back(gid(x, y, z));
  int h = 0, k = 0;
  for (int c : {c0, c1}) {
    if (c >= 0) h = std::max(h, T[c].height + 1);
    nd.child[k++] = c;
  }
  nd.height = h;
  T.push_back(std::move(nd));
  const int id = (int)T.size() - 1;
  for (int c : {c0, c1})
    if (c >= 0) T[c].parent = id;
  return id;
}

// device buffers released at the end of the setup whatever happens
struct DevScratch {
  std::vector<void *> p;
  ~DevScratch() {
    for (void *q : p)
      if (q) (void)hipFree(q);
  }
  template <typename T>
  bool get(T **out, size_t bytes) {
    void *q = nullptr;
    if (hipMalloc(&q, bytes) != hipSuccess) return false;
    p.push_back(q);
    *out = (T *)q;
    return true;
  }
  void release(void *q) {
    for (void *&r : p)
      if (r == q) {
        (void)hipFree(r);
        r = nullptr;
      }
  }
};

}  // namespace

void free_nd(NDData &nd) {
  void *ptrs[] = {nd.d_nodes, nd.d_idx, nd.d_src, nd.d_ftask, nd.d_btask, nd.M, nd.Wm, nd.uvec,
                  nd.st, nd.t, nd.d};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  nd = NDData{};
}

// Leaf size: the largest box volume left undivided.  Smaller leaves mean
// fewer bytes but one more tree level (two launches) per halving.
static int nd_leafmax(int dim) { return dim == 3 ? 64 : 64; }

int setup_coarse_nd(th_ctx *c, const std::vector<c64> &stencil) {
  hipStream_t s = c->stream;
  CoarseData &cd = c->coarse;
  NDData &nd = cd.nd;
  const int dim = c->dim, nx = c->nc1;
  const long long ncn = dim == 3 ? (long long)nx * nx * nx : (long long)nx * nx;
  if (ncn > (1LL << 31) - 1) {
    set_error("coarse grid too large for 32-bit vertex indices");
    return TH_EINVAL;
  }
  // tree
  std::vector<NDTmp> T;
  {
    const int box[6] = {0, nx, 0, nx, 0, dim == 3 ? nx : 1};
    if (nd_split(T, box, dim, nx, nd_leafmax(dim)) < 0) {
      set_error("empty coarse grid");
      return TH_EINVAL;
    }
  }
  const int nn = (int)T.size();
  int H = 0;
  for (const NDTmp &t : T) H = std::max(H, t.height + 1);
  // level order: by height, then creation order (post-order)
  std::vector<int> order(nn), pos(nn);
  for (int i = 0; i < nn; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return T[a].height < T[b].height; });
  for (int i = 0; i < nn; ++i) pos[order[i]] = i;
  nd.levels = H;
  nd.lv.assign(H, NDLevel{});
  for (int i = 0; i < nn; ++i) {
    const int h = T[order[i]].height;
    if (nd.lv[h].n1 == 0) nd.lv[h].n0 = i;
    nd.lv[h].n1 = i + 1;
  }
  // descriptors, index lists, update-vector offsets
  std::vector<NDNode> hn(nn);
  long long ioff = 0, soff = 0, moff = 0, woff = 0, uoff = 0;
  for (int i = 0; i < nn; ++i) {
    const NDTmp &t = T[order[i]];
    NDNode &d = hn[i];
    d.nI = (int)t.I.size();
    d.nB = (int)t.B.size();
    d.ldm = ceil_div(d.nI + d.nB, 8) * 8;
    d.ldw = ceil_div(d.nI, 8) * 8;
    d.ioff = ioff;
    d.soff = soff;
    d.moff = moff;
    d.woff = woff;
    d.uoff = uoff;
    ioff += d.nI + d.nB;
    soff += 2LL * (d.nI + d.nB);
    moff += (long long)d.nI * d.ldm;
    woff += (long long)d.nB * d.ldw;
    uoff += d.nB;
  }
  std::vector<int> hidx(ioff), hsrc(soff, -1);
  for (int i = 0; i < nn; ++i) {
    const NDTmp &t = T[order[i]];
    std::copy(t.I.begin(), t.I.end(), hidx.begin() + hn[i].ioff);
    std::copy(t.B.begin(), t.B.end(), hidx.begin() + hn[i].ioff + hn[i].nI);
  }
  // extend-add maps: every vertex of a child's B sits in the parent's I or B
  for (int i = 0; i < nn; ++i) {
    const NDTmp &t = T[order[i]];
    for (int k = 0; k < 2; ++k) {
      if (t.child[k] < 0) continue;
      const int ci = pos[t.child[k]];
      const NDTmp &ch = T[t.child[k]];
      for (int a = 0; a < (int)ch.B.size(); ++a) {
        const int v = ch.B[a];
        int fp;
        auto it = std::lower_bound(t.I.begin(), t.I.end(), v);
        if (it != t.I.end() && *it == v) {
          fp = (int)(it - t.I.begin());
        } else {
          auto jt = std::lower_bound(t.B.begin(), t.B.end(), v);
          if (jt == t.B.end() || *jt != v) {
            set_error("nested dissection: a child frame vertex is missing from its parent's front");
            return TH_EINVAL;
          }
          fp = hn[i].nI + (int)(jt - t.B.begin());
        }
        hsrc[hn[i].soff + 2 * fp + k] = (int)(hn[ci].uoff + a);
      }
    }
  }
  if (uoff > (1LL << 31) - 1) {
    set_error("coarse update vectors too large for 32-bit offsets");
    return TH_EINVAL;
  }
  // tasks per level
  std::vector<int2> ft, bt;
  for (int h = 0; h < H; ++h) {
    NDLevel &L = nd.lv[h];
    L.f0 = (int)ft.size();
    L.b0 = (int)bt.size();
    for (int i = L.n0; i < L.n1; ++i) {
      for (int r = 0; r < hn[i].nI + hn[i].nB; r += kNDRows) ft.push_back(make_int2(i, r));
      if (hn[i].nB > 0)
        for (int r = 0; r < hn[i].nI; r += kNDRows) bt.push_back(make_int2(i, r));
      L.maxI = std::max(L.maxI, hn[i].nI);
      L.maxB = std::max(L.maxB, hn[i].nB);
      L.fbytes += (long long)hn[i].nI * (hn[i].nI + hn[i].nB) * (long long)sizeof(c64);
      L.bbytes += (long long)hn[i].nI * hn[i].nB * (long long)sizeof(c64);
    }
    L.f1 = (int)ft.size();
    L.b1 = (int)bt.size();
  }
  const int R = c->desc.max_rhs;
  nd.ulen = std::max<long long>(uoff, 1);
  nd.nodes = nn;
  if (hipMalloc(&nd.d_nodes, nn * sizeof(NDNode)) != hipSuccess ||
      hipMalloc(&nd.d_idx, hidx.size() * sizeof(int)) != hipSuccess ||
      hipMalloc(&nd.d_src, hsrc.size() * sizeof(int)) != hipSuccess ||
      hipMalloc(&nd.d_ftask, std::max<size_t>(ft.size(), 1) * sizeof(int2)) != hipSuccess ||
      hipMalloc(&nd.d_btask, std::max<size_t>(bt.size(), 1) * sizeof(int2)) != hipSuccess ||
      hipMalloc(&nd.M, std::max<long long>(moff, 1) * sizeof(c64)) != hipSuccess ||
      hipMalloc(&nd.Wm, std::max<long long>(woff, 1) * sizeof(c64)) != hipSuccess ||
      hipMalloc(&nd.uvec, (size_t)R * nd.ulen * sizeof(c64)) != hipSuccess ||
      hipMalloc(&nd.st, stencil.size() * sizeof(c64)) != hipSuccess ||
      hipMalloc(&nd.t, (size_t)R * ncn * sizeof(c64)) != hipSuccess ||
      hipMalloc(&nd.d, (size_t)R * ncn * sizeof(c64)) != hipSuccess) {
    free_nd(nd);
    set_error("cannot allocate the nested-dissection factors");
    return TH_ENOMEM;
  }
  nd.bytes = (moff + woff + (long long)stencil.size()) * (long long)sizeof(c64);
  nd.fwd_bytes = moff * (long long)sizeof(c64);
  nd.bwd_bytes = woff * (long long)sizeof(c64);
  TH_HIP_CHECK_RET(hipMemcpyAsync(nd.st, stencil.data(), stencil.size() * sizeof(c64), hipMemcpyHostToDevice, s));
  TH_HIP_CHECK_RET(hipMemcpyAsync(nd.d_nodes, hn.data(), nn * sizeof(NDNode), hipMemcpyHostToDevice, s));
  TH_HIP_CHECK_RET(hipMemcpyAsync(nd.d_idx, hidx.data(), hidx.size() * sizeof(int), hipMemcpyHostToDevice, s));
  TH_HIP_CHECK_RET(hipMemcpyAsync(nd.d_src, hsrc.data(), hsrc.size() * sizeof(int), hipMemcpyHostToDevice, s));
  if (!ft.empty())
    TH_HIP_CHECK_RET(hipMemcpyAsync(nd.d_ftask, ft.data(), ft.size() * sizeof(int2), hipMemcpyHostToDevice, s));
  if (!bt.empty())
    TH_HIP_CHECK_RET(hipMemcpyAsync(nd.d_btask, bt.data(), bt.size() * sizeof(int2), hipMemcpyHostToDevice, s));

  // ---- factorisation, level by level
  DevScratch scr;
  const c64 *dst = nd.st;
  // frontal matrices of a batch of nodes, at most this many bytes at once
  const size_t fbudget = (size_t)8 << 30;
  std::vector<int> nIp(H), ldF(H), batch(H);
  size_t fmax = 0;
  int gj_nmax = 0, bmax = 1;
  for (int h = 0; h < H; ++h) {
    nIp[h] = ceil_div(std::max(nd.lv[h].maxI, 1), kGJBlock) * kGJBlock;
    ldF[h] = nIp[h] + nd.lv[h].maxB;
    const size_t fb = (size_t)ldF[h] * ldF[h] * sizeof(c64);
    const int m = nd.lv[h].n1 - nd.lv[h].n0;
    batch[h] = (int)std::max<size_t>(1, std::min<size_t>(m, fbudget / fb));
    fmax = std::max(fmax, fb * batch[h]);
    gj_nmax = std::max(gj_nmax, nIp[h]);
    bmax = std::max(bmax, batch[h]);
  }
  c64 *F = nullptr, *gws = nullptr;
  NDAsm *d_asm = nullptr;
  NDGemm *d_jobs = nullptr;
  if (!scr.get(&F, fmax) || !scr.get(&gws, gj_ws_bytes(bmax, gj_nmax)) ||
      !scr.get(&d_asm, bmax * sizeof(NDAsm)) || !scr.get(&d_jobs, 3 * bmax * sizeof(NDGemm))) {
    free_nd(nd);
    set_error("cannot allocate the nested-dissection setup workspace");
    return TH_ENOMEM;
  }
  if (int e = gj_ws_reset(gws, s)) {
    free_nd(nd);
    return e;
  }
  // update matrices of every level (row-major, ld = the level's largest nB),
  // released once the levels of all their parents are assembled
  std::vector<c64 *> pool(H, nullptr);
  std::vector<int> ldu(H, 1), free_after(H, -1);
  for (int i = 0; i < nn; ++i) {
    const NDTmp &t = T[order[i]];
    if (t.parent >= 0) free_after[t.height] = std::max(free_after[t.height], T[t.parent].height);
  }
  auto fail_nd = [&](int e) {
    free_nd(nd);
    return e;
  };
  for (int h = 0; h < H; ++h) {
    const NDLevel &L = nd.lv[h];
    const int m = L.n1 - L.n0;
    if (L.maxB > 0) {
      ldu[h] = L.maxB;
      if (!scr.get(&pool[h], (size_t)m * ldu[h] * ldu[h] * sizeof(c64))) {
        set_error("cannot allocate the nested-dissection update matrices");
        return fail_nd(TH_ENOMEM);
      }
    }
    const long long fs = (long long)ldF[h] * ldF[h];
    for (int b0 = 0; b0 < m; b0 += batch[h]) {
      const int nb = std::min(batch[h], m - b0);
      std::vector<NDAsm> ha(nb);
      std::vector<NDGemm> j1, j2, jc;
      for (int u = 0; u < nb; ++u) {
        const int i = L.n0 + b0 + u;
        const NDTmp &t = T[order[i]];
        for (int k = 0; k < 2; ++k) {
          ha[u].U[k] = nullptr;
          ha[u].ldu[k] = 1;
          ha[u].cuoff[k] = 0;
          if (t.child[k] < 0 || T[t.child[k]].B.empty()) continue;
          const int ci = pos[t.child[k]], ch = T[t.child[k]].height;
          ha[u].U[k] = pool[ch] + (long long)(ci - nd.lv[ch].n0) * ldu[ch] * ldu[ch];
          ha[u].ldu[k] = ldu[ch];
          ha[u].cuoff[k] = hn[ci].uoff;
        }
        const NDNode &d = hn[i];
        c64 *Fb = F + (long long)u * fs;
        const long long lf = ldF[h], ip = nIp[h];
        if (d.nB > 0) {
          NDGemm g{};
          // -T = -(F_BI G): C[b][i] at moff + i ldm + nI + b
          g.A = Fb + ip * lf; g.ars = lf; g.acs = 1;
          g.B = Fb; g.brs = lf; g.bcs = 1;
          g.C = nd.M + d.moff + d.nI; g.crs = 1; g.ccs = d.ldm;
          g.m = d.nB; g.n = d.nI; g.k = d.nI; g.alpha = -1.0;
          j1.push_back(g);
          // -W = -(G F_IB): C[i][b] at woff + b ldw + i
          g = NDGemm{};
          g.A = Fb; g.ars = lf; g.acs = 1;
          g.B = Fb + ip; g.brs = lf; g.bcs = 1;
          g.C = nd.Wm + d.woff; g.crs = 1; g.ccs = d.ldw;
          g.m = d.nI; g.n = d.nB; g.k = d.nI; g.alpha = -1.0;
          j1.push_back(g);
          // U = F_BB + F_BI (-W) into the level's pool
          g = NDGemm{};
          g.A = Fb + ip * lf; g.ars = lf; g.acs = 1;
          g.B = nd.Wm + d.woff; g.brs = 1; g.bcs = d.ldw;
          g.Cin = Fb + ip * lf + ip; g.cirs = lf; g.cics = 1;
          g.C = pool[h] + (long long)(b0 + u) * ldu[h] * ldu[h]; g.crs = ldu[h]; g.ccs = 1;
          g.m = d.nB; g.n = d.nB; g.k = d.nI; g.alpha = 1.0;
          j2.push_back(g);
        }
        NDGemm g{};
        // G into rows 0 .. nI - 1 of the node's column-major [G; -T]
        g.A = Fb; g.ars = lf; g.acs = 1;
        g.C = nd.M + d.moff; g.crs = 1; g.ccs = d.ldm;
        g.m = d.nI; g.n = d.nI; g.k = 0;
        jc.push_back(g);
      }
      TH_HIP_CHECK_RET(hipMemcpyAsync(d_asm, ha.data(), nb * sizeof(NDAsm), hipMemcpyHostToDevice, s));
      const long long tot = fs;
      const unsigned gx = (unsigned)std::min<long long>(ceil_div_ll(tot, 256), 4096);
      hipLaunchKernelGGL(k_nd_assemble, dim3(gx, nb), dim3(256), 0, s, (const NDNode *)nd.d_nodes,
                         (const NDAsm *)d_asm, L.n0 + b0, (const int *)nd.d_idx,
                         (const int *)nd.d_src, (const c64 *)dst, dim, nx, F, nIp[h], ldF[h], fs);
      TH_HIP_CHECK_RET(hipGetLastError());
      if (int e = gj_invert_batched(F, nIp[h], ldF[h], fs, nb, s, gws)) return fail_nd(e);
      auto run_gemm = [&](const std::vector<NDGemm> &jobs) -> int {
        if (jobs.empty()) return 0;
        int mm = 0, nnn = 0;
        for (const NDGemm &g : jobs) {
          mm = std::max(mm, g.m);
          nnn = std::max(nnn, g.n);
        }
        TH_HIP_CHECK_RET(hipMemcpyAsync(d_jobs, jobs.data(), jobs.size() * sizeof(NDGemm),
                                        hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_nd_gemm, dim3(ceil_div(nnn, kGemmT), ceil_div(mm, kGemmT), (unsigned)jobs.size()),
                           dim3(256), 0, s, (const NDGemm *)d_jobs);
        TH_HIP_CHECK_RET(hipGetLastError());
        // the job list is reused by the next launch: wait for this one to read it
        TH_HIP_CHECK_RET(hipStreamSynchronize(s));
        return 0;
      };
      if (int e = run_gemm(j1)) return fail_nd(e);
      if (int e = run_gemm(j2)) return fail_nd(e);
      {
        TH_HIP_CHECK_RET(hipMemcpyAsync(d_jobs, jc.data(), jc.size() * sizeof(NDGemm), hipMemcpyHostToDevice, s));
        const unsigned cx = (unsigned)std::min<long long>(ceil_div_ll((long long)L.maxI * L.maxI, 256), 4096);
        hipLaunchKernelGGL(k_nd_copy, dim3(cx, (unsigned)jc.size()), dim3(256), 0, s, (const NDGemm *)d_jobs);
        TH_HIP_CHECK_RET(hipGetLastError());
        TH_HIP_CHECK_RET(hipStreamSynchronize(s));
      }
    }
    // children's update matrices no longer needed
    for (int g = 0; g < h; ++g)
      if (pool[g] && free_after[g] <= h) {
        scr.release(pool[g]);
        pool[g] = nullptr;
      }
  }
  if (int e = gj_ws_status(gws, s, "the nested-dissection coarse factorisation")) return fail_nd(e);

  cd.kind = 1;
  cd.bytes = nd.bytes;
  return 0;
}

// Probe check of the coarse factorisation in use: x = A_c^{-1} (A_c xp) for a
// vector xp of unit-modulus entries; *err = max_v |x_v - xp_v|.
int coarse_probe_check(th_ctx *c, const std::vector<c64> &stencil, double *err) {
  hipStream_t s = c->stream;
  const int dim = c->dim, nx = c->nc1;
  const long long ncn = c->nc;
  std::vector<c64> hx(ncn);
  unsigned long long z = 0x9e3779b97f4a7c15ULL;
  for (long long v = 0; v < ncn; ++v) {  // xorshift64* phases
    z ^= z >> 12;
    z ^= z << 25;
    z ^= z >> 27;
    const unsigned long long w = z * 0x2545f4914f6cdd1dULL;
    const double a = 6.283185307179586 * (double)(w >> 11) * (1.0 / 9007199254740992.0);
    hx[v] = c64{std::cos(a), std::sin(a)};
  }
  DevScratch scr;
  c64 *dst = nullptr, *xp = nullptr, *bp = nullptr, *xs = nullptr;
  if (!scr.get(&dst, stencil.size() * sizeof(c64)) || !scr.get(&xp, ncn * sizeof(c64)) ||
      !scr.get(&bp, ncn * sizeof(c64)) || !scr.get(&xs, ncn * sizeof(c64))) {
    set_error("cannot allocate the coarse probe vectors");
    return TH_ENOMEM;
  }
  TH_HIP_CHECK_RET(hipMemcpyAsync(dst, stencil.data(), stencil.size() * sizeof(c64), hipMemcpyHostToDevice, s));
  TH_HIP_CHECK_RET(hipMemcpyAsync(xp, hx.data(), ncn * sizeof(c64), hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_cstencil_apply, dim3((unsigned)std::min<long long>(ceil_div_ll(ncn, 256), 4096)),
                     dim3(256), 0, s, (const c64 *)dst, dim, nx, (const c64 *)nullptr,
                     (const c64 *)xp, bp);
  TH_HIP_CHECK_RET(hipGetLastError());
  if (int e = launch_coarse_solve(c, bp, xs, 1, s, kCoarseExact)) return e;
  std::vector<c64> hs(ncn);
  TH_HIP_CHECK_RET(hipMemcpyAsync(hs.data(), xs, ncn * sizeof(c64), hipMemcpyDeviceToHost, s));
  TH_HIP_CHECK_RET(hipStreamSynchronize(s));
  double e = 0.0;
  for (long long v = 0; v < ncn; ++v) {
    const double dr = hs[v].re - hx[v].re, di = hs[v].im - hx[v].im;
    const double ev = std::sqrt(dr * dr + di * di);
    if (!(ev <= e)) e = ev;  // NaN propagates
  }
  *err = e;
  return 0;
}

// Modelled time of one coarse solve for max_rhs right-hand sides: every level
// streams its factor bytes once per pass of RC right-hand sides at 6.5 TB/s
// and takes at least 7 us (its launch and a few dependent memory round trips,
// measured on the C2 tree); refinement steps (FP64 operators only: the
// complex64 preconditioner skips them) add a solve and two short launches.
double coarse_model_nd(const th_ctx *c) {
  const NDData &nd = c->coarse.nd;
  const int R = c->desc.max_rhs;
  const int RC = R >= 8 ? 8 : (R >= 4 ? 4 : (R >= 2 ? 2 : 1));
  const double passes = (double)ceil_div(R, RC);
  double t = 0.0;
  for (const NDLevel &L : nd.lv) {
    t += std::max(7e-6, (double)L.fbytes * passes / 6.5e12);
    if (L.bbytes > 0) t += std::max(7e-6, (double)L.bbytes * passes / 6.5e12);
  }
  const int refine = c->desc.gemm == TH_GEMM_F64 ? nd.refine_pc : 0;
  return t * (1 + refine) + refine * 17e-6;
}

// Wavefronts per workgroup of a level: 4 where the level has enough tasks to
// fill the chip, more (16 for one or two right-hand sides per pass, 8 beyond)
// where few long nodes near the root would leave each wavefront a long
// sequential column loop.
constexpr int kNDFewTasks = 256;

template <int RC, int W>
static void nd_fwd_level(const th_ctx *c, const NDLevel &L, const c64 *rcv, c64 *uc, c64 *uvec,
                         int nrhs, hipStream_t s) {
  const NDData &nd = c->coarse.nd;
  hipLaunchKernelGGL((k_nd_fwd<RC, W>), dim3(L.f1 - L.f0, (unsigned)ceil_div(nrhs, RC)), dim3(64 * W),
                     0, s, (const NDNode *)nd.d_nodes, (const int2 *)nd.d_ftask + L.f0,
                     (const int *)nd.d_idx, (const int *)nd.d_src, (const c64 *)nd.M, rcv, uc,
                     uvec, c->nc, nd.ulen, nrhs);
}

template <int RC, int W>
static void nd_bwd_level(const th_ctx *c, const NDLevel &L, c64 *uc, int nrhs, hipStream_t s) {
  const NDData &nd = c->coarse.nd;
  hipLaunchKernelGGL((k_nd_bwd<RC, W>), dim3(L.b1 - L.b0, (unsigned)ceil_div(nrhs, RC)), dim3(64 * W),
                     0, s, (const NDNode *)nd.d_nodes, (const int2 *)nd.d_btask + L.b0,
                     (const int *)nd.d_idx, (const c64 *)nd.Wm, uc, c->nc, nrhs);
}

template <int RC>
static void nd_solve_t(const th_ctx *c, const c64 *rcv, c64 *uc, c64 *uvec, int nrhs,
                       hipStream_t s) {
  constexpr int WB = RC <= 2 ? 16 : 8;
  const NDData &nd = c->coarse.nd;
  const int gy = ceil_div(nrhs, RC);
  for (int h = 0; h < nd.levels; ++h) {
    const NDLevel &L = nd.lv[h];
    if (L.f1 <= L.f0) continue;
    if ((long long)(L.f1 - L.f0) * gy < kNDFewTasks)
      nd_fwd_level<RC, WB>(c, L, rcv, uc, uvec, nrhs, s);
    else
      nd_fwd_level<RC, 4>(c, L, rcv, uc, uvec, nrhs, s);
  }
  for (int h = nd.levels - 1; h >= 0; --h) {
    const NDLevel &L = nd.lv[h];
    if (L.b1 <= L.b0) continue;
    if ((long long)(L.b1 - L.b0) * gy < kNDFewTasks)
      nd_bwd_level<RC, WB>(c, L, uc, nrhs, s);
    else
      nd_bwd_level<RC, 4>(c, L, uc, nrhs, s);
  }
}

static void nd_solve(const th_ctx *c, const c64 *rcv, c64 *uc, c64 *uvec, int nrhs, hipStream_t s) {
  if (nrhs >= 8)
    nd_solve_t<8>(c, rcv, uc, uvec, nrhs, s);
  else if (nrhs >= 4)
    nd_solve_t<4>(c, rcv, uc, uvec, nrhs, s);
  else if (nrhs >= 2)
    nd_solve_t<2>(c, rcv, uc, uvec, nrhs, s);
  else
    nd_solve_t<1>(c, rcv, uc, uvec, nrhs, s);
}

// uc = A_c^{-1} rc: one solve with the factors, then `refine` steps of
// iterative refinement against the stencil matrix (FP64 residuals).  The
// separator blocks of interior boxes are real indefinite Helmholtz blocks that
// can be close to singular, which costs digits in the factors; refinement
// brings the solve back to the rounding level of the residual (exact
// accuracy), or to a probe error of 1e-8 inside the FP64 preconditioner.  For
// a result rounded to complex64 afterwards no refinement is done: the factors
// alone are far more accurate than that rounding.
int launch_coarse_nd(const th_ctx *c, const c64 *rcv, c64 *uc, int nrhs, hipStream_t s,
                     int accuracy, const CoarseScratch *ws) {
  const NDData &nd = c->coarse.nd;
  c64 *uvec = ws && ws->uvec ? ws->uvec : nd.uvec;
  c64 *t = ws && ws->t ? ws->t : nd.t;
  c64 *d = ws && ws->d ? ws->d : nd.d;
  nd_solve(c, rcv, uc, uvec, nrhs, s);
  const long long ncn = c->nc;
  const unsigned gx = (unsigned)std::min<long long>(ceil_div_ll(ncn, 256), 4096);
  const int steps = accuracy == kCoarseExact    ? nd.refine
                    : accuracy == kCoarsePrecond ? nd.refine_pc
                                                 : 0;
  for (int it = 0; it < steps; ++it) {
    hipLaunchKernelGGL(k_cstencil_apply, dim3(gx, nrhs), dim3(256), 0, s, (const c64 *)nd.st,
                       c->dim, c->nc1, rcv, (const c64 *)uc, t);
    nd_solve(c, t, d, uvec, nrhs, s);
    if (int e = launch_add(uc, d, (long long)nrhs * ncn, false, s)) return e;
  }
  TH_HIP_CHECK_RET(hipGetLastError());
  return 0;
}

}  // namespace th
