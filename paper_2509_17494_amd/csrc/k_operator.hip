// Matrix-free fine operator: out = f + sgn * (A u) for the Q_p Galerkin matrix
// of a(u, v) = int grad u . grad v - int kappa u v - int_{Gamma_abs} i k u v
// (eq. bilin_form; kappa = k^2 + i eps, or the shifted coefficient of A_s,
// Sec. 4.1) on the N x N (2-D) or N x N x N (3-D) mesh.
//
// Per cell of size h the operator is  K1 (x) M1 + M1 (x) K1 - kappa_c h^2 M1 (x) M1
// (1-D reference matrices on [0,1]; the 2-D stiffness does not scale with h),
// plus -i k_c h M1 on cell edges lying on an absorbing side.  It is applied by
// sum factorisation in two passes through LDS:
//   x pass: for every node row of the tile and every cell column, the x
//           contractions W = u M1^T and Z = u K1^T restricted to that cell;
//   y pass: every owned node sums, over the (at most 4) cells containing it,
//           K1 W + M1 (Z - kappa h^2 W) along y -- a fixed-order gather, so the
//           result is deterministic (no atomics).
// A workgroup owns the nodes of a TC x TC cell tile (low edges included) and
// reads one extra cell layer on the low sides; TC is picked per launch so
// that small meshes with few right-hand sides still give the chip enough
// workgroups.
//
// Dirichlet sides (op.dir): their nodes are eliminated with unit rows and
// columns, so u is read as zero there and the row of such a node is u itself.
#include "ctx.hpp"

namespace th {

// Shape of a 2-D tile of TC x TC cells: node rows and cell columns staged by
// the x pass; the y pass gives each local node row ay in [0, P) of the owned
// cells its own whole wavefronts (CW threads, one per cell), so ay is uniform
// per wavefront; threads and x-pass items per thread.
template <int P, int TC>
struct Tile2 {
  static constexpr int NP = P + 1;
  static constexpr int NROW = (TC + 1) * P + 1;
  static constexpr int NCC = TC + 1;
  static constexpr int CW = (TC * TC + 63) / 64 * 64;
  static constexpr int NT = P * CW;
  static constexpr int XI = (NROW * NCC + NT - 1) / NT;
};

// Robin term of node (ix, iy) on an absorbing side: -i k h (M1 along the side) u.
template <int P, typename T>
__device__ __forceinline__ void robin_add(const FineOp &op, const Ref1D &ref,
                                          const cx<T> *__restrict__ u, int ix, int iy,
                                          cx<T> &acc) {
  constexpr int NP = P + 1;
  const int N = op.N, n1 = op.n1, NPn = N * P;
  const int chx = min(ix / P, N - 1), chy = min(iy / P, N - 1);
  const int ncellx = (ix % P == 0 && ix > 0 && ix < NPn) ? 2 : 1;
  const int ncelly = (iy % P == 0 && iy > 0 && iy < NPn) ? 2 : 1;
  cx<T> s = {0, 0};
  if ((ix == 0 && (op.robin & 1)) || (ix == NPn && (op.robin & 2))) {
    const int cxq = (ix == 0) ? 0 : N - 1;
    for (int qy = ncelly - 1; qy >= 0; --qy) {
      const int cyq = chy - qy, ay = iy - cyq * P;
      const T kk = (T)op.kr[(long long)cyq * N + cxq];
      cx<T> m = {0, 0};
      for (int by = 0; by < NP; ++by)
        if (!on_dir(op.dir, 1, cyq * P + by, NPn))
          rmac(m, (T)ref.M[ay * NP + by], u[(long long)(cyq * P + by) * n1 + ix]);
      rmac(s, kk, m);
    }
  }
  if ((iy == 0 && (op.robin & 4)) || (iy == NPn && (op.robin & 8))) {
    const int cyq = (iy == 0) ? 0 : N - 1;
    for (int qx = ncellx - 1; qx >= 0; --qx) {
      const int cxq = chx - qx, ax = ix - cxq * P;
      const T kk = (T)op.kr[(long long)cyq * N + cxq];
      cx<T> m = {0, 0};
      for (int bx = 0; bx < NP; ++bx)
        if (!on_dir(op.dir, 0, cxq * P + bx, NPn))
          rmac(m, (T)ref.M[ax * NP + bx], u[(long long)iy * n1 + cxq * P + bx]);
      rmac(s, kk, m);
    }
  }
  // -i h s = (h s.im, -h s.re)
  const T h = (T)op.h;
  acc.re += h * s.im;
  acc.im -= h * s.re;
}

// x pass: one item per (staged node row, staged cell column), its u row
// segment loaded by every thread at once before any compute; y pass: thread
// (ay, cell) sums the nodes of the cell's local row ay on its low edges (and
// on its high edges at the domain's last node column; the ay = 0 wavefronts
// also take the last node row) over the cells that contain them --
// below-left, below, left, own, a fixed order that keeps the result
// deterministic.  ax is unrolled and ay uniform per wavefront, so the LDS
// offsets are per-lane bases plus constants and the K1 / M1 entries scalars.
template <int P, int TC, typename T>
__global__ __launch_bounds__((Tile2<P, TC>::NT)) void k_apply2d(FineOp op, Ref1D ref,
                                                               const cx<T> *__restrict__ u,
                                                               const cx<T> *__restrict__ f,
                                                               cx<T> *__restrict__ out, T sgn) {
  using S = Tile2<P, TC>;
  constexpr int NP = P + 1, NCC = S::NCC, NT = S::NT;
  __shared__ cx<T> WX[S::NROW * NCC * NP];
  __shared__ cx<T> ZX[S::NROW * NCC * NP];
  __shared__ cx<T> KH[NCC * NCC];

  const int N = op.N, n1 = op.n1, NPn = N * P;
  const long long rb = (long long)blockIdx.z * op.nf;
  u += rb;
  out += rb;
  if (f) f += rb;

  const int cx0 = blockIdx.x * TC, cy0 = blockIdx.y * TC;
  const int cxs = max(cx0 - 1, 0), cxe = min(cx0 + TC, N);
  const int cys = max(cy0 - 1, 0), cye = min(cy0 + TC, N);
  const int ncx = cxe - cxs, ncy = cye - cys;
  const int nrow = ncy * P + 1;
  const T h2 = (T)(op.h * op.h);

  cx<T> uv[S::XI][NP];
#pragma unroll
  for (int k = 0; k < S::XI; ++k) {
    const int it = threadIdx.x + k * NT;
    const int jr = min(it / NCC, nrow - 1), cc = min(it % NCC, ncx - 1);
    const cx<T> *urow = u + (long long)(cys * P + jr) * n1 + (cxs + cc) * P;
#pragma unroll
    for (int b = 0; b < NP; ++b) uv[k][b] = urow[b];
  }
  // the y pass's cell and node row, and its f values, loaded with the rest
  const int ay0 = __builtin_amdgcn_readfirstlane((int)threadIdx.x / S::CW);
  const int ci = threadIdx.x % S::CW;
  const int cxo = cx0 + ci % TC, cyo = cy0 + ci / TC;
  const bool owner = ci < TC * TC && cxo < N && cyo < N;
  const bool lastx = cxo == N - 1, lasty = cyo == N - 1;
  cx<T> fv[2][NP];
  {
    const int gx = min(cxo, N - 1) * P, gy = min(cyo, N - 1) * P;
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int ax = 0; ax < NP; ++ax) {
        fv[r][ax] = cx<T>{0, 0};
        const bool need = (r == 0 || (ay0 == 0 && lasty)) && (ax < P || lastx);
        if (f && need) fv[r][ax] = f[(long long)(gy + (r ? P : ay0)) * n1 + gx + ax];
      }
  }
  for (int i = threadIdx.x; i < ncx * ncy; i += NT) {
    const int ly = i / ncx, lx = i - ly * ncx;
    const c64 kd = op.kap[(long long)(cys + ly) * N + cxs + lx];
    KH[ly * NCC + lx] = cx<T>{(T)kd.re * h2, (T)kd.im * h2};
  }

  // x pass
#pragma unroll
  for (int k = 0; k < S::XI; ++k) {
    const int it = threadIdx.x + k * NT;
    const int jr = it / NCC, cc = it % NCC;
    if (jr >= nrow || cc >= ncx) continue;
    if (op.dir) {
      const int jy = cys * P + jr, c = cxs + cc;
      const bool rowd = on_dir(op.dir, 1, jy, NPn);
#pragma unroll
      for (int b = 0; b < NP; ++b)
        if (rowd || on_dir(op.dir, 0, c * P + b, NPn)) uv[k][b] = cx<T>{0, 0};
    }
#pragma unroll
    for (int a = 0; a < NP; ++a) {
      cx<T> w = {0, 0}, z = {0, 0};
#pragma unroll
      for (int b = 0; b < NP; ++b) {
        rmac(w, (T)ref.M[a * NP + b], uv[k][b]);
        rmac(z, (T)ref.K[a * NP + b], uv[k][b]);
      }
      WX[(jr * NCC + cc) * NP + a] = w;
      ZX[(jr * NCC + cc) * NP + a] = z;
    }
  }
  __syncthreads();

  // y pass
  if (!owner) return;
  const int cc = cxo - cxs, cr = cyo - cys;
  const bool left = cxo > 0, below = cyo > 0;
  // one cell's contribution to local node (lx, ly) of that cell
  auto cell = [&](int c, int r, int lx, int ly, cx<T> &acc) {
    const cx<T> kh = KH[r * NCC + c];
    const int rbase = r * P;
#pragma unroll
    for (int by = 0; by < NP; ++by) {
      const cx<T> w = WX[((rbase + by) * NCC + c) * NP + lx];
      const cx<T> z = ZX[((rbase + by) * NCC + c) * NP + lx];
      rmac(acc, (T)ref.K[ly * NP + by], w);
      cx<T> t = z - kh * w;
      rmac(acc, (T)ref.M[ly * NP + by], t);
    }
  };
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    if (r && !(ay0 == 0 && lasty)) break;
    const int ay = r ? P : ay0;
    const int iy = cyo * P + ay;
#pragma unroll
    for (int ax = 0; ax < NP; ++ax) {
      if (ax == P && !lastx) continue;
      const int ix = cxo * P + ax;
      const long long g = (long long)iy * n1 + ix;
      cx<T> acc = {0, 0};
      if (ay == 0 && below) {
        if (ax == 0 && left) cell(cc - 1, cr - 1, P, P, acc);
        cell(cc, cr - 1, ax, P, acc);
      }
      if (ax == 0 && left) cell(cc - 1, cr, P, ay, acc);
      cell(cc, cr, ax, ay, acc);
      if (op.robin && (ix == 0 || ix == NPn || iy == 0 || iy == NPn))
        robin_add<P, T>(op, ref, u, ix, iy, acc);
      if (op.dir && (on_dir(op.dir, 0, ix, NPn) || on_dir(op.dir, 1, iy, NPn))) acc = u[g];
      cx<T> o = fv[r][ax];
      o.re = fma(sgn, acc.re, o.re);
      o.im = fma(sgn, acc.im, o.im);
      out[g] = o;
    }
  }
}

// ---------------------------------------------------------------------------
// 3-D: per cell of size h the operator is
//   h (K1 (x) M1 (x) M1 + M1 (x) K1 (x) M1 + M1 (x) M1 (x) K1) - kappa_c h^3 M1 (x) M1 (x) M1
// (z (x) y (x) x), plus -i k_c h^2 M1 (x) M1 on cell faces lying on an absorbing
// side.  A workgroup owns the nodes of a TC^3 cell tile (low faces included)
// and stages the nodes of the tile grown by one cell on the low sides in LDS.
//   pass 1: per cell, node line (bz, ay): the x and y contractions
//           A1 = (My (x) Mx) u,  G = h (My (x) Kx + Ky (x) Mx) u
//   pass 2: every owned node sums, over the (at most 8) cells containing it,
//           the z contraction  Mz (G - kappa h^3 A1) + h Kz A1,
// again a fixed-order gather.  Orders 2 and 4 are provided in 3-D.
template <int P> struct Tile3Of;
template <> struct Tile3Of<2> { static constexpr int TC = 4; };
template <> struct Tile3Of<4> { static constexpr int TC = 2; };

template <int P, typename T>
__global__ __launch_bounds__(256) void k_apply3d(FineOp op, Ref1D ref, const cx<T> *__restrict__ u,
                                                 const cx<T> *__restrict__ f,
                                                 cx<T> *__restrict__ out, T sgn, int ntile) {
  constexpr int TC = Tile3Of<P>::TC;
  constexpr int NP = P + 1;
  constexpr int NC = TC + 1;          // staged cells per direction
  constexpr int NN = NC * P + 1;      // staged nodes per direction
  constexpr int CL = NP * NP * NP;    // partials per cell
  __shared__ cx<T> Us[NN * NN * NN];
  __shared__ cx<T> A1s[NC * NC * NC * CL];
  __shared__ cx<T> Gs[NC * NC * NC * CL];
  __shared__ T sK[NP * NP], sM[NP * NP];

  const int N = op.N, n1 = op.n1;
  const long long rb = (long long)blockIdx.y * op.nf;
  u += rb;
  out += rb;
  if (f) f += rb;

  const int tx = blockIdx.x % ntile, tt = blockIdx.x / ntile;
  const int ty = tt % ntile, tz = tt / ntile;
  const int cx0 = tx * TC, cy0 = ty * TC, cz0 = tz * TC;
  const int cxs = max(cx0 - 1, 0), cxe = min(cx0 + TC, N);
  const int cys = max(cy0 - 1, 0), cye = min(cy0 + TC, N);
  const int czs = max(cz0 - 1, 0), cze = min(cz0 + TC, N);
  const int ncx = cxe - cxs, ncy = cye - cys, ncz = cze - czs;
  const int nnx = ncx * P + 1, nny = ncy * P + 1, nnz = ncz * P + 1;

  for (int i = threadIdx.x; i < NP * NP; i += blockDim.x) {
    sK[i] = (T)ref.K[i];
    sM[i] = (T)ref.M[i];
  }
  for (int i = threadIdx.x; i < nnx * nny * nnz; i += blockDim.x) {
    const int jx = i % nnx, t = i / nnx;
    const int jy = t % nny, jz = t / nny;
    cx<T> v = u[((long long)(czs * P + jz) * n1 + cys * P + jy) * n1 + cxs * P + jx];
    if (op.dir && (on_dir(op.dir, 0, cxs * P + jx, N * P) || on_dir(op.dir, 1, cys * P + jy, N * P) ||
                   on_dir(op.dir, 2, czs * P + jz, N * P)))
      v = cx<T>{0, 0};
    Us[(jz * NN + jy) * NN + jx] = v;
  }
  __syncthreads();

  const T h = (T)op.h;
  // pass 1: items (cell, bz, ay)
  const int ncell = ncx * ncy * ncz;
  for (int it = threadIdx.x; it < ncell * NP * NP; it += blockDim.x) {
    const int ay = it % NP, t1 = it / NP;
    const int bz = t1 % NP, cl = t1 / NP;
    const int lx = cl % ncx, t2 = cl / ncx;
    const int ly = t2 % ncy, lz = t2 / ncy;
    cx<T> a1[NP], b1[NP], c1[NP];
#pragma unroll
    for (int a = 0; a < NP; ++a) a1[a] = b1[a] = c1[a] = cx<T>{0, 0};
    const cx<T> *ub = Us + ((lz * P + bz) * NN + ly * P) * NN + lx * P;
#pragma unroll
    for (int by = 0; by < NP; ++by) {
      cx<T> uv[NP];
#pragma unroll
      for (int bx = 0; bx < NP; ++bx) uv[bx] = ub[by * NN + bx];
      const T my = sM[ay * NP + by], ky = sK[ay * NP + by];
#pragma unroll
      for (int a = 0; a < NP; ++a) {
        cx<T> wm = {0, 0}, wk = {0, 0};
#pragma unroll
        for (int bx = 0; bx < NP; ++bx) {
          rmac(wm, sM[a * NP + bx], uv[bx]);
          rmac(wk, sK[a * NP + bx], uv[bx]);
        }
        rmac(a1[a], my, wm);
        rmac(b1[a], my, wk);
        rmac(c1[a], ky, wm);
      }
    }
    const int cell = (lz * NC + ly) * NC + lx;
#pragma unroll
    for (int a = 0; a < NP; ++a) {
      const int o = cell * CL + (bz * NP + ay) * NP + a;
      A1s[o] = a1[a];
      cx<T> g = b1[a] + c1[a];
      Gs[o] = cx<T>{h * g.re, h * g.im};
    }
  }
  __syncthreads();

  // pass 2 over owned nodes
  const int NPn = N * P;
  const int ix0 = cx0 * P, iy0 = cy0 * P, iz0 = cz0 * P;
  const int ix1 = (cx0 + TC >= N) ? NPn + 1 : (cx0 + TC) * P;
  const int iy1 = (cy0 + TC >= N) ? NPn + 1 : (cy0 + TC) * P;
  const int iz1 = (cz0 + TC >= N) ? NPn + 1 : (cz0 + TC) * P;
  const int nox = ix1 - ix0, noy = iy1 - iy0, noz = iz1 - iz0;
  const T h3 = (T)(op.h * op.h * op.h), h2 = (T)(op.h * op.h);

  for (int it = threadIdx.x; it < nox * noy * noz; it += blockDim.x) {
    const int jx = it % nox, t = it / nox;
    const int jy = t % noy, jz = t / noy;
    const int ix = ix0 + jx, iy = iy0 + jy, iz = iz0 + jz;
    const int chx = min(ix / P, N - 1), chy = min(iy / P, N - 1), chz = min(iz / P, N - 1);
    const int ncellx = (ix % P == 0 && ix > 0 && ix < NPn) ? 2 : 1;
    const int ncelly = (iy % P == 0 && iy > 0 && iy < NPn) ? 2 : 1;
    const int ncellz = (iz % P == 0 && iz > 0 && iz < NPn) ? 2 : 1;
    cx<T> acc = {0, 0};
    for (int qz = ncellz - 1; qz >= 0; --qz) {
      const int czq = chz - qz, az = iz - czq * P;
      for (int qy = ncelly - 1; qy >= 0; --qy) {
        const int cyq = chy - qy, ay = iy - cyq * P;
        for (int qx = ncellx - 1; qx >= 0; --qx) {
          const int cxq = chx - qx, ax = ix - cxq * P;
          const c64 kd = op.kap[((long long)czq * N + cyq) * N + cxq];
          const cx<T> kh = {(T)kd.re * h3, (T)kd.im * h3};
          const int cell = ((czq - czs) * NC + (cyq - cys)) * NC + (cxq - cxs);
#pragma unroll
          for (int bz = 0; bz < NP; ++bz) {
            const int o = cell * CL + (bz * NP + ay) * NP + ax;
            const cx<T> a1 = A1s[o], g = Gs[o];
            const T mz = sM[az * NP + bz], kz = sK[az * NP + bz];
            rmac(acc, mz, g - kh * a1);
            rmac(acc, h * kz, a1);
          }
        }
      }
    }
    // absorbing faces: -i h^2 k_c (M1 (x) M1 over the face) u
    if (op.robin) {
      cx<T> s = {0, 0};
      const int idx[3] = {ix, iy, iz};
      const int ch[3] = {chx, chy, chz};
      const int nq[3] = {ncellx, ncelly, ncellz};
      const int cs[3] = {cxs, cys, czs};
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const bool lo = idx[d] == 0 && (op.robin & (1 << (2 * d)));
        const bool hi = idx[d] == NPn && (op.robin & (2 << (2 * d)));
        if (!lo && !hi) continue;
        const int e1 = d == 0 ? 1 : 0, e2 = d == 2 ? 1 : 2;
        int cc[3];
        cc[d] = lo ? 0 : N - 1;
        for (int q2 = nq[e2] - 1; q2 >= 0; --q2) {
          cc[e2] = ch[e2] - q2;
          const int a2 = idx[e2] - cc[e2] * P;
          for (int q1 = nq[e1] - 1; q1 >= 0; --q1) {
            cc[e1] = ch[e1] - q1;
            const int a1 = idx[e1] - cc[e1] * P;
            const T kk = (T)op.kr[((long long)cc[2] * N + cc[1]) * N + cc[0]];
            cx<T> m = {0, 0};
            for (int b2 = 0; b2 < NP; ++b2) {
              cx<T> m1 = {0, 0};
              for (int b1 = 0; b1 < NP; ++b1) {
                int l[3];
                l[d] = idx[d] - cs[d] * P;
                l[e1] = (cc[e1] - cs[e1]) * P + b1;
                l[e2] = (cc[e2] - cs[e2]) * P + b2;
                rmac(m1, sM[a1 * NP + b1], Us[(l[2] * NN + l[1]) * NN + l[0]]);
              }
              rmac(m, sM[a2 * NP + b2], m1);
            }
            rmac(s, kk, m);
          }
        }
      }
      acc.re += h2 * s.im;
      acc.im -= h2 * s.re;
    }
    const long long g = ((long long)iz * n1 + iy) * n1 + ix;
    if (op.dir && (on_dir(op.dir, 0, ix, NPn) || on_dir(op.dir, 1, iy, NPn) ||
                   on_dir(op.dir, 2, iz, NPn)))
      acc = u[g];
    cx<T> o = f ? f[g] : cx<T>{0, 0};
    o.re = fma(sgn, acc.re, o.re);
    o.im = fma(sgn, acc.im, o.im);
    out[g] = o;
  }
}

template <int P, typename T>
static int launch_apply3_t(const FineOp &op, const Ref1D &ref, const void *u, const void *f,
                           void *out, int nrhs, double sgn, hipStream_t s) {
  constexpr int TC = Tile3Of<P>::TC;
  const int nt = ceil_div(op.N, TC);
  dim3 grid(nt * nt * nt, nrhs);
  hipLaunchKernelGGL((k_apply3d<P, T>), grid, dim3(256), 0, s, op, ref, (const cx<T> *)u,
                     (const cx<T> *)f, (cx<T> *)out, (T)sgn, nt);
  TH_HIP_CHECK_RET(hipGetLastError());
  return 0;
}

template <int P, int TC, typename T>
static void launch_apply2(const FineOp &op, const Ref1D &ref, const void *u, const void *f,
                          void *out, int nrhs, double sgn, hipStream_t s) {
  dim3 grid(ceil_div(op.N, TC), ceil_div(op.N, TC), nrhs);
  hipLaunchKernelGGL((k_apply2d<P, TC, T>), grid, dim3(Tile2<P, TC>::NT), 0, s, op, ref,
                     (const cx<T> *)u, (const cx<T> *)f, (cx<T> *)out, (T)sgn);
}

// Tile edge (cells) per order: the largest of three whose grid still has
// kApplyWGs workgroups, else the smallest (small meshes with one RHS would
// otherwise leave most of the chip idle; every workgroup's time is about one
// memory round trip, so more and smaller tiles finish sooner).
constexpr long long kApplyWGs = 256;
template <int P> struct Tiles2;
template <> struct Tiles2<2> { static constexpr int t[3] = {16, 8, 4}; };
template <> struct Tiles2<4> { static constexpr int t[3] = {8, 4, 2}; };
template <> struct Tiles2<6> { static constexpr int t[3] = {5, 3, 2}; };
template <> struct Tiles2<8> { static constexpr int t[3] = {4, 2, 1}; };

template <int P, typename T>
static int launch_apply_t(const FineOp &op, const Ref1D &ref, const void *u, const void *f,
                          void *out, int nrhs, double sgn, hipStream_t s) {
  auto wgs = [&](int tc) { return (long long)ceil_div(op.N, tc) * ceil_div(op.N, tc) * nrhs; };
  constexpr int T0 = Tiles2<P>::t[0], T1 = Tiles2<P>::t[1], T2 = Tiles2<P>::t[2];
  if (wgs(T0) >= kApplyWGs)
    launch_apply2<P, T0, T>(op, ref, u, f, out, nrhs, sgn, s);
  else if (wgs(T1) >= kApplyWGs)
    launch_apply2<P, T1, T>(op, ref, u, f, out, nrhs, sgn, s);
  else
    launch_apply2<P, T2, T>(op, ref, u, f, out, nrhs, sgn, s);
  TH_HIP_CHECK_RET(hipGetLastError());
  return 0;
}

int launch_apply(const FineOp &op, const Ref1D &ref, const void *u, const void *f, void *out,
                 int nrhs, bool f32, double sgn, hipStream_t s) {
  if (op.dim == 3) {
    switch (op.P) {
      case 2: return f32 ? launch_apply3_t<2, float>(op, ref, u, f, out, nrhs, sgn, s)
                         : launch_apply3_t<2, double>(op, ref, u, f, out, nrhs, sgn, s);
      case 4: return f32 ? launch_apply3_t<4, float>(op, ref, u, f, out, nrhs, sgn, s)
                         : launch_apply3_t<4, double>(op, ref, u, f, out, nrhs, sgn, s);
    }
    set_error("3-D problems support orders 2 and 4");
    return TH_EUNSUPPORTED;
  }
  switch (op.P) {
    case 2: return f32 ? launch_apply_t<2, float>(op, ref, u, f, out, nrhs, sgn, s)
                       : launch_apply_t<2, double>(op, ref, u, f, out, nrhs, sgn, s);
    case 4: return f32 ? launch_apply_t<4, float>(op, ref, u, f, out, nrhs, sgn, s)
                       : launch_apply_t<4, double>(op, ref, u, f, out, nrhs, sgn, s);
    case 6: return f32 ? launch_apply_t<6, float>(op, ref, u, f, out, nrhs, sgn, s)
                       : launch_apply_t<6, double>(op, ref, u, f, out, nrhs, sgn, s);
    case 8: return f32 ? launch_apply_t<8, float>(op, ref, u, f, out, nrhs, sgn, s)
                       : launch_apply_t<8, double>(op, ref, u, f, out, nrhs, sgn, s);
  }
  set_error("unsupported order");
  return TH_EUNSUPPORTED;
}

}  // namespace th
