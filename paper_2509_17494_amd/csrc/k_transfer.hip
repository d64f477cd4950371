// Inter-grid transfers (Sec. 4.2): prolongation I_P = Q_{p/2} interpolation
// from the coarse vertex grid (spacing 2h/p) to the fine GLL nodes, and the
// restriction I_P^T of Alg. 1.
//
// On each fine cell the interpolant is a tensor product of 1-D degree-p/2
// Lagrange interpolants through the r+1 = p/2+1 coarse points of the cell, so
// the global operator is P1 (x) P1 (x P1 in 3-D) with P1 the (pN+1) x (rN+1) 1-D matrix
// P1[i][J] = L[a][b], (c, a) = cell and local index of fine node i, b = J - c r
// (cell-edge nodes get the same value from either cell: they coincide with
// coarse points).  Both kernels are gathers (no atomics): prolongation per
// fine node over the (r+1)^d coarse points of its cell, restriction per
// coarse point over the fine nodes of the cells around it, every fine node
// counted once.
//
// Dirichlet sides (dir, bit per side): their fine nodes and coarse vertices are
// not unknowns; the rows of I_P for those fine nodes and its columns for those
// vertices are zero.  The weights are masked per axis (a point lies on a
// Dirichlet side when one of its coordinates does).
#include "ctx.hpp"

namespace th {

template <int P>
__device__ __forceinline__ double p1w(const double *L, int N, int i, int J) {
  constexpr int R = P / 2;
  const int c = min(i / P, N - 1);
  const int a = i - c * P, b = J - c * R;
  return (b >= 0 && b <= R) ? L[a * (R + 1) + b] : 0.0;
}

// The grids are n1^DIM (fine) and nc1^DIM (coarse), x fastest; in 2-D the z
// loops collapse to one iteration with unit weight.  The coarse vector has its
// own type TV: a complex64 two-grid step reads and writes the FP64 coarse
// solve's vectors directly, rounding each coarse value to T as it is read
// (prolongation) or the T sum to FP64 as it is stored (restriction), which is
// what a separate conversion would do.
template <int DIM, int P, typename T, typename TV>
__global__ __launch_bounds__(256) void k_prolong(int N, int dir, Ref1D ref,
                                                 const cx<TV> *__restrict__ uc,
                                                 cx<T> *__restrict__ u, T omega, long long nf,
                                                 long long ncn) {
  constexpr int R = P / 2;
  constexpr int RZ = DIM == 3 ? R : 0;
  const int n1 = N * P + 1, nc1 = N * R + 1;
  const long long rhs = blockIdx.y;
  uc += rhs * ncn;
  u += rhs * nf;
  for (long long g = blockIdx.x * (long long)blockDim.x + threadIdx.x; g < nf;
       g += (long long)gridDim.x * blockDim.x) {
    const int ix = (int)(g % n1);
    const long long t = g / n1;
    const int iy = (int)(t % n1), iz = (int)(t / n1);
    const int cxq = min(ix / P, N - 1), cyq = min(iy / P, N - 1);
    const int czq = DIM == 3 ? min(iz / P, N - 1) : 0;
    const int ax = ix - cxq * P, ay = iy - cyq * P, az = iz - czq * P;
    if (dir && (on_dir(dir, 0, ix, n1 - 1) || on_dir(dir, 1, iy, n1 - 1) ||
                (DIM == 3 && on_dir(dir, 2, iz, n1 - 1))))
      continue;  // a zero row of I_P: u keeps its value
    cx<T> acc = {0, 0};
#pragma unroll
    for (int bz = 0; bz <= RZ; ++bz) {
      const T wz = DIM == 3 ? (T)ref.L[az * (R + 1) + bz] : (T)1;
      if (wz == (T)0 || (DIM == 3 && on_dir(dir, 2, czq * R + bz, nc1 - 1))) continue;
      cx<T> pl = {0, 0};
#pragma unroll
      for (int by = 0; by <= R; ++by) {
        const T wy = (T)ref.L[ay * (R + 1) + by];
        if (wy == (T)0 || on_dir(dir, 1, cyq * R + by, nc1 - 1)) continue;
        cx<T> row = {0, 0};
        const cx<TV> *ucr = uc + ((long long)(czq * R + bz) * nc1 + cyq * R + by) * nc1 + cxq * R;
#pragma unroll
        for (int bx = 0; bx <= R; ++bx) {
          const T wx = (T)ref.L[ax * (R + 1) + bx];
          if (wx == (T)0 || on_dir(dir, 0, cxq * R + bx, nc1 - 1)) continue;
          rmac(row, wx, ccast<T>(ucr[bx]));
        }
        rmac(pl, wy, row);
      }
      if (DIM == 3) rmac(acc, wz, pl);
      else acc = pl;
    }
    cx<T> o = u[g];
    o.re = fma(omega, acc.re, o.re);
    o.im = fma(omega, acc.im, o.im);
    u[g] = o;
  }
}

template <int DIM, int P, typename T, typename TV>
__global__ __launch_bounds__(256) void k_restrict(int N, int dir, Ref1D ref,
                                                  const cx<T> *__restrict__ r,
                                                  cx<TV> *__restrict__ rc, long long nf,
                                                  long long ncn) {
  constexpr int R = P / 2;
  const int n1 = N * P + 1, nc1 = N * R + 1;
  const long long rhs = blockIdx.y;
  r += rhs * nf;
  rc += rhs * ncn;
  for (long long G = blockIdx.x * (long long)blockDim.x + threadIdx.x; G < ncn;
       G += (long long)gridDim.x * blockDim.x) {
    const int Jx = (int)(G % nc1);
    const long long t = G / nc1;
    const int Jy = (int)(t % nc1), Jz = (int)(t / nc1);
    if (on_dir(dir, 0, Jx, nc1 - 1) || on_dir(dir, 1, Jy, nc1 - 1) ||
        (DIM == 3 && on_dir(dir, 2, Jz, nc1 - 1))) {
      rc[G] = cx<TV>{0, 0};
      continue;
    }
    // cells whose coarse points include J: c R <= J <= c R + R; fine node range of those cells
    const int ixs = max((Jx % R == 0) ? Jx / R - 1 : Jx / R, 0) * P;
    const int ixe = (min(Jx / R, N - 1) + 1) * P;
    const int iys = max((Jy % R == 0) ? Jy / R - 1 : Jy / R, 0) * P;
    const int iye = (min(Jy / R, N - 1) + 1) * P;
    const int izs = DIM == 3 ? max((Jz % R == 0) ? Jz / R - 1 : Jz / R, 0) * P : 0;
    const int ize = DIM == 3 ? (min(Jz / R, N - 1) + 1) * P : 0;
    cx<T> acc = {0, 0};
    for (int iz = izs; iz <= ize; ++iz) {
      const T wz = DIM == 3 ? (T)p1w<P>(ref.L, N, iz, Jz) : (T)1;
      if (wz == (T)0 || (DIM == 3 && on_dir(dir, 2, iz, n1 - 1))) continue;
      cx<T> pl = {0, 0};
      for (int iy = iys; iy <= iye; ++iy) {
        const T wy = (T)p1w<P>(ref.L, N, iy, Jy);
        if (wy == (T)0 || on_dir(dir, 1, iy, n1 - 1)) continue;
        cx<T> row = {0, 0};
        const cx<T> *rr = r + ((long long)iz * n1 + iy) * n1;
        for (int ix = ixs; ix <= ixe; ++ix) {
          const T wx = (T)p1w<P>(ref.L, N, ix, Jx);
          if (wx == (T)0 || on_dir(dir, 0, ix, n1 - 1)) continue;
          rmac(row, wx, rr[ix]);
        }
        rmac(pl, wy, row);
      }
      if (DIM == 3) rmac(acc, wz, pl);
      else acc = pl;
    }
    rc[G] = ccast<TV>(acc);
  }
}

static long long ipow(long long b, int e) {
  long long r = 1;
  while (e-- > 0) r *= b;
  return r;
}

template <int DIM, int P, typename T, typename TV>
static int prolong_t(int N, int dir, const Ref1D &ref, const void *uc, void *u, double omega,
                     int nrhs, hipStream_t s) {
  const long long nf = ipow(N * P + 1, DIM), ncn = ipow(N * (P / 2) + 1, DIM);
  int blocks = (int)std::min<long long>(ceil_div_ll(nf, 256), 65535);
  hipLaunchKernelGGL((k_prolong<DIM, P, T, TV>), dim3(blocks, nrhs), dim3(256), 0, s, N, dir, ref,
                     (const cx<TV> *)uc, (cx<T> *)u, (T)omega, nf, ncn);
  TH_HIP_CHECK_RET(hipGetLastError());
  return 0;
}

template <int DIM, int P, typename T, typename TV>
static int restrict_t(int N, int dir, const Ref1D &ref, const void *r, void *rc, int nrhs,
                      hipStream_t s) {
  const long long nf = ipow(N * P + 1, DIM), ncn = ipow(N * (P / 2) + 1, DIM);
  int blocks = (int)std::min<long long>(ceil_div_ll(ncn, 256), 65535);
  hipLaunchKernelGGL((k_restrict<DIM, P, T, TV>), dim3(blocks, nrhs), dim3(256), 0, s, N, dir, ref,
                     (const cx<T> *)r, (cx<TV> *)rc, nf, ncn);
  TH_HIP_CHECK_RET(hipGetLastError());
  return 0;
}

#define TH_DISPATCH_P(P_, F32_, CALL_F, CALL_D)   \
  switch (P_) {                                   \
    case 2: return F32_ ? CALL_F(2) : CALL_D(2);  \
    case 4: return F32_ ? CALL_F(4) : CALL_D(4);  \
    case 6: return F32_ ? CALL_F(6) : CALL_D(6);  \
    case 8: return F32_ ? CALL_F(8) : CALL_D(8);  \
  }

int launch_prolong(int dim, int N, int P, int dir, const Ref1D &ref, const void *uc, void *u,
                   double omega, int nrhs, bool f32, hipStream_t s, bool coarse64) {
  if (dim == 3) {
#define CF(p) (coarse64 ? prolong_t<3, p, float, double>(N, dir, ref, uc, u, omega, nrhs, s) \
                        : prolong_t<3, p, float, float>(N, dir, ref, uc, u, omega, nrhs, s))
#define CD(p) prolong_t<3, p, double, double>(N, dir, ref, uc, u, omega, nrhs, s)
    TH_DISPATCH_P(P, f32, CF, CD)
#undef CF
#undef CD
  } else {
#define CF(p) (coarse64 ? prolong_t<2, p, float, double>(N, dir, ref, uc, u, omega, nrhs, s) \
                        : prolong_t<2, p, float, float>(N, dir, ref, uc, u, omega, nrhs, s))
#define CD(p) prolong_t<2, p, double, double>(N, dir, ref, uc, u, omega, nrhs, s)
    TH_DISPATCH_P(P, f32, CF, CD)
#undef CF
#undef CD
  }
  set_error("unsupported order");
  return TH_EUNSUPPORTED;
}

int launch_restrict(int dim, int N, int P, int dir, const Ref1D &ref, const void *r, void *rc,
                    int nrhs, bool f32, hipStream_t s, bool coarse64) {
  if (dim == 3) {
#define CF(p) (coarse64 ? restrict_t<3, p, float, double>(N, dir, ref, r, rc, nrhs, s) \
                        : restrict_t<3, p, float, float>(N, dir, ref, r, rc, nrhs, s))
#define CD(p) restrict_t<3, p, double, double>(N, dir, ref, r, rc, nrhs, s)
    TH_DISPATCH_P(P, f32, CF, CD)
#undef CF
#undef CD
  } else {
#define CF(p) (coarse64 ? restrict_t<2, p, float, double>(N, dir, ref, r, rc, nrhs, s) \
                        : restrict_t<2, p, float, float>(N, dir, ref, r, rc, nrhs, s))
#define CD(p) restrict_t<2, p, double, double>(N, dir, ref, r, rc, nrhs, s)
    TH_DISPATCH_P(P, f32, CF, CD)
#undef CF
#undef CD
  }
  set_error("unsupported order");
  return TH_EUNSUPPORTED;
}

}  // namespace th
