// Device helpers shared by the slab-factor kernels (k_slab.hip: setup, the
// sweeps over whole G_t; k_slab_pk.hip: the sweeps over packed G_t): slab
// geometry, the two storages of G_t, the coupling-band products and the
// workgroup order of the sweeps.
#pragma once

#include "ctx.hpp"

namespace th {

__host__ __device__ __forceinline__ int slab_rows(const Sub &s, int t, int P) {
  return (t < s.nsl - 1 ? P : P + 1) * s.lsz;
}

__host__ __device__ __forceinline__ int slab_ld(int m) { return (m + 7) & ~7; }

// entries of the G_t of slabs before t (all of them have P layers)
__host__ __device__ __forceinline__ long long slab_goff(const Sub &s, int t, int P) {
  const int m = P * s.lsz;
  return s.boff + (long long)t * m * slab_ld(m);
}

// Packed storage of a symmetric G_t (m x m): its nf = m / 64 full 64-row
// blocks hold the lower block triangle as skewed 64 x 64 tiles, its last
// m - 64 nf rows a dense strip.  Tile (R, C), R >= C, step k, lane l holds
// G[64 R + (l + k) mod 64][64 C + l] at 64 (step) + l: one step is 64
// consecutive entries, and lane l meets column l and row (l + k) of the tile,
// so one load serves both G x and G^T x (the mirrored half of the tile is
// never read).  Diagonal tiles need steps 0 .. 32 only (steps k and 64 - k
// mirror each other; step 32 holds every pair twice).  Tiles are ordered by
// column block, the diagonal tile (steps 0 .. 31) first; then step 32 of
// every diagonal tile, in block order; then the strip (rows 64 nf + j, all m
// columns, rows padded to slab_ld(m)).  About m (m + 1) / 2 entries instead
// of m slab_ld(m).
__host__ __device__ __forceinline__ long long pk_tile_steps(int nf) {
  return 33LL * nf + 32LL * nf * (nf - 1);
}
__host__ __device__ __forceinline__ long long pk_elems(int m) {
  const int nf = m / 64;
  return 64 * pk_tile_steps(nf) + (long long)(m - 64 * nf) * slab_ld(m);
}
__host__ __device__ __forceinline__ long long pk_goff(const Sub &s, int t, int P) {
  return s.boff + (long long)t * pk_elems(P * s.lsz);
}
// tile and step of packed step index st
__host__ __device__ __forceinline__ void pk_step(int nf, long long st, int &R, int &C, int &k) {
  if (st >= 32LL * nf * nf) {  // step 32 of the diagonal tiles
    R = C = (int)(st - 32LL * nf * nf);
    k = 32;
    return;
  }
  int c = 0;
  for (;;) {
    const long long n = 32 + 64LL * (nf - 1 - c);
    if (st < n) break;
    st -= n;
    ++c;
  }
  C = c;
  if (st < 32) {
    R = c;
    k = (int)st;
  } else {
    R = c + 1 + (int)((st - 32) / 64);
    k = (int)((st - 32) % 64);
  }
}

__host__ __device__ __forceinline__ int band_width(int P, int dim) {
  return (dim == 3 ? (2 * P + 1) * (2 * P + 1) : (2 * P + 1)) * P;
}

// middle slab of the twisted elimination; the lower chain has slab_mid
// slabs, the upper chain nsl - 1 - slab_mid
__host__ __device__ __forceinline__ int slab_mid(const Sub &s) { return (s.nsl - 1) / 2; }

enum { kLowerChain = 0, kUpperChain = 1, kMiddle = 2 };

// The slab t of subdomain s at step i of a chain of n aligned steps (lower
// slab t at step t + n - D, upper slab nsl - 1 - j at step j + n - U), or the
// middle.  on: the subdomain has a slab at this step; lo / up: the correction
// from the lower (t - 1) / upper (t + 1) neighbour applies; rev: the block is
// handled in reversed node order during setup.
struct SlabRole {
  int t, on, lo, up, rev;
};

__host__ __device__ __forceinline__ SlabRole slab_role(const Sub &s, int mode, int i, int n) {
  const int M = slab_mid(s), U = s.nsl - 1 - M;
  SlabRole r;
  if (mode == kLowerChain) {
    r.t = i - (n - M);
    r.on = r.t >= 0;
    r.lo = r.t >= 1;
    r.up = 0;
    r.rev = 0;
  } else if (mode == kUpperChain) {
    const int j = i - (n - U);
    r.t = s.nsl - 1 - j;
    r.on = j >= 0;
    r.lo = 0;
    r.up = j >= 1;
    r.rev = 1;
  } else {
    r.t = M;
    r.on = 1;
    r.lo = M >= 1;
    r.up = U >= 1;
    r.rev = 0;
  }
  return r;
}

// Omega-local index of band entry k of first-layer node a of slab t (t >= 1),
// or -1 outside Omega.  k = ((jy (2P+1)) + jx) P + lb; the node sits at
// in-layer position (xa - P + jx, ya - P + jy) in layer (t - 1) P + lb.
__device__ __forceinline__ int band_col(const Sub &s, int t, int a, int k, int P, int dim) {
  const int lb = k % P, j = k / P;
  const int jx = j % (2 * P + 1), jy = j / (2 * P + 1);
  const int xa = a % s.nox, ya = dim == 3 ? a / s.nox : 0;
  const int xb = xa - P + jx, yb = dim == 3 ? ya - P + jy : 0;
  if (xb < 0 || xb >= s.nox || yb < 0 || (dim == 3 && yb >= s.noy)) return -1;
  return ((t - 1) * P + lb) * s.lsz + yb * s.nox + xb;
}

// acc[q] = sum over the band of first-layer node j of slab t (t >= 1) of
// A[t][t-1] times v[slab t - 1] (vb: offset of slab t - 1 of right-hand side
// r0).  Branch-free: positions outside Omega are clamped to a node inside
// (its value is finite) and meet a zero band coefficient, so every load can
// be issued before its use.
template <typename TB, typename T, int RC, int P, int DIM>
__device__ __forceinline__ void band_lower(const Sub &s, const cx<TB> *__restrict__ Ct,
                                           const cx<T> *__restrict__ V, long long vb,
                                           long long xrows, int nq, int j, cx<T> (&acc)[RC]) {
  constexpr int W2 = 2 * P + 1;
  const int xa = j % s.nox, ya = DIM == 3 ? j / s.nox : 0;
  const cx<TB> *cr = Ct + j;
#pragma unroll
  for (int q = 0; q < RC; ++q) acc[q] = {0, 0};
#pragma unroll
  for (int jy = 0; jy < (DIM == 3 ? W2 : 1); ++jy) {
    const int yb = DIM == 3 ? min(max(ya - P + jy, 0), s.noy - 1) : 0;
#pragma unroll
    for (int jx = 0; jx < W2; ++jx) {
      const int xb = min(max(xa - P + jx, 0), s.nox - 1);
      cx<TB> l[P];
      cx<T> y[P][RC];
#pragma unroll
      for (int lb = 0; lb < P; ++lb) {
        l[lb] = cr[(long long)((jy * W2 + jx) * P + lb) * s.lsz];
#pragma unroll
        for (int q = 0; q < RC; ++q)
          y[lb][q] = V[vb + (long long)min(q, nq - 1) * xrows + lb * s.lsz + yb * s.nox + xb];
      }
#pragma unroll
      for (int lb = 0; lb < P; ++lb)
#pragma unroll
        for (int q = 0; q < RC; ++q) cmac(acc[q], ccast<T>(l[lb]), y[lb][q]);
    }
  }
}

// acc[q] = (A[t][t+1] v[first layer of t + 1])[j] for node j of slab t
// (t + 1 <= nsl - 1, so slab t has P layers): the band of slab t + 1 read
// transposed, node j in layer lb couples to the first-layer nodes a within P
// positions, through band entry ((2P - jy') (2P+1) + 2P - jx') P + lb of a,
// where a sits at (xj - P + jx', yj - P + jy').  Cn: band of slab t + 1, vn:
// offset of its first layer.  Out-of-range a are clamped and their
// coefficient replaced by zero.
template <typename TB, typename T, int RC, int P, int DIM>
__device__ __forceinline__ void band_upper(const Sub &s, const cx<TB> *__restrict__ Cn,
                                           const cx<T> *__restrict__ V, long long vn,
                                           long long xrows, int nq, int j, cx<T> (&acc)[RC]) {
  constexpr int W2 = 2 * P + 1;
  const int lb = j / s.lsz, jj = j - lb * s.lsz;
  const int xj = jj % s.nox, yj = DIM == 3 ? jj / s.nox : 0;
#pragma unroll
  for (int q = 0; q < RC; ++q) acc[q] = {0, 0};
#pragma unroll
  for (int jy = 0; jy < (DIM == 3 ? W2 : 1); ++jy) {
    const int ya = DIM == 3 ? yj - P + jy : 0;
    const bool iny = DIM == 3 ? (ya >= 0 && ya < s.noy) : true;
    const int yac = DIM == 3 ? min(max(ya, 0), s.noy - 1) : 0;
    cx<TB> l[W2];
    cx<T> y[W2][RC];
#pragma unroll
    for (int jx = 0; jx < W2; ++jx) {
      const int xa = xj - P + jx;
      const int xac = min(max(xa, 0), s.nox - 1);
      const int a = yac * s.nox + xac;
      const int k = (((DIM == 3 ? 2 * P - jy : 0) * W2) + 2 * P - jx) * P + lb;
      l[jx] = Cn[(long long)k * s.lsz + a];
      if (!(iny && xa >= 0 && xa < s.nox)) l[jx] = cx<TB>{0, 0};
#pragma unroll
      for (int q = 0; q < RC; ++q) y[jx][q] = V[vn + (long long)min(q, nq - 1) * xrows + a];
    }
#pragma unroll
    for (int jx = 0; jx < W2; ++jx)
#pragma unroll
      for (int q = 0; q < RC; ++q) cmac(acc[q], ccast<T>(l[jx]), y[jx][q]);
  }
}

// Workgroup -> (subdomain, row block, right-hand-side chunk) of the sweep
// launches, XCD-aware: workgroup b runs on XCD b % 8, and all row blocks of a
// subdomain get consecutive b with the same remainder, so the workgroups that
// each stage the same slab right-hand side (band products included) share one
// L2.  Returns false for the padding workgroups of the last group.
struct SweepItem {
  int si, yb, z;
};
__device__ __forceinline__ bool sweep_item(int nsub, int ny, SweepItem &it) {
  const int b = blockIdx.x, t = b >> 3;
  const int groups = (nsub + 7) >> 3;
  it.yb = t % ny;
  const int g = (t / ny) % groups;
  it.z = t / (ny * groups);
  it.si = 8 * g + (b & 7);
  return it.si < nsub;
}

// dispatch of the packed sweeps (k_slab_pk.hip) for rc right-hand sides per chunk
template <typename TB, typename T>
int slab_pk_sweeps(const th_ctx *c, int nrhs, int rc, hipStream_t s);

}  // namespace th
