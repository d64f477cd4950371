// Sweeps of the slab-factor subdomain solves over packed G_t (each
// symmetric G_t stored once; the storage is described with pk_elems).
#include <algorithm>

#include "k_slab.hpp"

namespace th {

// Packed G_t: the forward sweep of each chain in one launch, one workgroup per
// (subdomain, chain) and right-hand-side chunk walking its slabs in order
// (k_slab_fwd_chain), then the middles (k_slab_fwd_pk), then the backward
// sweep of each chain in one launch (k_slab_bwd_chain): three launches per
// application instead of one per step, since a chain depends on nothing but
// its own previous slab; the middle needs both chains, the backward the
// middle.  The loads of G_t never depend on the right-hand side, so a
// workgroup streams its chain's factors without a break: the loads of the
// next slab's first units go out while the current slab is finished.
//
// In a forward slab the kPkWaves wavefronts share the work units of G_t:
// segments of kPkLoads steps of a tile, the diagonal tiles' steps 32 in groups
// and the rows of the strip, each at most kPkLoads loads of 64 consecutive
// entries, the next unit's loads issued before the current one is used.  In a tile segment lane l keeps aC, the partial of G x for row
// 64 C + l (column product, from x of the row block), and aR, the partial for
// row 64 R + (l + k) mod 64 (row product, from x of the column block), which
// moves one lane down after every step so that each lane always adds to the
// row its next entry belongs to.  Diagonal tiles skip the row product at step
// 0 and have it not at step 32, whose entries the column product already
// counts in full.  A strip
// row is a dense row product (reduced over the wavefront) plus column products
// into the full blocks.  Each wavefront adds its partials into its own LDS
// rows; the sum over the wavefronts in a fixed order gives y_t, which is
// written out and kept in LDS for the next slab's coupling product.
constexpr int kPkWaves = 8, kPkLoads = 8;
constexpr int kPkMaxRows = 64 * kPkLoads;  // a strip row is one work unit
constexpr int kPkBwdRows = 8;              // rows of E_t^T (G_t^T) per backward unit

// value held by lane (l + 1) mod 64 (DPP wavefront rotation)
__device__ __forceinline__ float lane_next(float v) {
  return __builtin_bit_cast(
      float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x134, 0xf, 0xf, false));
}
__device__ __forceinline__ double lane_next(double v) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)u, 0x134, 0xf, 0xf,
                                                            false);
  const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), 0x134,
                                                            0xf, 0xf, false);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// slab t of a subdomain in the packed storage: rows, full 64-row blocks,
// strip row length, work units (4 nf^2 tile segments of kPkLoads steps, the
// diagonal tiles' steps 32 in groups of kPkLoads, the strip rows), offset of
// its G_t in the store and of its strip
struct PkSlab {
  int t, m, nf, ld, nseg, nk32, nunit;
  long long g0, nt;
};
__device__ __forceinline__ PkSlab pk_slab(const Sub &s, int t, int P) {
  PkSlab c;
  c.t = t;
  c.m = slab_rows(s, t, P);
  c.nf = c.m / 64;
  c.ld = slab_ld(c.m);
  c.nseg = 4 * c.nf * c.nf;
  c.nk32 = (c.nf + kPkLoads - 1) / kPkLoads;
  c.nunit = c.nseg + c.nk32 + (c.m - 64 * c.nf);
  c.g0 = pk_goff(s, t, P);
  c.nt = 64 * pk_tile_steps(c.nf);
  return c;
}

// one work unit: cnt loads at base + 64 q (+ lane) from the store; kind 0: a
// tile segment (steps k0 .. k0 + cnt - 1 of tile (R, C)), 1: steps 32 of the
// diagonal tiles C .. C + cnt - 1, 2: strip row R (entries past m not used)
struct PkUnit {
  long long base;
  int cnt, R, C, k0, kind, m;
};
__device__ __forceinline__ PkUnit pk_unit(int u, const PkSlab &c) {
  PkUnit w;
  w.m = c.m;
  w.k0 = 0;
  if (u < c.nseg) {
    const int nf = c.nf;
    int col = 0, seg = u;
    long long st = 0;
    for (;;) {
      const int ns = 4 + 8 * (nf - 1 - col);
      if (seg < ns) break;
      seg -= ns;
      st += 32 + 64LL * (nf - 1 - col);
      ++col;
    }
    w.C = col;
    w.kind = 0;
    w.cnt = kPkLoads;
    if (seg < 4) {
      w.R = col;
      w.k0 = kPkLoads * seg;
      st += w.k0;
    } else {
      const int o = seg - 4;
      w.R = col + 1 + o / 8;
      w.k0 = kPkLoads * (o % 8);
      st += 32 + 64LL * (o / 8) + w.k0;
    }
    w.base = c.g0 + 64 * st;
  } else if (u < c.nseg + c.nk32) {
    w.kind = 1;
    w.C = kPkLoads * (u - c.nseg);
    w.R = w.C;
    w.cnt = min(kPkLoads, c.nf - w.C);
    w.base = c.g0 + 64 * (32LL * c.nf * c.nf + w.C);
  } else {
    w.kind = 2;
    w.R = u - c.nseg - c.nk32;
    w.C = 0;
    w.cnt = (c.m + 63) / 64;
    w.base = c.g0 + c.nt + (long long)w.R * c.ld;
  }
  return w;
}

// All kPkLoads loads of a unit, none predicated: a strip row's lanes past m
// and the loads past cnt of a short unit read an entry of the unit again
// (values pk_compute never uses), so every unit issues the same loads and a
// buffer's loads are waited for exactly where they are used.
template <typename TB, typename T>
__device__ __forceinline__ void pk_load(const cx<TB> *__restrict__ B, const PkUnit &w, int lane,
                                        cx<T> (&gv)[kPkLoads]) {
  const cx<TB> *p = B + w.base;
#pragma unroll
  for (int q = 0; q < kPkLoads; ++q) {
    const int qq = min(q, w.cnt - 1), e = 64 * qq + lane;
    gv[q] = ccast<T>(ld_stream(p + (w.kind != 2 || e < w.m ? e : 0)));
  }
}

// a unit's products into the wavefront's partials pw (rows of the full
// blocks); a strip row's value goes to out (and to keep, when given)
template <typename T, int RC>
__device__ __forceinline__ void pk_compute(const PkUnit &w, const cx<T> (&gv)[kPkLoads],
                                           const cx<T> *__restrict__ x, cx<T> *__restrict__ pw,
                                           int nf, int lane, cx<T> *__restrict__ out,
                                           long long xrows, int nq, cx<T> *__restrict__ keep) {
  if (w.kind == 0) {
    const int R = w.R, C = w.C;
    // the row product skips step 0 of a diagonal tile (its entries, the
    // diagonal, are counted by the column product)
    const bool skip0 = R == C && w.k0 == 0;
    cx<T> xc[RC], aC[RC], aR[RC];
#pragma unroll
    for (int q = 0; q < RC; ++q) {
      xc[q] = x[(64 * C + lane) * RC + q];
      aC[q] = aR[q] = cx<T>{0, 0};
    }
#pragma unroll
    for (int u = 0; u < kPkLoads; ++u) {
      const int rr = 64 * R + ((lane + w.k0 + u) & 63);
#pragma unroll
      for (int q = 0; q < RC; ++q) cmac(aC[q], gv[u], x[rr * RC + q]);
      if (u > 0 || !skip0)
#pragma unroll
        for (int q = 0; q < RC; ++q) cmac(aR[q], gv[u], xc[q]);
#pragma unroll
      for (int q = 0; q < RC; ++q) aR[q] = cx<T>{lane_next(aR[q].re), lane_next(aR[q].im)};
    }
    const int k1 = w.k0 + kPkLoads;
#pragma unroll
    for (int q = 0; q < RC; ++q) {
      cx<T> &pc = pw[(64 * C + lane) * RC + q];
      pc = pc + aC[q];
    }
#pragma unroll
    for (int q = 0; q < RC; ++q) {
      cx<T> &pr = pw[(64 * R + ((lane + k1) & 63)) * RC + q];
      pr = pr + aR[q];
    }
    return;
  }
  if (w.kind == 1) {
    // step 32 of diagonal tile C + u: column product only
#pragma unroll
    for (int u = 0; u < kPkLoads; ++u)
      if (u < w.cnt) {
        const int c0 = 64 * (w.C + u);
#pragma unroll
        for (int q = 0; q < RC; ++q) {
          cx<T> &pc = pw[(c0 + lane) * RC + q];
          cmac(pc, gv[u], x[(c0 + ((lane + 32) & 63)) * RC + q]);
        }
      }
    return;
  }
  const int r = 64 * nf + w.R;
  cx<T> xr[RC], acc[RC];
#pragma unroll
  for (int q = 0; q < RC; ++q) {
    xr[q] = x[r * RC + q];
    acc[q] = cx<T>{0, 0};
  }
#pragma unroll
  for (int u = 0; u < kPkLoads; ++u) {
    if (u < w.cnt) {
      const int c = 64 * u + lane;
      const bool ok = c < w.m;
      const cx<T> g = ok ? gv[u] : cx<T>{0, 0};
      const int cc = ok ? c : 0;
#pragma unroll
      for (int q = 0; q < RC; ++q) cmac(acc[q], g, x[cc * RC + q]);
      if (u < nf)
#pragma unroll
        for (int q = 0; q < RC; ++q) {
          cx<T> &pc = pw[c * RC + q];
          cmac(pc, gv[u], xr[q]);
        }
    }
  }
#pragma unroll
  for (int q = 0; q < RC; ++q) {
    const cx<T> v = {wave_sum(acc[q].re), wave_sum(acc[q].im)};
    if (lane == 0) {
      if (q < nq) out[(long long)q * xrows + r] = v;
      if (keep) keep[r * RC + q] = v;
    }
  }
}

// This wavefront's units of slab c (u = wave, wave + kPkWaves, ...: n of
// them) in two register buffers: the load sequence is its units, one repeat
// of the last if n is odd, its first unit of slab nx (has_nx; else a repeat),
// and the buffers take them in turn (A, B, A, ...), so that on return A holds
// the next slab's first unit, whose loads are in flight.  Each unit's
// successor is loaded before the unit is used, and no value moves between
// the buffers.  On entry A holds the first unit (if any).
template <typename TB, typename T, int RC>
__device__ __forceinline__ void pk_units(const cx<TB> *__restrict__ B, const PkSlab &c,
                                         const PkSlab &nx, bool has_nx, PkUnit &uA,
                                         cx<T> (&gA)[kPkLoads], PkUnit &uB,
                                         cx<T> (&gB)[kPkLoads], const cx<T> *__restrict__ x,
                                         cx<T> *__restrict__ pw, int lane, int wave,
                                         cx<T> *__restrict__ out, long long xrows, int nq,
                                         cx<T> *__restrict__ keep) {
  const int n = wave < c.nunit ? (c.nunit - 1 - wave) / kPkWaves + 1 : 0;
  const PkUnit first = has_nx && wave < nx.nunit ? pk_unit(wave, nx) : uA;
  if (n == 0) {
    uA = first;
    pk_load<TB, T>(B, uA, lane, gA);
    return;
  }
  for (int i = 0; i < n; i += 2) {
    // load i + 1: a unit, or (n odd) a repeat of unit i
    if (i + 1 < n) uB = pk_unit(wave + (i + 1) * kPkWaves, c);
    else uB = uA;
    pk_load<TB, T>(B, uB, lane, gB);
    pk_compute<T, RC>(uA, gA, x, pw, c.nf, lane, out, xrows, nq, keep);
    // load i + 2: a unit or the next slab's first
    const PkUnit nb = i + 2 < n ? pk_unit(wave + (i + 2) * kPkWaves, c) : first;
    uA = nb;
    pk_load<TB, T>(B, uA, lane, gA);
    if (i + 1 < n) pk_compute<T, RC>(uB, gB, x, pw, c.nf, lane, out, xrows, nq, keep);
  }
}

// y[a] = sum of the wavefronts' partials for the rows of the full blocks,
// to out and (when given) keep
template <typename T, int RC>
__device__ __forceinline__ void pk_sum(const cx<T> *__restrict__ part, int nf, int stride,
                                       cx<T> *__restrict__ out, long long xrows, int nq,
                                       cx<T> *__restrict__ keep) {
  for (int a = threadIdx.x; a < 64 * nf; a += 64 * kPkWaves)
#pragma unroll
    for (int q = 0; q < RC; ++q) {
      cx<T> v = part[a * RC + q];
      for (int w = 1; w < kPkWaves; ++w) v = v + part[((long long)w * stride + a) * RC + q];
      if (q < nq) out[(long long)q * xrows + a] = v;
      if (keep) keep[a * RC + q] = v;
    }
}

// the coupling products of the staging, reading the neighbouring slab from
// LDS (kept: [row][RC] in slab-local order) instead of memory.  The lower one
// by items (first-layer node j, layer lb of slab t - 1): acc = the terms of
// A[t][t-1] y_{t-1} of row j from layer lb; the items of a row are summed
// afterwards, so that a thread has (2P+1)^(d-1) coefficient loads in flight
// rather than P times as many.
template <typename TB, typename T, int RC, int P, int DIM>
__device__ __forceinline__ void band_lower_item(const Sub &s, const cx<TB> *__restrict__ Ct,
                                                const cx<T> *__restrict__ src, long long qs,
                                                int rs, int qmax, int j, int lb,
                                                cx<T> (&acc)[RC]) {
  constexpr int W2 = 2 * P + 1;
  const int xa = j % s.nox, ya = DIM == 3 ? j / s.nox : 0;
  const cx<TB> *cr = Ct + j;
#pragma unroll
  for (int q = 0; q < RC; ++q) acc[q] = {0, 0};
#pragma unroll
  for (int jy = 0; jy < (DIM == 3 ? W2 : 1); ++jy) {
    const int yb = DIM == 3 ? min(max(ya - P + jy, 0), s.noy - 1) : 0;
    cx<TB> l[W2];
#pragma unroll
    for (int jx = 0; jx < W2; ++jx) l[jx] = cr[(long long)((jy * W2 + jx) * P + lb) * s.lsz];
#pragma unroll
    for (int jx = 0; jx < W2; ++jx) {
      const int xb = min(max(xa - P + jx, 0), s.nox - 1);
      const long long r = (long long)(lb * s.lsz + yb * s.nox + xb) * rs;
#pragma unroll
      for (int q = 0; q < RC; ++q) cmac(acc[q], ccast<T>(l[jx]), src[min(q, qmax) * qs + r]);
    }
  }
}

// w[j] -= (SUB) or += A[t][t-1] v_{t-1} for the first-layer rows j < lsz of
// slab t (the lower coupling); v_{t-1} entry (row r, right-hand side q) at
// src[q qs + r rs] (memory or LDS); by (row, layer) items whose sums go
// through bp (P lsz x RC entries of free LDS); ends with a barrier
template <bool SUB, typename TB, typename T, int RC, int P, int DIM>
__device__ __forceinline__ void band_lower_staged(const Sub &s, const cx<TB> *__restrict__ Ct,
                                                  const cx<T> *__restrict__ src, long long qs,
                                                  int rs, int qmax, cx<T> *__restrict__ bp,
                                                  cx<T> *__restrict__ w) {
  for (int i = threadIdx.x; i < P * s.lsz; i += 64 * kPkWaves) {
    const int lb = i / s.lsz, j = i - lb * s.lsz;
    cx<T> acc[RC];
    band_lower_item<TB, T, RC, P, DIM>(s, Ct, src, qs, rs, qmax, j, lb, acc);
#pragma unroll
    for (int q = 0; q < RC; ++q) bp[i * RC + q] = acc[q];
  }
  __syncthreads();
  for (int j = threadIdx.x; j < s.lsz; j += 64 * kPkWaves)
#pragma unroll
    for (int q = 0; q < RC; ++q) {
      cx<T> v = w[j * RC + q];
#pragma unroll
      for (int lb = 0; lb < P; ++lb)
        v = SUB ? v - bp[(lb * s.lsz + j) * RC + q] : v + bp[(lb * s.lsz + j) * RC + q];
      w[j * RC + q] = v;
    }
  __syncthreads();
}

// The upper coupling by items (row j of slab t, group g of the band
// positions: halves of the in-layer offsets in 2-D, every kUpGroups-th row
// offset in 3-D): acc = those terms of A[t][t+1] v_{t+1}[first layer] for
// row j, v entry (first-layer node a, right-hand side q) at
// src[q qs + a rs]; out-of-range positions meet a zero coefficient.
template <int P, int DIM>
constexpr int up_groups() {
  return DIM == 3 ? (2 * P + 1 < 4 ? 2 * P + 1 : 4) : 2;
}

template <typename TB, typename T, int RC, int P, int DIM>
__device__ __forceinline__ void band_upper_item(const Sub &s, const cx<TB> *__restrict__ Cn,
                                                const cx<T> *__restrict__ src, long long qs,
                                                int rs, int qmax, int j, int g,
                                                cx<T> (&acc)[RC]) {
  constexpr int W2 = 2 * P + 1, NG = up_groups<P, DIM>(), H = (W2 + 1) / 2;
  const int lb = j / s.lsz, jj = j - lb * s.lsz;
  const int xj = jj % s.nox, yj = DIM == 3 ? jj / s.nox : 0;
#pragma unroll
  for (int q = 0; q < RC; ++q) acc[q] = {0, 0};
#pragma unroll
  for (int jy0 = 0; jy0 < (DIM == 3 ? W2 : 1); jy0 += (DIM == 3 ? NG : 1)) {
    const int jy = DIM == 3 ? jy0 + g : 0;
    if (DIM == 3 && jy >= W2) break;
    const int ya = DIM == 3 ? yj - P + jy : 0;
    const bool iny = DIM == 3 ? (ya >= 0 && ya < s.noy) : true;
    const int yac = DIM == 3 ? min(max(ya, 0), s.noy - 1) : 0;
    constexpr int NX = DIM == 3 ? W2 : H;
    const int jx0 = DIM == 3 ? 0 : g * H;
    cx<TB> l[NX];
    int aa[NX];
#pragma unroll
    for (int i = 0; i < NX; ++i) {
      const int jx = min(jx0 + i, W2 - 1);
      const int xa = xj - P + jx;
      const int xac = min(max(xa, 0), s.nox - 1);
      aa[i] = yac * s.nox + xac;
      const int k = (((DIM == 3 ? 2 * P - jy : 0) * W2) + 2 * P - jx) * P + lb;
      l[i] = Cn[(long long)k * s.lsz + aa[i]];
      if (!(iny && xa >= 0 && xa < s.nox && jx0 + i < W2)) l[i] = cx<TB>{0, 0};
    }
#pragma unroll
    for (int i = 0; i < NX; ++i)
#pragma unroll
      for (int q = 0; q < RC; ++q)
        cmac(acc[q], ccast<T>(l[i]), src[min(q, qmax) * qs + (long long)aa[i] * rs]);
  }
}

// w[j] -= A[t][t+1] v_{t+1}[first layer] for the m rows of slab t, by items
// whose sums go through bp (up_groups m x RC entries of free LDS); ends
// with a barrier
template <typename TB, typename T, int RC, int P, int DIM>
__device__ __forceinline__ void band_upper_staged(const Sub &s, const cx<TB> *__restrict__ Cn,
                                                  const cx<T> *__restrict__ src, long long qs,
                                                  int rs, int qmax, int m, cx<T> *__restrict__ bp,
                                                  cx<T> *__restrict__ w) {
  constexpr int NG = up_groups<P, DIM>();
  for (int i = threadIdx.x; i < NG * m; i += 64 * kPkWaves) {
    const int g = i / m, j = i - g * m;
    cx<T> acc[RC];
    band_upper_item<TB, T, RC, P, DIM>(s, Cn, src, qs, rs, qmax, j, g, acc);
#pragma unroll
    for (int q = 0; q < RC; ++q) bp[i * RC + q] = acc[q];
  }
  __syncthreads();
  for (int j = threadIdx.x; j < m; j += 64 * kPkWaves)
#pragma unroll
    for (int q = 0; q < RC; ++q) {
      cx<T> v = w[j * RC + q];
#pragma unroll
      for (int g = 0; g < NG; ++g) v = v - bp[(g * m + j) * RC + q];
      w[j * RC + q] = v;
    }
  __syncthreads();
}

// w[j] -= (SUB) or += the sum of the items of row j in bp: the nl rows of
// one layer with items (row, layer) in layer-major order (ng = P), or the m
// rows of a slab with items (row, group) group-major (ng = up_groups)
template <bool SUB, typename T, int RC>
__device__ __forceinline__ void band_items_apply(int rows, int ng, const cx<T> *__restrict__ bp,
                                                 cx<T> *__restrict__ w) {
  for (int j = threadIdx.x; j < rows; j += 64 * kPkWaves)
#pragma unroll
    for (int q = 0; q < RC; ++q) {
      cx<T> v = w[j * RC + q];
      for (int g = 0; g < ng; ++g)
        v = SUB ? v - bp[(g * rows + j) * RC + q] : v + bp[(g * rows + j) * RC + q];
      w[j * RC + q] = v;
    }
}

template <typename TB, typename T, int RC, int P, int DIM>
__device__ __forceinline__ void band_upper_lds(const Sub &s, const cx<TB> *__restrict__ Cn,
                                               const cx<T> *__restrict__ kept, int j,
                                               cx<T> (&acc)[RC]) {
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
#pragma unroll
    for (int jx = 0; jx < W2; ++jx) {
      const int xa = xj - P + jx;
      const int xac = min(max(xa, 0), s.nox - 1);
      const int k = (((DIM == 3 ? 2 * P - jy : 0) * W2) + 2 * P - jx) * P + lb;
      l[jx] = Cn[(long long)k * s.lsz + yac * s.nox + xac];
      if (!(iny && xa >= 0 && xa < s.nox)) l[jx] = cx<TB>{0, 0};
    }
#pragma unroll
    for (int jx = 0; jx < W2; ++jx) {
      const int a = yac * s.nox + min(max(xj - P + jx, 0), s.nox - 1);
#pragma unroll
      for (int q = 0; q < RC; ++q) cmac(acc[q], ccast<T>(l[jx]), kept[a * RC + q]);
    }
  }
}

// Forward sweep of every chain (lower: slabs 0 .. M - 1, upper: nsl - 1 ..
// M + 1) in one launch.  LDS: the slab's right-hand sides [ldx][RC], the
// previous slab's y [ldx][RC], the partials [kPkWaves][ldx / 64][64][RC]
// (also the coupling items of the staging).
template <typename TB, typename T, int RC, int P, int DIM>
__global__ __launch_bounds__(64 * kPkWaves, RC == 1 ? 4 : 2) void k_slab_fwd_chain(
    const Sub *__restrict__ subs, const cx<TB> *__restrict__ B, const cx<T> *__restrict__ Z,
    cx<T> *__restrict__ V, long long xrows, int nrhs, int nsub, int ldx) {
  constexpr int W2 = 2 * P + 1, CB = (DIM == 3 ? W2 * W2 : W2) * P;
  extern __shared__ __align__(16) char slab_smem[];
  SweepItem it;
  if (!sweep_item(nsub, 2, it)) return;  // uniform
  const Sub s = subs[it.si];
  const int M = slab_mid(s);
  const bool upper = it.yb == 1;
  const int n = upper ? s.nsl - 1 - M : M;
  if (n == 0) return;  // uniform: a chain without slabs
  const int r0 = it.z * RC, nq = min(RC, nrhs - r0);
  const long long vq = (long long)r0 * xrows + s.xoff;
  const int lane = threadIdx.x % 64, wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
  const int pstride = (ldx / 64) * 64;
  cx<T> *x = (cx<T> *)slab_smem;
  cx<T> *kept = x + ldx * RC;
  cx<T> *part = kept + ldx * RC;
  cx<T> *pw = part + wave * pstride * RC;
  PkSlab c = pk_slab(s, upper ? s.nsl - 1 : 0, P);
  // (a wavefront without a unit of this slab loads one anyway: every buffer
  // always holds a unit of the store, see pk_units)
  PkUnit uA = pk_unit(min(wave, c.nunit - 1), c), uB;
  cx<T> gA[kPkLoads], gB[kPkLoads];
  pk_load<TB, T>(B, uA, lane, gA);
  for (int k = 0; k < n; ++k) {
    const int t = c.t;
    const long long row0 = (long long)t * P * s.lsz;
    // right-hand side of slab t: Z less the coupling to the previous slab of
    // the chain, by items (upper: (row, group) for every row; lower: (first-
    // layer row, layer)) whose sums go through bp = the partials' space; the
    // Z rows and the items' coefficients are loaded in one round
    constexpr int NG = up_groups<P, DIM>();
    const int nit = k == 0 ? 0 : (upper ? NG * c.m : P * s.lsz);
    const cx<TB> *Cb = B + s.coff + (long long)(upper ? t : t - 1) * s.lsz * CB;
    for (int i = threadIdx.x; i < max(c.m, nit); i += 64 * kPkWaves) {
      cx<T> zv[RC], acc[RC];
      const int iz = min(i, c.m - 1);
#pragma unroll
      for (int q = 0; q < RC; ++q) zv[q] = Z[vq + (long long)min(q, nq - 1) * xrows + row0 + iz];
      if (i < nit) {
        if (upper)
          band_upper_item<TB, T, RC, P, DIM>(s, Cb, kept, 1, RC, RC - 1, i % c.m, i / c.m, acc);
        else
          band_lower_item<TB, T, RC, P, DIM>(s, Cb, kept, 1, RC, RC - 1, i % s.lsz, i / s.lsz,
                                             acc);
#pragma unroll
        for (int q = 0; q < RC; ++q) part[i * RC + q] = acc[q];
      }
      if (i < c.m)
#pragma unroll
        for (int q = 0; q < RC; ++q) x[i * RC + q] = q < nq ? zv[q] : cx<T>{0, 0};
    }
    __syncthreads();
    if (nit) band_items_apply<true, T, RC>(upper ? c.m : s.lsz, upper ? NG : P, part, x);
    __syncthreads();  // x staged; kept (the previous y) and bp no longer read
    for (int e = lane; e < c.nf * 64 * RC; e += 64) pw[e] = cx<T>{0, 0};
    const bool has_nx = k + 1 < n;
    const PkSlab nx = has_nx ? pk_slab(s, upper ? t - 1 : t + 1, P) : c;
    cx<T> *out = V + vq + row0;
    pk_units<TB, T, RC>(B, c, nx, has_nx, uA, gA, uB, gB, x, pw, lane, wave, out, xrows, nq,
                        kept);
    __syncthreads();
    pk_sum<T, RC>(part, c.nf, pstride, out, xrows, nq, kept);
    __syncthreads();  // kept holds y_t; x and the partials free
    c = nx;
  }
}

// Forward step for the middles (both corrections, from y_{M-1} and y_{M+1}
// in memory), or, as a single step i < S, for one slab of each chain.  LDS:
// the slab's right-hand sides [m][RC], then the partials.
template <typename TB, typename T, int RC, int P, int DIM>
__global__ __launch_bounds__(64 * kPkWaves, RC == 1 ? 4 : 2) void k_slab_fwd_pk(
    const Sub *__restrict__ subs, const cx<TB> *__restrict__ B, const cx<T> *__restrict__ Z,
    cx<T> *__restrict__ V, long long xrows, int nrhs, int i, int S, int nsub) {
  constexpr int W2 = 2 * P + 1, CB = (DIM == 3 ? W2 * W2 : W2) * P;
  extern __shared__ __align__(16) char slab_smem[];
  SweepItem it;
  if (!sweep_item(nsub, i < S ? 2 : 1, it)) return;  // uniform
  const Sub s = subs[it.si];
  const int M = slab_mid(s), U = s.nsl - 1 - M;
  int t, lo, up;
  if (i == S) {
    t = M;
    lo = M >= 1;
    up = U >= 1;
  } else if (it.yb == 0) {
    t = i - (S - M);
    lo = t >= 1;
    up = 0;
  } else {
    const int j = i - (S - U);
    t = j >= 0 ? s.nsl - 1 - j : -1;
    lo = 0;
    up = j >= 1;
  }
  if (t < 0) return;  // uniform: no slab of this chain at this step
  const PkSlab c = pk_slab(s, t, P);
  const int r0 = it.z * RC, nq = min(RC, nrhs - r0);
  const long long row0 = (long long)t * P * s.lsz;
  const long long vq = (long long)r0 * xrows + s.xoff;
  const int lane = threadIdx.x % 64, wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
  cx<T> *x = (cx<T> *)slab_smem;
  cx<T> *part = x + c.m * RC;
  cx<T> *pw = part + wave * c.nf * 64 * RC;
  // (a wavefront without a unit of this slab loads one anyway: every buffer
  // always holds a unit of the store, see pk_units)
  PkUnit uA = pk_unit(min(wave, c.nunit - 1), c), uB;
  cx<T> gA[kPkLoads], gB[kPkLoads];
  pk_load<TB, T>(B, uA, lane, gA);
  for (int j = threadIdx.x; j < c.m; j += 64 * kPkWaves) {
    cx<T> v[RC];
#pragma unroll
    for (int q = 0; q < RC; ++q)
      v[q] = q < nq ? Z[vq + (long long)q * xrows + row0 + j] : cx<T>{0, 0};
    if (up) {
      cx<T> w[RC];
      band_upper<TB, T, RC, P, DIM>(s, B + s.coff + (long long)t * s.lsz * CB, V,
                                    vq + (long long)(t + 1) * P * s.lsz, xrows, nq, j, w);
#pragma unroll
      for (int q = 0; q < RC; ++q) v[q] = v[q] - w[q];
    }
#pragma unroll
    for (int q = 0; q < RC; ++q) x[j * RC + q] = v[q];
  }
  if (lo)
    band_lower_staged<true, TB, T, RC, P, DIM>(s, B + s.coff + (long long)(t - 1) * s.lsz * CB,
                                               V + vq + (long long)(t - 1) * P * s.lsz, xrows, 1,
                                               nq - 1, part, x);
  for (int e = lane; e < c.nf * 64 * RC; e += 64) pw[e] = cx<T>{0, 0};
  __syncthreads();
  cx<T> *out = V + vq + row0;
  pk_units<TB, T, RC>(B, c, c, false, uA, gA, uB, gB, x, pw, lane, wave, out, xrows, nq, nullptr);
  __syncthreads();
  pk_sum<T, RC>(part, c.nf, c.nf * 64, out, xrows, nq, nullptr);
}

// Backward sweep of every chain in one launch (lower: slabs M - 1 .. 0,
// x_t = y_t - E_t w with w = x_{t+1} on the first layer of slab t + 1; upper:
// slabs M + 1 .. nsl - 1, x_t = y_t - G_t[:, first layer] w with
// w = A[t][t-1] x_{t-1}); x_M and y_t in memory, each x_t written there and
// kept in LDS for the next slab.  The rows of the stored E_t^T (G_t[:, first
// layer]^T) are split in units of kPkBwdRows rows of one 64-row block, the
// next unit's loads issued before the current one is used (across slabs as
// well).  LDS: w [ldx][RC], the previous slab's x [ldx][RC], the partials
// [kPkWaves][ceil(ldx / 64) 64][RC].
struct BwdSlab {
  int t, m, nrb, nch, nunit, ld;
  long long g0;
};
__device__ __forceinline__ BwdSlab bwd_slab(const Sub &s, int t, int P, bool upper) {
  BwdSlab c;
  c.t = t;
  c.m = slab_rows(s, t, P);
  c.ld = slab_ld(c.m);
  c.nrb = (c.m + 63) / 64;
  c.nch = (s.lsz + kPkBwdRows - 1) / kPkBwdRows;
  c.nunit = c.nrb * c.nch;
  c.g0 = upper ? s.ecoff + (long long)t * s.lsz * slab_ld(P * s.lsz)
               : s.ecoff + (long long)t * s.lsz * c.ld;
  return c;
}

// the kPkBwdRows row loads of unit u, none predicated (rows past n_layer
// repeat the last; lanes past m read the row's first entry: their sums
// belong to no row)
template <typename TB, typename T>
__device__ __forceinline__ void bwd_load(const cx<TB> *__restrict__ B, const BwdSlab &c, int u,
                                         int nl, int lane, cx<T> (&gv)[kPkBwdRows]) {
  const int rb = u / c.nch, c0 = (u % c.nch) * kPkBwdRows, a = 64 * rb + lane;
  const cx<TB> *p = B + c.g0 + (a < c.m ? a : 0);
#pragma unroll
  for (int q = 0; q < kPkBwdRows; ++q)
    gv[q] = ccast<T>(ld_stream(p + (long long)min(c0 + q, nl - 1) * c.ld));
}

// partials of unit u: the rows c0 .. c0 + kPkBwdRows - 1 of one 64-row block
template <typename T, int RC>
__device__ __forceinline__ void bwd_compute(const BwdSlab &c, int u, int nl, int lane,
                                            const cx<T> (&gv)[kPkBwdRows],
                                            const cx<T> *__restrict__ w, cx<T> *__restrict__ pw) {
  const int rb = u / c.nch, c0 = (u % c.nch) * kPkBwdRows;
  cx<T> acc[RC];
#pragma unroll
  for (int q = 0; q < RC; ++q) acc[q] = cx<T>{0, 0};
#pragma unroll
  for (int h = 0; h < kPkBwdRows; ++h)
    if (c0 + h < nl)
#pragma unroll
      for (int q = 0; q < RC; ++q) cmac(acc[q], gv[h], w[(c0 + h) * RC + q]);
#pragma unroll
  for (int q = 0; q < RC; ++q) {
    cx<T> &p = pw[(64 * rb + lane) * RC + q];
    p = p + acc[q];
  }
}

// the backward counterpart of pk_units (a unit is its index in slab c, or
// in slab nx for the next slab's first)
template <typename TB, typename T, int RC>
__device__ __forceinline__ void bwd_units(const cx<TB> *__restrict__ B, const BwdSlab &c,
                                          const BwdSlab &nx, bool has_nx,
                                          cx<T> (&gA)[kPkBwdRows], cx<T> (&gB)[kPkBwdRows],
                                          const cx<T> *__restrict__ w, cx<T> *__restrict__ pw,
                                          int nl, int lane, int wave) {
  const int n = wave < c.nunit ? (c.nunit - 1 - wave) / kPkWaves + 1 : 0;
  const bool nx_unit = has_nx && wave < nx.nunit;
  // the next slab's first unit, or a repeat of this slab's first
  const BwdSlab &fs = nx_unit ? nx : c;
  const int fu = nx_unit ? wave : min(wave, c.nunit - 1);
  if (n == 0) {
    bwd_load<TB, T>(B, fs, fu, nl, lane, gA);
    return;
  }
  for (int i = 0; i < n; i += 2) {
    const int ua = wave + i * kPkWaves;
    const int ub = i + 1 < n ? ua + kPkWaves : ua;
    bwd_load<TB, T>(B, c, ub, nl, lane, gB);
    bwd_compute<T, RC>(c, ua, nl, lane, gA, w, pw);
    if (i + 2 < n)
      bwd_load<TB, T>(B, c, ua + 2 * kPkWaves, nl, lane, gA);
    else
      bwd_load<TB, T>(B, fs, fu, nl, lane, gA);
    if (i + 1 < n) bwd_compute<T, RC>(c, ub, nl, lane, gB, w, pw);
  }
}

template <typename TB, typename T, int RC, int P, int DIM>
__global__ __launch_bounds__(64 * kPkWaves, RC == 1 ? 4 : 2) void k_slab_bwd_chain(
    const Sub *__restrict__ subs, const cx<TB> *__restrict__ B, cx<T> *__restrict__ V,
    long long xrows, int nrhs, int nsub, int ldx) {
  constexpr int W2 = 2 * P + 1, CB = (DIM == 3 ? W2 * W2 : W2) * P;
  extern __shared__ __align__(16) char slab_smem[];
  SweepItem it;
  if (!sweep_item(nsub, 2, it)) return;  // uniform
  const Sub s = subs[it.si];
  const int M = slab_mid(s), nl = s.lsz;
  const bool upper = it.yb == 1;
  const int n = upper ? s.nsl - 1 - M : M;
  if (n == 0) return;  // uniform
  const int r0 = it.z * RC, nq = min(RC, nrhs - r0);
  const long long vq = (long long)r0 * xrows + s.xoff;
  const int lane = threadIdx.x % 64, wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
  const int pstride = ((ldx + 63) / 64) * 64;
  cx<T> *w = (cx<T> *)slab_smem;
  cx<T> *kept = w + ldx * RC;
  cx<T> *part = kept + ldx * RC;
  cx<T> *pw = part + wave * pstride * RC;
  BwdSlab c = bwd_slab(s, upper ? M + 1 : M - 1, P, upper);
  cx<T> gA[kPkBwdRows], gB[kPkBwdRows];
  bwd_load<TB, T>(B, c, min(wave, c.nunit - 1), nl, lane, gA);
  for (int k = 0; k < n; ++k) {
    const int t = c.t;
    const long long row0 = (long long)t * P * s.lsz;
    // w: lower, x_{t+1} on the first layer of slab t + 1; upper, the coupling
    // A[t][t-1] x_{t-1} (by items); x_M in memory, later slabs in kept
    if (upper) {
      // items (first-layer row, layer) of the coupling into bp, then their sums
      const cx<TB> *Ct = B + s.coff + (long long)(t - 1) * s.lsz * CB;
      const cx<T> *src = k > 0 ? kept : V + vq + (long long)(t - 1) * P * s.lsz;
      const long long qs = k > 0 ? 1 : xrows;
      const int rs = k > 0 ? RC : 1, qmax = k > 0 ? RC - 1 : nq - 1;
      for (int i = threadIdx.x; i < P * nl; i += 64 * kPkWaves) {
        cx<T> acc[RC];
        band_lower_item<TB, T, RC, P, DIM>(s, Ct, src, qs, rs, qmax, i % nl, i / nl, acc);
#pragma unroll
        for (int q = 0; q < RC; ++q) part[i * RC + q] = acc[q];
      }
      for (int j = threadIdx.x; j < nl; j += 64 * kPkWaves)
#pragma unroll
        for (int q = 0; q < RC; ++q) w[j * RC + q] = cx<T>{0, 0};
      __syncthreads();
      band_items_apply<false, T, RC>(nl, P, part, w);
    } else {
      for (int j = threadIdx.x; j < nl; j += 64 * kPkWaves)
#pragma unroll
        for (int q = 0; q < RC; ++q)
          w[j * RC + q] = k > 0    ? kept[j * RC + q]
                          : q < nq ? V[vq + (long long)q * xrows + (long long)(t + 1) * P * s.lsz + j]
                                   : cx<T>{0, 0};
    }
    __syncthreads();  // w staged; kept (the previous x) and bp no longer read
    for (int e = lane; e < c.nrb * 64 * RC; e += 64) pw[e] = cx<T>{0, 0};
    const bool has_nx = k + 1 < n;
    const BwdSlab nx = has_nx ? bwd_slab(s, upper ? t + 1 : t - 1, P, upper) : c;
    bwd_units<TB, T, RC>(B, c, nx, has_nx, gA, gB, w, pw, nl, lane, wave);
    // y_t of the (at most two) rows this thread finishes, loaded while the
    // other wavefronts finish their units
    static_assert(kPkMaxRows <= 2 * 64 * kPkWaves, "two rows per thread");
    cx<T> yv[2][RC];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int a = threadIdx.x + h * 64 * kPkWaves;
#pragma unroll
      for (int q = 0; q < RC; ++q)
        yv[h][q] = a < c.m && q < nq ? V[vq + (long long)q * xrows + row0 + a] : cx<T>{0, 0};
    }
    __syncthreads();
    // x_t = y_t - the sum of the partials, to memory and kept
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int a = threadIdx.x + h * 64 * kPkWaves;
      if (a < c.m)
#pragma unroll
        for (int q = 0; q < RC; ++q) {
          cx<T> v = part[a * RC + q];
          for (int ww = 1; ww < kPkWaves; ++ww)
            v = v + part[((long long)ww * pstride + a) * RC + q];
          const cx<T> xv = yv[h][q] - v;
          if (q < nq) V[vq + (long long)q * xrows + row0 + a] = xv;
          kept[a * RC + q] = xv;
        }
    }
    __syncthreads();  // kept holds x_t; w and the partials free
    c = nx;
  }
}

// LDS bytes of the packed sweeps for `rhs_bytes` bytes of right-hand sides
// per row: the slab's right-hand sides (w), the previous slab's result and
// every wavefront's partials of the slab's 64-row blocks
size_t slab_pk_lds(const th_ctx *c, size_t rhs_bytes) {
  const size_t m = (size_t)c->max_slab_rows;
  return (2 * m + (size_t)kPkWaves * 64 * ((m + 63) / 64)) * rhs_bytes;
}
int slab_pk_max_rows() { return kPkMaxRows; }

// both chains' forward sweeps, the middles, both chains' backward sweeps
template <typename TB, typename T, int RC, int P, int DIM>
static int pk_sweeps_pd(const th_ctx *c, int nrhs, hipStream_t s) {
  const unsigned nsub = (unsigned)c->subs.size();
  const int ldx = c->max_slab_rows;
  const unsigned nz = (unsigned)ceil_div(nrhs, RC);
  const cx<TB> *B = (const cx<TB> *)c->d_B;
  const unsigned groups8 = 8 * (unsigned)ceil_div((int)nsub, 8);  // XCD-aware 1-D grids
  const size_t shm = slab_pk_lds(c, RC * sizeof(cx<T>));
  const dim3 chains(groups8 * 2 * nz), block(64 * kPkWaves);
  hipLaunchKernelGGL((k_slab_fwd_chain<TB, T, RC, P, DIM>), chains, block, shm, s, c->d_subs, B,
                     (const cx<T> *)c->w_x, (cx<T> *)c->w_z, c->x_rows, nrhs, (int)nsub, ldx);
  hipLaunchKernelGGL((k_slab_fwd_pk<TB, T, RC, P, DIM>), dim3(groups8 * nz), block, shm, s,
                     c->d_subs, B, (const cx<T> *)c->w_x, (cx<T> *)c->w_z, c->x_rows, nrhs, 0, 0,
                     (int)nsub);
  hipLaunchKernelGGL((k_slab_bwd_chain<TB, T, RC, P, DIM>), chains, block, shm, s, c->d_subs, B,
                     (cx<T> *)c->w_z, c->x_rows, nrhs, (int)nsub, ldx);
  TH_HIP_CHECK_RET(hipGetLastError());
  return 0;
}

template <typename TB, typename T, int RC>
static int pk_sweeps_rc(const th_ctx *c, int nrhs, hipStream_t s) {
  if (c->dim == 3) {
    if (c->P == 2) return pk_sweeps_pd<TB, T, RC, 2, 3>(c, nrhs, s);
    if (c->P == 4) return pk_sweeps_pd<TB, T, RC, 4, 3>(c, nrhs, s);
  } else {
    switch (c->P) {
      case 2: return pk_sweeps_pd<TB, T, RC, 2, 2>(c, nrhs, s);
      case 4: return pk_sweeps_pd<TB, T, RC, 4, 2>(c, nrhs, s);
      case 6: return pk_sweeps_pd<TB, T, RC, 6, 2>(c, nrhs, s);
      case 8: return pk_sweeps_pd<TB, T, RC, 8, 2>(c, nrhs, s);
    }
  }
  set_error("unsupported order for the slab layout");
  return TH_EUNSUPPORTED;
}

template <typename TB, typename T>
int slab_pk_sweeps(const th_ctx *c, int nrhs, int rc, hipStream_t s) {
  if (rc == 4) return pk_sweeps_rc<TB, T, 4>(c, nrhs, s);
  if (rc == 2) return pk_sweeps_rc<TB, T, 2>(c, nrhs, s);
  return pk_sweeps_rc<TB, T, 1>(c, nrhs, s);
}

template int slab_pk_sweeps<double, double>(const th_ctx *, int, int, hipStream_t);
template int slab_pk_sweeps<double, float>(const th_ctx *, int, int, hipStream_t);
template int slab_pk_sweeps<float, double>(const th_ctx *, int, int, hipStream_t);
template int slab_pk_sweeps<float, float>(const th_ctx *, int, int, hipStream_t);

}  // namespace th
