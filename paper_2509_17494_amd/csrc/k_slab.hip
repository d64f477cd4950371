// Slab-factor layout of the subdomain solves (Alg. 2, w_i = (A_s^(i))^{-1} R_i r).
//
// In its Omega-local numbering (x fastest, slowest axis y in 2-D, z in 3-D)
// A_s^(i) couples node layers only through shared cells, so grouping the
// layers of one cell row into a slab (P layers; the last slab also takes the
// top layer) makes it block tridiagonal: slab t couples to slab t - 1 only
// through its first layer (A[t][t-1] is zero outside the first-layer rows,
// and A[t-1][t] = A[t][t-1]^T since A_s^(i) is complex symmetric).
//
// The block elimination is twisted: with the middle slab M = (n - 1) / 2 of
// the n slabs, the lower chain 0 .. M - 1 is eliminated upwards and the upper
// chain n - 1 .. M + 1 downwards, both at once, and they meet in M:
//   lower   S_0 = T_0,          S_t = T_t - A[t][t-1] G_{t-1} A[t-1][t]
//           (first-layer block only)
//   upper   S_{n-1} = T_{n-1},  S_t = T_t - A[t][t+1] G_{t+1} A[t+1][t]
//           (A[t][t+1] has nonzero columns only on the first layer of t + 1,
//           so only G_{t+1} restricted to that layer enters; a full update)
//   middle  both corrections;   G_t = S_t^{-1} everywhere.
// The apply is
//   forward   y_t = G_t (r_t - A[t][t-1] y_{t-1})        lower chain
//             y_t = G_t (r_t - A[t][t+1] y_{t+1})        upper chain
//             y_M = G_M (r_M - both terms),  x_M = y_M
//   backward  x_t = y_t - E_t x_{t+1}[first layer],  E_t = G_t A[t][t+1]   (lower)
//             x_t = y_t - G_t[:, first layer] (A[t][t-1] x_{t-1})         (upper)
// with one launch per step for all subdomains and both chains: about n + 1
// launches instead of 2n - 1 for the one-sided elimination.  The chains of
// all subdomains are aligned so that they reach their middles at the same step.
// With G_t stored packed (each symmetric G_t once, k_slab_pk.hip) the sweeps
// take three launches instead: every chain's forward sweep, the middles, every
// chain's backward sweep.
//
// Stored per subdomain: every G_t transposed (entry (b, a) at b ld_t + a, rows
// padded to ld_t, a multiple of 8 entries, so one output row per thread reads
// consecutive entries of a row and every row starts on a 128-byte line); the
// couplings A[t][t-1] of every slab t >= 1 as bands: for each first-layer node
// a the (2P+1)^(d-1) x P block of slab t - 1 nodes within P positions of a in
// every in-layer direction (zero where a node lies outside Omega or shares no
// cell with a), stored entry-major (entry k of node a at k n_layer + a, so
// that neighbouring nodes read neighbouring entries), read directly by the
// lower chain and transposed by the upper one; and the E_t of the lower chain (m_t x n_layer, the product the
// elimination forms anyway) transposed, likewise padded.  The upper chain's
// backward step reads the first n_layer rows of the stored G_t^T (G_t is
// symmetric); with packed G_t those rows are stored apart, beside the E_t.  The bytes per application are the G_t plus a fraction 1/P of
// them, instead of the n_U x n_Omega rows of an explicit inverse.
//
// Elimination without pivoting is stable here for the reason given for the
// Gauss-Jordan inverses: i A_s^(i) has a positive definite Hermitian part,
// which every Schur complement keeps (Dirichlet nodes are decoupled unit
// rows).  The blocks of the upper chain, whose correction is largest on their
// top layers, are inverted in reversed node order, so that Gauss-Jordan meets
// the corrected rows first, as it does in the lower chain.
#include <algorithm>

#include "k_slab.hpp"

namespace th {

// ---------------------------------------------------------------------------
// setup (FP64), batched over subdomains s0 .. s0 + gridDim.z - 1; every
// kernel resolves the slab of its subdomain from (mode, i, n)

// W = the diagonal block T_t of A (rows and columns of slab t, reversed for
// the upper chain), identity padding; identity where the subdomain has no
// slab at this step.
__global__ __launch_bounds__(256) void k_slab_copy(const Sub *__restrict__ subs, int s0,
                                                   const c64 *__restrict__ A, int lda,
                                                   long long amat, c64 *__restrict__ W, int ldw,
                                                   long long wmat, int mode, int i, int n, int P) {
  const Sub s = subs[s0 + blockIdx.z];
  const SlabRole r = slab_role(s, mode, i, n);
  const long long e = blockIdx.x * 256LL + threadIdx.x;
  if (e >= (long long)ldw * ldw) return;
  const int a = (int)(e / ldw), b = (int)(e % ldw);
  c64 v = a == b ? c64{1.0, 0.0} : c64{0, 0};
  if (r.on) {
    const int m = slab_rows(s, r.t, P);
    const long long r0 = (long long)r.t * P * s.lsz;
    if (a < m && b < m) {
      const int ia = r.rev ? m - 1 - a : a, ib = r.rev ? m - 1 - b : b;
      v = A[blockIdx.z * amat + (r0 + ia) * lda + r0 + ib];
    }
  }
  W[blockIdx.z * wmat + e] = v;
}

// lower correction, first factor: T1 = G_{t-1} A[t-1][first layer of t]
// (m_{t-1} x lsz), G_{t-1} in natural order in Gp
__global__ __launch_bounds__(256) void k_slab_t1(const Sub *__restrict__ subs, int s0,
                                                 const c64 *__restrict__ A, int lda,
                                                 long long amat, const c64 *__restrict__ Gp,
                                                 int ldw, long long wmat, c64 *__restrict__ T1,
                                                 int ldt, long long tmat, int mode, int i, int n,
                                                 int P) {
  const Sub s = subs[s0 + blockIdx.z];
  const SlabRole sr = slab_role(s, mode, i, n);
  if (!sr.on || !sr.lo) return;
  const int mp = P * s.lsz;
  const long long e = blockIdx.x * 256LL + threadIdx.x;
  if (e >= (long long)mp * s.lsz) return;
  const int r = (int)(e / s.lsz), c = (int)(e % s.lsz);
  const long long rp = (long long)(sr.t - 1) * P * s.lsz, r0 = (long long)sr.t * P * s.lsz;
  const c64 *g = Gp + blockIdx.z * wmat + (long long)r * ldw;
  const c64 *u = A + blockIdx.z * amat + rp * lda + r0 + c;
  c64 acc = {0, 0};
  for (int k = 0; k < mp; ++k) cmac(acc, g[k], u[(long long)k * lda]);
  T1[blockIdx.z * tmat + (long long)r * ldt + c] = acc;
}

// lower correction of the first-layer block of S_t (natural order):
// W[a][a'] -= sum_k A[first layer a][slab t - 1, k] T1[k][a']
__global__ __launch_bounds__(256) void k_slab_schur(const Sub *__restrict__ subs, int s0,
                                                    const c64 *__restrict__ A, int lda,
                                                    long long amat, const c64 *__restrict__ T1,
                                                    int ldt, long long tmat, c64 *__restrict__ W,
                                                    int ldw, long long wmat, int mode, int i,
                                                    int n, int P) {
  const Sub s = subs[s0 + blockIdx.z];
  const SlabRole sr = slab_role(s, mode, i, n);
  if (!sr.on || !sr.lo) return;
  const long long e = blockIdx.x * 256LL + threadIdx.x;
  if (e >= (long long)s.lsz * s.lsz) return;
  const int a = (int)(e / s.lsz), a2 = (int)(e % s.lsz);
  const int mp = P * s.lsz;
  const long long rp = (long long)(sr.t - 1) * P * s.lsz, r0 = (long long)sr.t * P * s.lsz;
  const c64 *l = A + blockIdx.z * amat + (r0 + a) * lda + rp;
  const c64 *t1 = T1 + blockIdx.z * tmat + a2;
  c64 acc = {0, 0};
  for (int k = 0; k < mp; ++k) cmac(acc, l[k], t1[(long long)k * ldt]);
  c64 &w = W[blockIdx.z * wmat + (long long)a * ldw + a2];
  w = w - acc;
}

// upper correction, first factor: T1 = A[t][first layer of t + 1] G_{t+1}
// restricted to that layer (m_t x lsz); G_{t+1} in reversed order in Gn
__global__ __launch_bounds__(256) void k_slab_t1_up(const Sub *__restrict__ subs, int s0,
                                                    const c64 *__restrict__ A, int lda,
                                                    long long amat, const c64 *__restrict__ Gn,
                                                    int ldw, long long wmat,
                                                    c64 *__restrict__ T1, int ldt, long long tmat,
                                                    int mode, int i, int n, int P) {
  const Sub s = subs[s0 + blockIdx.z];
  const SlabRole sr = slab_role(s, mode, i, n);
  if (!sr.on || !sr.up) return;
  const int m = P * s.lsz, mn = slab_rows(s, sr.t + 1, P);
  const long long e = blockIdx.x * 256LL + threadIdx.x;
  if (e >= (long long)m * s.lsz) return;
  const int r = (int)(e / s.lsz), c = (int)(e % s.lsz);
  const long long r0 = (long long)sr.t * P * s.lsz, rn = (long long)(sr.t + 1) * P * s.lsz;
  const c64 *u = A + blockIdx.z * amat + (r0 + r) * lda + rn;
  const c64 *g = Gn + blockIdx.z * wmat + (mn - 1 - c);
  c64 acc = {0, 0};
  for (int k = 0; k < s.lsz; ++k) cmac(acc, u[k], g[(long long)(mn - 1 - k) * ldw]);
  T1[blockIdx.z * tmat + (long long)r * ldt + c] = acc;
}

// upper correction of the whole block (reversed order when rev):
// W[p][q] -= sum_k T1[row of p][k] A[row of q][first layer of t + 1, k]
__global__ __launch_bounds__(256) void k_slab_schur_up(const Sub *__restrict__ subs, int s0,
                                                       const c64 *__restrict__ A, int lda,
                                                       long long amat, const c64 *__restrict__ T1,
                                                       int ldt, long long tmat,
                                                       c64 *__restrict__ W, int ldw,
                                                       long long wmat, int mode, int i, int n,
                                                       int P) {
  const Sub s = subs[s0 + blockIdx.z];
  const SlabRole sr = slab_role(s, mode, i, n);
  if (!sr.on || !sr.up) return;
  const int m = P * s.lsz;
  const long long e = blockIdx.x * 256LL + threadIdx.x;
  if (e >= (long long)m * m) return;
  const int p = (int)(e / m), q = (int)(e % m);
  const int rp = sr.rev ? m - 1 - p : p, rq = sr.rev ? m - 1 - q : q;
  const long long r0 = (long long)sr.t * P * s.lsz, rn = (long long)(sr.t + 1) * P * s.lsz;
  const c64 *t1 = T1 + blockIdx.z * tmat + (long long)rp * ldt;
  const c64 *u = A + blockIdx.z * amat + (r0 + rq) * lda + rn;
  c64 acc = {0, 0};
  for (int k = 0; k < s.lsz; ++k) cmac(acc, t1[k], u[k]);
  c64 &w = W[blockIdx.z * wmat + (long long)p * ldw + q];
  w = w - acc;
}

// store G_t (W, reversed when rev) transposed with rows padded to slab_ld,
// or packed (pk); with pk, the upper chain also stores G_t[:, first layer]
// transposed (n_layer rows of slab_ld(m) entries) in the backward region,
// which its backward step reads; for t >= 1, the coupling band of slab t
template <typename TB>
__global__ __launch_bounds__(256) void k_slab_store(const Sub *__restrict__ subs, int s0,
                                                    const c64 *__restrict__ A, int lda,
                                                    long long amat, const c64 *__restrict__ W,
                                                    int ldw, long long wmat,
                                                    cx<TB> *__restrict__ B, int mode, int i, int n,
                                                    int P, int dim, int pk) {
  const Sub s = subs[s0 + blockIdx.z];
  const SlabRole sr = slab_role(s, mode, i, n);
  if (!sr.on) return;
  const int t = sr.t;
  const int m = slab_rows(s, t, P);
  long long e = blockIdx.x * 256LL + threadIdx.x;
  const c64 *w = W + blockIdx.z * wmat;
  // G_t[a][b] in natural order
  auto g = [&](int a, int b) {
    const int wa = sr.rev ? m - 1 - a : a, wb = sr.rev ? m - 1 - b : b;
    const c64 v = w[(long long)wa * ldw + wb];
    return cx<TB>{(TB)v.re, (TB)v.im};
  };
  const int cb = band_width(P, dim);
  if (pk) {
    const int nf = m / 64;
    const long long nt = 64 * pk_tile_steps(nf), ng = pk_elems(m);
    if (e < nt) {
      int R, C, k;
      pk_step(nf, e / 64, R, C, k);
      const int l = (int)(e % 64);
      B[pk_goff(s, t, P) + e] = g(64 * R + ((l + k) & 63), 64 * C + l);
      return;
    }
    if (e < ng) {
      const long long f = e - nt;
      const int j = (int)(f / slab_ld(m)), b = (int)(f % slab_ld(m));
      B[pk_goff(s, t, P) + e] = b < m ? g(64 * nf + j, b) : cx<TB>{0, 0};
      return;
    }
    e -= ng;
    const long long nfl = mode == kUpperChain ? (long long)s.lsz * m : 0;
    if (e < nfl) {
      const int c = (int)(e / m), a = (int)(e % m);
      const long long off = s.ecoff + (long long)t * s.lsz * slab_ld(P * s.lsz);
      B[off + (long long)c * slab_ld(m) + a] = g(a, c);
      return;
    }
    e -= nfl;
  } else {
    const long long ng = (long long)m * m;
    if (e < ng) {
      const int b = (int)(e / m), a = (int)(e % m);
      B[slab_goff(s, t, P) + (long long)b * slab_ld(m) + a] = g(a, b);
      return;
    }
    e -= ng;
  }
  if (t >= 1 && e < (long long)s.lsz * cb) {
    const long long f = e;
    const int a = (int)(f / cb), k = (int)(f % cb);
    const int col = band_col(s, t, a, k, P, dim);
    const long long r0 = (long long)t * P * s.lsz;
    c64 v = {0, 0};
    if (col >= 0) v = A[blockIdx.z * amat + (r0 + a) * lda + col];
    B[s.coff + (long long)(t - 1) * s.lsz * cb + (long long)k * s.lsz + a] =
        cx<TB>{(TB)v.re, (TB)v.im};
  }
}

// store E_{t-1} = T1 of the lower correction (rows of slab t - 1, columns:
// first layer of slab t) transposed
template <typename TB>
__global__ __launch_bounds__(256) void k_slab_store_e(const Sub *__restrict__ subs, int s0,
                                                      const c64 *__restrict__ T1, int ldt,
                                                      long long tmat, cx<TB> *__restrict__ B,
                                                      int mode, int i, int n, int P) {
  const Sub s = subs[s0 + blockIdx.z];
  const SlabRole sr = slab_role(s, mode, i, n);
  if (!sr.on || !sr.lo) return;
  const int mp = P * s.lsz;
  const long long e = blockIdx.x * 256LL + threadIdx.x;
  if (e >= (long long)s.lsz * mp) return;
  const int cc = (int)(e / mp), r = (int)(e % mp);
  const c64 v = T1[blockIdx.z * tmat + (long long)r * ldt + cc];
  B[s.ecoff + ((long long)(sr.t - 1) * s.lsz + cc) * slab_ld(mp) + r] =
      cx<TB>{(TB)v.re, (TB)v.im};
}

// One step of the twisted elimination for every subdomain of the batch: the
// block in W, its corrections from the lower neighbour's inverse in Wlo and
// the upper neighbour's in Wup (null: none at this step), inversion, store.
static int slab_setup_step(th_ctx *c, int s0, int nb, const c64 *A, int npad, long long amat,
                           c64 *W, const c64 *Wlo, const c64 *Wup, c64 *T1, int ldw, int ldt,
                           int max_lsz, int max_m, c64 *pws, int mode, int i, int n,
                           hipStream_t s) {
  const int P = c->P;
  const long long wmat = (long long)ldw * ldw, tmat = (long long)ldw * ldt;
  const long long ml = (long long)P * max_lsz;
  const bool f32 = c->desc.gemm == TH_GEMM_F32;
  hipLaunchKernelGGL(k_slab_copy, dim3((unsigned)ceil_div_ll(wmat, 256), 1, nb), dim3(256), 0, s,
                     c->d_subs, s0, A, npad, amat, W, ldw, wmat, mode, i, n, P);
  if (Wlo) {
    hipLaunchKernelGGL(k_slab_t1, dim3((unsigned)ceil_div_ll(ml * max_lsz, 256), 1, nb),
                       dim3(256), 0, s, c->d_subs, s0, A, npad, amat, Wlo, ldw, wmat, T1, ldt,
                       tmat, mode, i, n, P);
    hipLaunchKernelGGL(k_slab_schur, dim3((unsigned)ceil_div_ll((long long)max_lsz * max_lsz, 256),
                                          1, nb),
                       dim3(256), 0, s, c->d_subs, s0, A, npad, amat, (const c64 *)T1, ldt, tmat,
                       W, ldw, wmat, mode, i, n, P);
    const dim3 ge((unsigned)ceil_div_ll(ml * max_lsz, 256), 1, nb);
    if (f32)
      hipLaunchKernelGGL((k_slab_store_e<float>), ge, dim3(256), 0, s, c->d_subs, s0,
                         (const c64 *)T1, ldt, tmat, (cx<float> *)c->d_B, mode, i, n, P);
    else
      hipLaunchKernelGGL((k_slab_store_e<double>), ge, dim3(256), 0, s, c->d_subs, s0,
                         (const c64 *)T1, ldt, tmat, (cx<double> *)c->d_B, mode, i, n, P);
  }
  if (Wup) {
    hipLaunchKernelGGL(k_slab_t1_up, dim3((unsigned)ceil_div_ll(ml * max_lsz, 256), 1, nb),
                       dim3(256), 0, s, c->d_subs, s0, A, npad, amat, Wup, ldw, wmat, T1, ldt,
                       tmat, mode, i, n, P);
    hipLaunchKernelGGL(k_slab_schur_up, dim3((unsigned)ceil_div_ll(ml * ml, 256), 1, nb),
                       dim3(256), 0, s, c->d_subs, s0, A, npad, amat, (const c64 *)T1, ldt, tmat,
                       W, ldw, wmat, mode, i, n, P);
  }
  TH_HIP_CHECK_RET(hipGetLastError());
  int rc = gj_invert_batched(W, ldw, ldw, wmat, nb, s, pws);
  if (rc) return rc;
  // G_t (whole or packed), G_t[:, first layer] (packed, upper chain), band
  const long long nst = (long long)max_m * slab_ld(max_m) + (long long)max_lsz * max_m +
                        (long long)max_lsz * band_width(P, c->dim);
  if (f32)
    hipLaunchKernelGGL((k_slab_store<float>), dim3((unsigned)ceil_div_ll(nst, 256), 1, nb),
                       dim3(256), 0, s, c->d_subs, s0, A, npad, amat, (const c64 *)W, ldw, wmat,
                       (cx<float> *)c->d_B, mode, i, n, P, c->dim, c->slab_pk);
  else
    hipLaunchKernelGGL((k_slab_store<double>), dim3((unsigned)ceil_div_ll(nst, 256), 1, nb),
                       dim3(256), 0, s, c->d_subs, s0, A, npad, amat, (const c64 *)W, ldw, wmat,
                       (cx<double> *)c->d_B, mode, i, n, P, c->dim, c->slab_pk);
  TH_HIP_CHECK_RET(hipGetLastError());
  return 0;
}

// The lower chain in buffers W[0] / W[1], the upper chain in the two buffers
// its last inverse does not occupy, the middle in the remaining one.
int setup_slab_factors(th_ctx *c, int s0, int nb, const c64 *A, int npad, long long amat,
                       c64 *const W[3], c64 *T1, int ldw, int ldt, c64 *pws, hipStream_t s) {
  const int P = c->P;
  int max_nsl = 0, max_m = 0, max_lsz = 0;
  for (int i = s0; i < s0 + nb; ++i) {
    max_nsl = std::max(max_nsl, c->subs[i].nsl);
    max_m = std::max(max_m, slab_rows(c->subs[i], c->subs[i].nsl - 1, P));
    max_lsz = std::max(max_lsz, c->subs[i].lsz);
  }
  const int nlo = (max_nsl - 1) / 2, nup = max_nsl - 1 - nlo;
  int prev = -1, cur = 0, rc = 0;
  for (int i = 0; i < nlo && rc == 0; ++i) {
    rc = slab_setup_step(c, s0, nb, A, npad, amat, W[cur], prev >= 0 ? W[prev] : nullptr,
                         nullptr, T1, ldw, ldt, max_lsz, max_m, pws, kLowerChain, i, nlo, s);
    prev = cur;
    cur = 1 - cur;
  }
  const int wlo = prev;
  int free_buf[2], nf = 0;
  for (int k = 0; k < 3; ++k)
    if (k != wlo && nf < 2) free_buf[nf++] = k;
  prev = -1;
  for (int i = 0; i < nup && rc == 0; ++i) {
    cur = free_buf[i & 1];
    rc = slab_setup_step(c, s0, nb, A, npad, amat, W[cur], nullptr,
                         prev >= 0 ? W[prev] : nullptr, T1, ldw, ldt, max_lsz, max_m, pws,
                         kUpperChain, i, nup, s);
    prev = cur;
  }
  const int wup = prev;
  int mid = 0;
  while (mid == wlo || mid == wup) ++mid;
  if (rc == 0)
    rc = slab_setup_step(c, s0, nb, A, npad, amat, W[mid], wlo >= 0 ? W[wlo] : nullptr,
                         wup >= 0 ? W[wup] : nullptr, T1, ldw, ldt, max_lsz, max_m, pws, kMiddle,
                         0, 0, s);
  return rc;
}

// ---------------------------------------------------------------------------
// apply

// Z = R_i r in the Omega-local numbering
template <typename T>
__global__ __launch_bounds__(256) void k_slab_gather(const Sub *__restrict__ subs,
                                                     const cx<T> *__restrict__ r,
                                                     cx<T> *__restrict__ Z, int P, int n1,
                                                     long long nf, long long xrows) {
  const Sub s = subs[blockIdx.y];
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k >= s.nOm) return;
  const long long q = blockIdx.z;
  Z[q * xrows + s.xoff + k] = r[q * nf + om_node(s, k, P, n1)];
}

// acc[q] = sum_{b0 <= b < b1} G^T[b][a] x[b][q] for the output row a of the
// thread: g points at entry (0, a) of the stored G_t^T (rows of ld entries);
// loads in batches of kRowsInFlight rows, all issued before their use.
constexpr int kRowsInFlight = 16;

template <typename TB, typename T, int RC>
__device__ __forceinline__ void slab_gemv_row(const cx<TB> *__restrict__ g, int m, int b0, int b1,
                                              const cx<T> *__restrict__ x, cx<T> (&acc)[RC]) {
  constexpr int U = kRowsInFlight;
#pragma unroll
  for (int q = 0; q < RC; ++q) acc[q] = {0, 0};
  for (int b = b0; b < b1; b += U) {
    cx<T> gv[U];
#pragma unroll
    for (int u = 0; u < U; ++u)
      gv[u] = b + u < b1 ? ccast<T>(ld_stream(g + (long long)(b + u) * m)) : cx<T>{0, 0};
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (b + u < b1)
#pragma unroll
        for (int q = 0; q < RC; ++q) cmac(acc[q], gv[u], x[(b + u) * RC + q]);
  }
}

// The first kRowsAhead rows of a thread's range, loaded before the workgroup
// forms its right-hand side (they do not depend on it), so that streaming
// starts at once; slab_gemv_ahead then consumes them and the rest.
constexpr int kRowsAhead = 6;

template <typename TB, typename T>
__device__ __forceinline__ void slab_rows_ahead(const cx<TB> *__restrict__ g, int m, int b0, int b1,
                                                cx<T> (&ga)[kRowsAhead]) {
#pragma unroll
  for (int u = 0; u < kRowsAhead; ++u)
    ga[u] = b0 + u < b1 ? ccast<T>(ld_stream(g + (long long)(b0 + u) * m)) : cx<T>{0, 0};
}

template <typename TB, typename T, int RC>
__device__ __forceinline__ void slab_gemv_ahead(const cx<TB> *__restrict__ g, int m, int b0, int b1,
                                                const cx<T> (&ga)[kRowsAhead],
                                                const cx<T> *__restrict__ x, cx<T> (&acc)[RC]) {
  cx<T> rest[RC];
  slab_gemv_row<TB, T, RC>(g, m, min(b0 + kRowsAhead, b1), b1, x, rest);
#pragma unroll
  for (int q = 0; q < RC; ++q) acc[q] = {0, 0};
#pragma unroll
  for (int u = 0; u < kRowsAhead; ++u)
    if (b0 + u < b1)
#pragma unroll
      for (int q = 0; q < RC; ++q) cmac(acc[q], ga[u], x[(b0 + u) * RC + q]);
#pragma unroll
  for (int q = 0; q < RC; ++q) acc[q] = acc[q] + rest[q];
}

// Wavefronts per workgroup of the forward and backward sweeps (measured on
// C2: 8 and 2 take a smoother step from 1.095 to 1.076 ms against 4 and 4;
// the backward rows, n_layer per slab, are too few for more).  The NW
// wavefronts of a workgroup share its 64 output rows and split the rows b of
// G_t^T (E_t^T) in NW parts; their partial sums are added in wavefront order
// through LDS (red: NW x 64 x RC) by the first wavefront, which returns them
// in acc (other wavefronts return false).
constexpr int kFwdWaves = 8, kBwdWaves = 2;

template <typename T, int RC, int NW>
__device__ __forceinline__ bool slab_sum_waves(cx<T> (&acc)[RC], cx<T> *__restrict__ red) {
  if (NW == 1) return true;
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  __syncthreads();  // red overlays the staged right-hand side: every wavefront is done with it
#pragma unroll
  for (int q = 0; q < RC; ++q) red[(wave * 64 + lane) * RC + q] = acc[q];
  __syncthreads();
  if (wave != 0) return false;
#pragma unroll
  for (int q = 0; q < RC; ++q) {
    cx<T> v = red[lane * RC + q];
    for (int w = 1; w < NW; ++w) v = v + red[(w * 64 + lane) * RC + q];
    acc[q] = v;
  }
  return true;
}

// Forward step i of the twisted sweep (i < S: the lower chain in row blocks yb
// < nyb, the upper chain above; i = S: the middles) for all subdomains and RC
// right-hand sides: the right-hand side of the slab is formed in LDS by every
// workgroup of it (band products unrolled, so their loads are issued
// together); a workgroup then covers 64 rows a of the slab, one per lane,
// its kFwdWaves wavefronts reading a part each of the rows b of the stored
// G_t^T.  LDS: the slab's right-hand sides [ldx][RC], then the partial sums.
template <typename TB, typename T, int RC, int P, int DIM>
__global__ __launch_bounds__(64 * kFwdWaves) void k_slab_fwd(const Sub *__restrict__ subs,
                                                 const cx<TB> *__restrict__ B,
                                                 const cx<T> *__restrict__ Z,
                                                 cx<T> *__restrict__ V, long long xrows,
                                                 int nrhs, int i, int S, int nyb, int ldx,
                                                 int nsub) {
  constexpr int W2 = 2 * P + 1, CB = (DIM == 3 ? W2 * W2 : W2) * P;
  extern __shared__ __align__(16) char slab_smem[];
  cx<T> *x = (cx<T> *)slab_smem;
  cx<T> *red = x;  // the partial sums reuse the staged right-hand side's LDS
  SweepItem it;
  if (!sweep_item(nsub, i < S ? 2 * nyb : nyb, it)) return;  // uniform
  const Sub s = subs[it.si];
  const int M = slab_mid(s), U = s.nsl - 1 - M;
  int t, lo, up, yb = it.yb;
  if (i == S) {
    t = M;
    lo = M >= 1;
    up = U >= 1;
  } else if (yb < nyb) {
    t = i - (S - M);
    lo = t >= 1;
    up = 0;
  } else {
    yb -= nyb;
    const int j = i - (S - U);
    t = j >= 0 ? s.nsl - 1 - j : -1;
    lo = 0;
    up = j >= 1;
  }
  if (t < 0) return;  // uniform: no slab of this chain at this step
  const int m = slab_rows(s, t, P);
  const int a0 = yb * 64;
  if (a0 >= m) return;  // uniform
  const int r0 = it.z * RC, nq = min(RC, nrhs - r0);
  const long long row0 = (long long)t * P * s.lsz;
  const long long vq = (long long)r0 * xrows + s.xoff;
  const int a = a0 + threadIdx.x % 64, wave = threadIdx.x / 64;
  const int bq = (m + kFwdWaves - 1) / kFwdWaves, ld = slab_ld(m);
  const int gb0 = min(wave * bq, m), gb1 = min((wave + 1) * bq, m);
  const cx<TB> *gp = B + slab_goff(s, t, P) + min(a, ld - 1);
  cx<T> ga[kRowsAhead];
  slab_rows_ahead<TB, T>(gp, ld, gb0, gb1, ga);
  for (int j = threadIdx.x; j < m; j += 64 * kFwdWaves) {
    cx<T> v[RC];
#pragma unroll
    for (int q = 0; q < RC; ++q)
      v[q] = q < nq ? Z[vq + (long long)q * xrows + row0 + j] : cx<T>{0, 0};
    if (lo && j < s.lsz) {
      cx<T> w[RC];
      band_lower<TB, T, RC, P, DIM>(s, B + s.coff + (long long)(t - 1) * s.lsz * CB, V,
                                    vq + (long long)(t - 1) * P * s.lsz, xrows, nq, j, w);
#pragma unroll
      for (int q = 0; q < RC; ++q) v[q] = v[q] - w[q];
    }
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
  __syncthreads();
  cx<T> acc[RC];
  slab_gemv_ahead<TB, T, RC>(gp, ld, gb0, gb1, ga, x, acc);
  if (!slab_sum_waves<T, RC, kFwdWaves>(acc, red) || a >= m) return;
#pragma unroll
  for (int q = 0; q < RC; ++q)
    if (q < nq) V[vq + (long long)q * xrows + row0 + a] = acc[q];
}

// Backward step j of the twisted sweep: the lower chain's slab M - 1 - j in
// row blocks yb < nyb, x_t = y_t - E_t w with w = x_{t+1} on the first layer of
// slab t + 1; the upper chain's slab M + 1 + j above, x_t = y_t - G_t[:, first
// layer] w with w = A[t][t-1] x_{t-1} (band product).  w is staged in LDS;
// 64 output rows per workgroup, its kBwdWaves wavefronts splitting the n_layer
// rows of the stored E_t^T (the first n_layer rows of the stored G_t^T).
template <typename TB, typename T, int RC, int P, int DIM>
__global__ __launch_bounds__(64 * kBwdWaves) void k_slab_bwd(const Sub *__restrict__ subs,
                                                 const cx<TB> *__restrict__ B,
                                                 cx<T> *__restrict__ V, long long xrows, int nrhs,
                                                 int jstep, int nyb, int ldx, int nsub) {
  constexpr int W2 = 2 * P + 1, CB = (DIM == 3 ? W2 * W2 : W2) * P;
  extern __shared__ __align__(16) char slab_smem[];
  cx<T> *w = (cx<T> *)slab_smem;
  cx<T> *red = w;  // the partial sums reuse the staged right-hand side's LDS
  SweepItem it;
  if (!sweep_item(nsub, 2 * nyb, it)) return;  // uniform
  const Sub s = subs[it.si];
  const int M = slab_mid(s), U = s.nsl - 1 - M;
  int yb = it.yb;
  const bool upper = yb >= nyb;
  if (upper) yb -= nyb;
  if (upper ? jstep >= U : jstep >= M) return;  // uniform
  const int t = upper ? M + 1 + jstep : M - 1 - jstep;
  const int m = slab_rows(s, t, P), nl = s.lsz;
  const int a0 = yb * 64;
  if (a0 >= m) return;  // uniform
  const int r0 = it.z * RC, nq = min(RC, nrhs - r0);
  const long long vq = (long long)r0 * xrows + s.xoff;
  const long long row0 = (long long)t * P * s.lsz;
  const int a = a0 + threadIdx.x % 64, wave = threadIdx.x / 64;
  const int cq = (nl + kBwdWaves - 1) / kBwdWaves;
  const int ld = slab_ld(m);
  // lower: E_t^T; upper: the first n_layer rows of G_t^T
  const cx<TB> *g = upper ? B + slab_goff(s, t, P) : B + s.ecoff + (long long)t * nl * ld;
  const int c0 = min(wave * cq, nl), c1 = min((wave + 1) * cq, nl);
  // the rows and y_t do not depend on w: their loads go out before w is formed
  cx<T> ga[kRowsAhead], yo[RC];
  slab_rows_ahead<TB, T>(g + min(a, ld - 1), ld, c0, c1, ga);
#pragma unroll
  for (int q = 0; q < RC; ++q)
    yo[q] = q < nq && a < m ? V[vq + (long long)q * xrows + row0 + a] : cx<T>{0, 0};
  for (int c = threadIdx.x; c < nl; c += 64 * kBwdWaves) {
    cx<T> v[RC];
    if (upper) {
      band_lower<TB, T, RC, P, DIM>(s, B + s.coff + (long long)(t - 1) * s.lsz * CB, V,
                                    vq + (long long)(t - 1) * P * s.lsz, xrows, nq, c, v);
    } else {
#pragma unroll
      for (int q = 0; q < RC; ++q)
        v[q] = q < nq ? V[vq + (long long)q * xrows + (long long)(t + 1) * P * s.lsz + c]
                      : cx<T>{0, 0};
    }
#pragma unroll
    for (int q = 0; q < RC; ++q) w[c * RC + q] = v[q];
  }
  __syncthreads();
  cx<T> acc[RC];
  slab_gemv_ahead<TB, T, RC>(g + min(a, ld - 1), ld, c0, c1, ga, w, acc);
  if (!slab_sum_waves<T, RC, kBwdWaves>(acc, red) || a >= m) return;
#pragma unroll
  for (int q = 0; q < RC; ++q)
    if (q < nq) V[vq + (long long)q * xrows + row0 + a] = yo[q] - acc[q];
}

// Y_i[j] = x[U node j] / L_j
template <typename T>
__global__ __launch_bounds__(256) void k_slab_extract(const Sub *__restrict__ subs,
                                                      const int *__restrict__ nblk,
                                                      const cx<T> *__restrict__ V,
                                                      cx<T> *__restrict__ Y, int P,
                                                      long long xrows, long long yrows) {
  const Sub s = subs[blockIdx.y];
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= s.nU) return;
  const long long q = blockIdx.z;
  int gn[3], uj;
  u_node(s, j, P, gn, uj);
  const T invL = (T)(1.0 / (double)(nblk[2 * gn[0] + 1] * nblk[2 * gn[1] + 1] * nblk[2 * gn[2] + 1]));
  const cx<T> v = V[q * xrows + s.xoff + uj];
  Y[q * yrows + s.yoff + j] = cx<T>{v.re * invL, v.im * invL};
}

// LDS entries per right-hand side of the sweeps: the staged slab right-hand
// side, whose space the wavefronts' partial sums take over afterwards
static size_t slab_lds_rows(const th_ctx *c) {
  return std::max<size_t>((size_t)c->max_slab_rows, 64 * (size_t)std::max(kFwdWaves, kBwdWaves));
}

template <typename TB, typename T, int RC, int P, int DIM>
static int slab_sweeps_pd(const th_ctx *c, int nrhs, hipStream_t s) {
  const unsigned nsub = (unsigned)c->subs.size();
  const int ldx = c->max_slab_rows;
  const size_t shm = slab_lds_rows(c) * RC * sizeof(cx<T>);
  const int nyb = ceil_div(ldx, 64);
  const unsigned nz = (unsigned)ceil_div(nrhs, RC);
  const int S = c->max_nsl / 2;  // chain steps: the longest upper chain
  const cx<TB> *B = (const cx<TB> *)c->d_B;
  const unsigned groups8 = 8 * (unsigned)ceil_div((int)nsub, 8);  // XCD-aware 1-D grids
  for (int i = 0; i <= S; ++i)
    hipLaunchKernelGGL((k_slab_fwd<TB, T, RC, P, DIM>),
                       dim3(groups8 * (unsigned)(i < S ? 2 * nyb : nyb) * nz), dim3(64 * kFwdWaves),
                       shm, s, c->d_subs, B, (const cx<T> *)c->w_x, (cx<T> *)c->w_z, c->x_rows, nrhs,
                       i, S, nyb, ldx, (int)nsub);
  for (int j = 0; j < S; ++j)
    hipLaunchKernelGGL((k_slab_bwd<TB, T, RC, P, DIM>), dim3(groups8 * (unsigned)(2 * nyb) * nz),
                       dim3(64 * kBwdWaves), shm, s, c->d_subs, B, (cx<T> *)c->w_z, c->x_rows, nrhs, j,
                       nyb, ldx, (int)nsub);
  return 0;
}

template <typename TB, typename T, int RC>
static int slab_sweeps_t(const th_ctx *c, int nrhs, hipStream_t s) {
  if (c->dim == 3) {
    if (c->P == 2) return slab_sweeps_pd<TB, T, RC, 2, 3>(c, nrhs, s);
    if (c->P == 4) return slab_sweeps_pd<TB, T, RC, 4, 3>(c, nrhs, s);
  } else {
    switch (c->P) {
      case 2: return slab_sweeps_pd<TB, T, RC, 2, 2>(c, nrhs, s);
      case 4: return slab_sweeps_pd<TB, T, RC, 4, 2>(c, nrhs, s);
      case 6: return slab_sweeps_pd<TB, T, RC, 6, 2>(c, nrhs, s);
      case 8: return slab_sweeps_pd<TB, T, RC, 8, 2>(c, nrhs, s);
    }
  }
  set_error("unsupported order for the slab layout");
  return TH_EUNSUPPORTED;
}

// right-hand sides per sweep pass: the slab's right-hand sides must fit in 48 KiB of LDS
template <typename TB, typename T>
static int slab_apply_t(const th_ctx *c, const void *r, void *y, int nrhs, hipStream_t s) {
  const unsigned nsub = (unsigned)c->subs.size();
  hipLaunchKernelGGL((k_slab_gather<T>), dim3(ceil_div(c->max_nom, 256), nsub, nrhs), dim3(256), 0,
                     s, c->d_subs, (const cx<T> *)r, (cx<T> *)c->w_x, c->P, c->n1, c->nf,
                     c->x_rows);
  const size_t row_bytes = slab_lds_rows(c) * sizeof(cx<T>);
  int rc;
  if (c->slab_pk) {
    // packed: the largest chunk whose LDS fits in 64 KiB (two workgroups
    // per compute unit)
    auto fits = [&](int r) { return slab_pk_lds(c, r * sizeof(cx<T>)) <= kSlabPkLds; };
    rc = slab_pk_sweeps<TB, T>(c, nrhs, nrhs >= 4 && fits(4) ? 4 : (nrhs >= 2 && fits(2) ? 2 : 1),
                               s);
  } else if (nrhs >= 4 && 4 * row_bytes <= 48 * 1024)
    rc = slab_sweeps_t<TB, T, 4>(c, nrhs, s);
  else if (nrhs >= 2 && 2 * row_bytes <= 48 * 1024)
    rc = slab_sweeps_t<TB, T, 2>(c, nrhs, s);
  else
    rc = slab_sweeps_t<TB, T, 1>(c, nrhs, s);
  if (rc) return rc;
  hipLaunchKernelGGL((k_slab_extract<T>), dim3(ceil_div(c->max_ldb, 256), nsub, nrhs), dim3(256),
                     0, s, c->d_subs, (const int *)c->d_nblk, (const cx<T> *)c->w_z, (cx<T> *)y,
                     c->P, c->x_rows, c->y_rows);
  TH_HIP_CHECK_RET(hipGetLastError());
  return 0;
}

int launch_dd_slab(const th_ctx *c, const void *r, void *y, int nrhs, bool f32, hipStream_t s) {
  if (c->desc.gemm == TH_GEMM_F32)
    return f32 ? slab_apply_t<float, float>(c, r, y, nrhs, s)
               : slab_apply_t<float, double>(c, r, y, nrhs, s);
  return f32 ? slab_apply_t<double, float>(c, r, y, nrhs, s)
             : slab_apply_t<double, double>(c, r, y, nrhs, s);
}

}  // namespace th
