// Slab-factor layout of the subdomain solves (Alg. 2, w_i = (A_s^(i))^{-1} R_i r).
//
// In its Omega-local numbering (x fastest, slowest axis y in 2-D, z in 3-D)
// A_s^(i) couples node layers only through shared cells, so grouping the
// layers of one cell row into a slab (P layers; the last slab also takes the
// top layer) makes it block tridiagonal: slab t couples to slab t - 1 only
// through its first layer.  Setup runs the block elimination in natural order
//   S_0 = T_0,  S_t = T_t - L_t S_{t-1}^{-1} L_t^T  (first-layer block only),
//   G_t = S_t^{-1}
// (A_s^(i) is complex symmetric, so the upper coupling is L_t^T), and the
// apply is
//   forward   y_t = G_t (r_t - L_t y_{t-1})
//   backward  x_t = y_t - E_t x_{t+1}[first layer of t + 1],  E_t = G_t L_{t+1}^T,
// one launch per slab for all subdomains.  Stored per subdomain: every G_t
// transposed (entry (b, a) at b ld_t + a, rows padded to ld_t, a multiple of
// 8 entries, so one output row per thread reads consecutive entries of a row
// and every row starts on a 128-byte line); the couplings L_t of every slab t >= 1 as
// bands: for each first-layer node a the (2P+1)^(d-1) x P block of slab t - 1
// nodes within P positions of a in every in-layer direction (zero where a node
// lies outside Omega or shares no cell with a); and every E_t (m_t x n_layer,
// the product the elimination forms anyway) transposed, likewise padded.  The bytes per
// application are the G_t plus the E_t (a fraction 1/P of them) instead of the
// n_U x n_Omega rows of an explicit inverse.  Elimination without pivoting is
// stable here for the reason given for the Gauss-Jordan inverses: i A_s^(i)
// has a positive definite Hermitian part, which every Schur complement keeps
// (Dirichlet nodes are decoupled unit rows).
#include <algorithm>

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

__host__ __device__ __forceinline__ int band_width(int P, int dim) {
  return (dim == 3 ? (2 * P + 1) * (2 * P + 1) : (2 * P + 1)) * P;
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

// ---------------------------------------------------------------------------
// setup (FP64), batched over subdomains s0 .. s0 + gridDim.z - 1

// W = the diagonal block T_t of A (rows and columns of slab t), identity
// padding; identity for subdomains with fewer slabs.
__global__ __launch_bounds__(256) void k_slab_copy(const Sub *__restrict__ subs, int s0,
                                                   const c64 *__restrict__ A, int lda,
                                                   long long amat, c64 *__restrict__ W, int ldw,
                                                   long long wmat, int t, int P) {
  const Sub s = subs[s0 + blockIdx.z];
  const long long e = blockIdx.x * 256LL + threadIdx.x;
  if (e >= (long long)ldw * ldw) return;
  const int a = (int)(e / ldw), b = (int)(e % ldw);
  c64 v = a == b ? c64{1.0, 0.0} : c64{0, 0};
  if (t < s.nsl) {
    const int m = slab_rows(s, t, P);
    const long long r0 = (long long)t * P * s.lsz;
    if (a < m && b < m) v = A[blockIdx.z * amat + (r0 + a) * lda + r0 + b];
  }
  W[blockIdx.z * wmat + e] = v;
}

// T1 = G_{t-1} U where U = A[slab t - 1, first layer of t] (m_{t-1} x lsz)
__global__ __launch_bounds__(256) void k_slab_t1(const Sub *__restrict__ subs, int s0,
                                                 const c64 *__restrict__ A, int lda,
                                                 long long amat, const c64 *__restrict__ Gp,
                                                 int ldw, long long wmat, c64 *__restrict__ T1,
                                                 int ldt, long long tmat, int t, int P) {
  const Sub s = subs[s0 + blockIdx.z];
  if (t >= s.nsl) return;
  const int mp = P * s.lsz;
  const long long e = blockIdx.x * 256LL + threadIdx.x;
  if (e >= (long long)mp * s.lsz) return;
  const int r = (int)(e / s.lsz), c = (int)(e % s.lsz);
  const long long rp = (long long)(t - 1) * P * s.lsz, r0 = (long long)t * P * s.lsz;
  const c64 *g = Gp + blockIdx.z * wmat + (long long)r * ldw;
  const c64 *u = A + blockIdx.z * amat + rp * lda + r0 + c;
  c64 acc = {0, 0};
  for (int k = 0; k < mp; ++k) cmac(acc, g[k], u[(long long)k * lda]);
  T1[blockIdx.z * tmat + (long long)r * ldt + c] = acc;
}

// first-layer block of S_t: W[a][a'] -= sum_k A[first layer a][slab t - 1, k] T1[k][a']
__global__ __launch_bounds__(256) void k_slab_schur(const Sub *__restrict__ subs, int s0,
                                                    const c64 *__restrict__ A, int lda,
                                                    long long amat, const c64 *__restrict__ T1,
                                                    int ldt, long long tmat, c64 *__restrict__ W,
                                                    int ldw, long long wmat, int t, int P) {
  const Sub s = subs[s0 + blockIdx.z];
  if (t >= s.nsl) return;
  const long long e = blockIdx.x * 256LL + threadIdx.x;
  if (e >= (long long)s.lsz * s.lsz) return;
  const int a = (int)(e / s.lsz), a2 = (int)(e % s.lsz);
  const int mp = P * s.lsz;
  const long long rp = (long long)(t - 1) * P * s.lsz, r0 = (long long)t * P * s.lsz;
  const c64 *l = A + blockIdx.z * amat + (r0 + a) * lda + rp;
  const c64 *t1 = T1 + blockIdx.z * tmat + a2;
  c64 acc = {0, 0};
  for (int k = 0; k < mp; ++k) cmac(acc, l[k], t1[(long long)k * ldt]);
  c64 &w = W[blockIdx.z * wmat + (long long)a * ldw + a2];
  w = w - acc;
}

// store G_t = W transposed (rows padded to slab_ld) and, for t >= 1, the
// coupling band of slab t
template <typename TB>
__global__ __launch_bounds__(256) void k_slab_store(const Sub *__restrict__ subs, int s0,
                                                    const c64 *__restrict__ A, int lda,
                                                    long long amat, const c64 *__restrict__ W,
                                                    int ldw, long long wmat,
                                                    cx<TB> *__restrict__ B, int t, int P,
                                                    int dim) {
  const Sub s = subs[s0 + blockIdx.z];
  if (t >= s.nsl) return;
  const int m = slab_rows(s, t, P);
  const long long e = blockIdx.x * 256LL + threadIdx.x;
  const long long ng = (long long)m * m;
  const int cb = band_width(P, dim);
  if (e < ng) {
    const int b = (int)(e / m), a = (int)(e % m);
    const c64 v = W[blockIdx.z * wmat + (long long)a * ldw + b];
    B[slab_goff(s, t, P) + (long long)b * slab_ld(m) + a] = cx<TB>{(TB)v.re, (TB)v.im};
  } else if (t >= 1 && e < ng + (long long)s.lsz * cb) {
    const long long f = e - ng;
    const int a = (int)(f / cb), k = (int)(f % cb);
    const int col = band_col(s, t, a, k, P, dim);
    const long long r0 = (long long)t * P * s.lsz;
    c64 v = {0, 0};
    if (col >= 0) v = A[blockIdx.z * amat + (r0 + a) * lda + col];
    B[s.coff + (long long)(t - 1) * s.lsz * cb + f] = cx<TB>{(TB)v.re, (TB)v.im};
  }
}

// store E_{t-1} = T1 (rows of slab t - 1, columns: first layer of slab t) transposed
template <typename TB>
__global__ __launch_bounds__(256) void k_slab_store_e(const Sub *__restrict__ subs, int s0,
                                                      const c64 *__restrict__ T1, int ldt,
                                                      long long tmat, cx<TB> *__restrict__ B, int t,
                                                      int P) {
  const Sub s = subs[s0 + blockIdx.z];
  if (t >= s.nsl) return;
  const int mp = P * s.lsz;
  const long long e = blockIdx.x * 256LL + threadIdx.x;
  if (e >= (long long)s.lsz * mp) return;
  const int cc = (int)(e / mp), r = (int)(e % mp);
  const c64 v = T1[blockIdx.z * tmat + (long long)r * ldt + cc];
  B[s.ecoff + ((long long)(t - 1) * s.lsz + cc) * slab_ld(mp) + r] = cx<TB>{(TB)v.re, (TB)v.im};
}

int setup_slab_factors(th_ctx *c, int s0, int nb, const c64 *A, int npad, long long amat, c64 *W0,
                       c64 *W1, c64 *T1, int ldw, int ldt, c64 *pws, hipStream_t s) {
  const int P = c->P;
  const long long wmat = (long long)ldw * ldw, tmat = (long long)ldw * ldt;
  int max_nsl = 0, max_m = 0;
  long long max_lsz = 0;
  for (int i = s0; i < s0 + nb; ++i) {
    max_nsl = std::max(max_nsl, c->subs[i].nsl);
    max_m = std::max(max_m, slab_rows(c->subs[i], c->subs[i].nsl - 1, P));
    max_lsz = std::max<long long>(max_lsz, c->subs[i].lsz);
  }
  const int cb = band_width(P, c->dim);
  c64 *W = W0, *Wp = W1;
  for (int t = 0; t < max_nsl; ++t) {
    hipLaunchKernelGGL(k_slab_copy, dim3((unsigned)ceil_div_ll(wmat, 256), 1, nb), dim3(256), 0, s,
                       c->d_subs, s0, A, npad, amat, W, ldw, wmat, t, P);
    if (t > 0) {
      hipLaunchKernelGGL(k_slab_t1, dim3((unsigned)ceil_div_ll((long long)P * max_lsz * max_lsz, 256),
                                         1, nb),
                         dim3(256), 0, s, c->d_subs, s0, A, npad, amat, (const c64 *)Wp, ldw,
                         wmat, T1, ldt, tmat, t, P);
      hipLaunchKernelGGL(k_slab_schur, dim3((unsigned)ceil_div_ll(max_lsz * max_lsz, 256), 1, nb),
                         dim3(256), 0, s, c->d_subs, s0, A, npad, amat, (const c64 *)T1, ldt,
                         tmat, W, ldw, wmat, t, P);
      const dim3 ge((unsigned)ceil_div_ll((long long)P * max_lsz * max_lsz, 256), 1, nb);
      if (c->desc.gemm == TH_GEMM_F32)
        hipLaunchKernelGGL((k_slab_store_e<float>), ge, dim3(256), 0, s, c->d_subs, s0,
                           (const c64 *)T1, ldt, tmat, (cx<float> *)c->d_B, t, P);
      else
        hipLaunchKernelGGL((k_slab_store_e<double>), ge, dim3(256), 0, s, c->d_subs, s0,
                           (const c64 *)T1, ldt, tmat, (cx<double> *)c->d_B, t, P);
    }
    TH_HIP_CHECK_RET(hipGetLastError());
    int rc = gj_invert_batched(W, ldw, ldw, wmat, nb, s, pws);
    if (rc) return rc;
    const long long nst = (long long)max_m * max_m + max_lsz * cb;
    if (c->desc.gemm == TH_GEMM_F32)
      hipLaunchKernelGGL((k_slab_store<float>), dim3((unsigned)ceil_div_ll(nst, 256), 1, nb),
                         dim3(256), 0, s, c->d_subs, s0, A, npad, amat, (const c64 *)W, ldw, wmat,
                         (cx<float> *)c->d_B, t, P, c->dim);
    else
      hipLaunchKernelGGL((k_slab_store<double>), dim3((unsigned)ceil_div_ll(nst, 256), 1, nb),
                         dim3(256), 0, s, c->d_subs, s0, A, npad, amat, (const c64 *)W, ldw, wmat,
                         (cx<double> *)c->d_B, t, P, c->dim);
    TH_HIP_CHECK_RET(hipGetLastError());
    std::swap(W, Wp);
  }
  return 0;
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
constexpr int kRowsAhead = 8;

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

// The four wavefronts of a workgroup share its 64 output rows and split the
// rows b of G_t^T in quarters; their partial sums are added in wavefront order
// through LDS (red: 4 x 64 x RC) by the first wavefront, which returns them in
// acc (other wavefronts return false).
template <typename T, int RC>
__device__ __forceinline__ bool slab_sum_waves(cx<T> (&acc)[RC], cx<T> *__restrict__ red) {
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
#pragma unroll
  for (int q = 0; q < RC; ++q) red[(wave * 64 + lane) * RC + q] = acc[q];
  __syncthreads();
  if (wave != 0) return false;
#pragma unroll
  for (int q = 0; q < RC; ++q) {
    cx<T> v = red[lane * RC + q];
    for (int w = 1; w < 4; ++w) v = v + red[(w * 64 + lane) * RC + q];
    acc[q] = v;
  }
  return true;
}

// Forward step of slab t for all subdomains and RC right-hand sides: the
// right-hand side r_t - L_t y_{t-1} is formed in LDS by every workgroup of the
// subdomain (the band loops unrolled, so their loads are issued together);
// a workgroup then covers 64 rows a of the slab, one per lane, its four
// wavefronts reading a quarter each of the rows b of the stored G_t^T.
// LDS: the slab's right-hand sides [ldx][RC], then the partial sums.
template <typename TB, typename T, int RC, int P, int DIM>
__global__ __launch_bounds__(256) void k_slab_fwd(const Sub *__restrict__ subs,
                                                 const cx<TB> *__restrict__ B,
                                                 const cx<T> *__restrict__ Z,
                                                 cx<T> *__restrict__ V, long long xrows,
                                                 int nrhs, int t, int ldx) {
  constexpr int W2 = 2 * P + 1, CB = (DIM == 3 ? W2 * W2 : W2) * P;
  extern __shared__ __align__(16) char slab_smem[];
  cx<T> *x = (cx<T> *)slab_smem;
  cx<T> *red = x + (long long)ldx * RC;
  const Sub s = subs[blockIdx.x];
  if (t >= s.nsl) return;  // uniform
  const int m = slab_rows(s, t, P);
  const int a0 = blockIdx.y * 64;
  if (a0 >= m) return;  // uniform
  const int r0 = blockIdx.z * RC, nq = min(RC, nrhs - r0);
  const long long row0 = (long long)t * P * s.lsz;
  const cx<TB> *Ct = B + s.coff + (long long)(t - 1) * s.lsz * CB;
  const int a = a0 + threadIdx.x % 64, wave = threadIdx.x / 64;
  const int bq = (m + 3) / 4, ld = slab_ld(m);
  const int gb0 = min(wave * bq, m), gb1 = min((wave + 1) * bq, m);
  const cx<TB> *gp = B + slab_goff(s, t, P) + min(a, ld - 1);
  cx<T> ga[kRowsAhead];
  slab_rows_ahead<TB, T>(gp, ld, gb0, gb1, ga);
  for (int j = threadIdx.x; j < m; j += 256) {
    cx<T> v[RC];
#pragma unroll
    for (int q = 0; q < RC; ++q)
      v[q] = q < nq ? Z[(long long)(r0 + q) * xrows + s.xoff + row0 + j] : cx<T>{0, 0};
    if (t > 0 && j < s.lsz) {
      // Branch-free band product: positions outside Omega are clamped to a
      // node inside (its value is finite) and meet a zero band coefficient,
      // so every load can be issued before its use.
      const int xa = j % s.nox, ya = DIM == 3 ? j / s.nox : 0;
      const cx<TB> *cr = Ct + (long long)j * CB;
      const long long vb = (long long)r0 * xrows + s.xoff + (long long)(t - 1) * P * s.lsz;
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
            l[lb] = cr[(jy * W2 + jx) * P + lb];
#pragma unroll
            for (int q = 0; q < RC; ++q)
              y[lb][q] = V[vb + (long long)min(q, nq - 1) * xrows + lb * s.lsz + yb * s.nox + xb];
          }
#pragma unroll
          for (int lb = 0; lb < P; ++lb)
#pragma unroll
            for (int q = 0; q < RC; ++q) {
              v[q].re -= (T)l[lb].re * y[lb][q].re - (T)l[lb].im * y[lb][q].im;
              v[q].im -= (T)l[lb].re * y[lb][q].im + (T)l[lb].im * y[lb][q].re;
            }
        }
      }
    }
#pragma unroll
    for (int q = 0; q < RC; ++q) x[j * RC + q] = v[q];
  }
  __syncthreads();
  cx<T> acc[RC];
  slab_gemv_ahead<TB, T, RC>(gp, ld, gb0, gb1, ga, x, acc);
  if (!slab_sum_waves<T, RC>(acc, red) || a >= m) return;
#pragma unroll
  for (int q = 0; q < RC; ++q)
    if (q < nq) V[(long long)(r0 + q) * xrows + s.xoff + row0 + a] = acc[q];
}

// Backward step of slab t < nsl - 1: x_t = y_t - E_t w with w = x_{t+1} on
// the first layer of slab t + 1 (staged in LDS), the same division of work
// as the forward step over the n_layer rows of the stored E_t^T.
template <typename TB, typename T, int RC>
__global__ __launch_bounds__(256) void k_slab_bwd(const Sub *__restrict__ subs,
                                                 const cx<TB> *__restrict__ B,
                                                 cx<T> *__restrict__ V, long long xrows, int nrhs,
                                                 int t, int ldx, int P) {
  extern __shared__ __align__(16) char slab_smem[];
  cx<T> *w = (cx<T> *)slab_smem;
  cx<T> *red = w + (long long)ldx * RC;
  const Sub s = subs[blockIdx.x];
  if (t >= s.nsl - 1) return;  // uniform
  const int m = P * s.lsz, nl = s.lsz;
  const int a0 = blockIdx.y * 64;
  if (a0 >= m) return;  // uniform
  const int r0 = blockIdx.z * RC, nq = min(RC, nrhs - r0);
  const long long row0 = (long long)t * P * s.lsz, rn = (long long)(t + 1) * P * s.lsz;
  for (int j = threadIdx.x; j < nl; j += 256)
#pragma unroll
    for (int q = 0; q < RC; ++q)
      w[j * RC + q] = q < nq ? V[(long long)(r0 + q) * xrows + s.xoff + rn + j] : cx<T>{0, 0};
  __syncthreads();
  const int a = a0 + threadIdx.x % 64, wave = threadIdx.x / 64;
  const int cq = (nl + 3) / 4;
  cx<T> acc[RC];
  const int ld = slab_ld(m);
  slab_gemv_row<TB, T, RC>(B + s.ecoff + (long long)t * nl * ld + min(a, ld - 1), ld,
                           min(wave * cq, nl), min((wave + 1) * cq, nl), w, acc);
  if (!slab_sum_waves<T, RC>(acc, red) || a >= m) return;
#pragma unroll
  for (int q = 0; q < RC; ++q)
    if (q < nq) {
      cx<T> &o = V[(long long)(r0 + q) * xrows + s.xoff + row0 + a];
      o = o - acc[q];
    }
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

template <typename TB, typename T, int RC, int P, int DIM>
static int slab_sweeps_pd(const th_ctx *c, int nrhs, hipStream_t s) {
  const unsigned nsub = (unsigned)c->subs.size();
  const int ldx = c->max_slab_rows;
  const size_t shm = ((size_t)ldx + 256) * RC * sizeof(cx<T>);
  const dim3 grid(nsub, (unsigned)ceil_div(ldx, 64), (unsigned)ceil_div(nrhs, RC));
  const cx<TB> *B = (const cx<TB> *)c->d_B;
  for (int t = 0; t < c->max_nsl; ++t)
    hipLaunchKernelGGL((k_slab_fwd<TB, T, RC, P, DIM>), grid, dim3(256), shm, s, c->d_subs, B,
                       (const cx<T> *)c->w_x, (cx<T> *)c->w_z, c->x_rows, nrhs, t, ldx);
  for (int t = c->max_nsl - 2; t >= 0; --t)
    hipLaunchKernelGGL((k_slab_bwd<TB, T, RC>), grid, dim3(256), shm, s, c->d_subs, B,
                       (cx<T> *)c->w_z, c->x_rows, nrhs, t, ldx, P);
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
  const size_t row_bytes = ((size_t)c->max_slab_rows + 256) * sizeof(cx<T>);
  int rc;
  if (nrhs >= 4 && 4 * row_bytes <= 48 * 1024)
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
