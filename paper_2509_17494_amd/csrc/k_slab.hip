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
//   backward  x_t = y_t - G_t L_{t+1}^T x_{t+1}[first layer of t + 1],
// one launch per slab for all subdomains.  Stored per subdomain: every G_t
// transposed (entry (b, a) at b m_t + a, so one output row per thread reads
// consecutive entries of a row), then the couplings L_t of every slab t >= 1
// as bands: for each first-layer node a the (2P+1)^(d-1) x P block of slab
// t - 1 nodes within P positions of a in every in-layer direction (zero where a
// node lies outside Omega or shares no cell with a).  The bytes per
// application are twice the G_t (forward and backward) instead of the
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

// entries of the G_t of slabs before t (all of them have P layers)
__host__ __device__ __forceinline__ long long slab_goff(const Sub &s, int t, int P) {
  const long long m = (long long)P * s.lsz;
  return s.boff + (long long)t * m * m;
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

// store G_t = W transposed and, for t >= 1, the coupling band of slab t
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
    B[slab_goff(s, t, P) + e] = cx<TB>{(TB)v.re, (TB)v.im};
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

// Forward step of slab t for all subdomains and RC right-hand sides: the
// right-hand side r_t - L_t y_{t-1} is formed in LDS by every workgroup of the
// subdomain; each thread then owns one row a of the slab (64 rows per
// workgroup) and reads row b of the stored G_t^T for b = 0 .. m - 1.
template <typename TB, typename T, int RC>
__global__ __launch_bounds__(64) void k_slab_fwd(const Sub *__restrict__ subs,
                                                 const cx<TB> *__restrict__ B,
                                                 const cx<T> *__restrict__ Z,
                                                 cx<T> *__restrict__ V, long long xrows,
                                                 int nrhs, int t, int P, int dim) {
  extern __shared__ __align__(16) char slab_smem[];
  cx<T> *x = (cx<T> *)slab_smem;  // [m][RC]
  const Sub s = subs[blockIdx.x];
  if (t >= s.nsl) return;  // uniform
  const int m = slab_rows(s, t, P);
  const int a0 = blockIdx.y * 64;
  if (a0 >= m) return;  // uniform
  const int r0 = blockIdx.z * RC, nq = min(RC, nrhs - r0);
  const long long row0 = (long long)t * P * s.lsz;
  const int cb = band_width(P, dim);
  const cx<TB> *Ct = B + s.coff + (long long)(t - 1) * s.lsz * cb;
  for (int j = threadIdx.x; j < m; j += 64) {
#pragma unroll
    for (int q = 0; q < RC; ++q) {
      cx<T> v = {0, 0};
      if (q < nq) {
        const long long base = (long long)(r0 + q) * xrows + s.xoff;
        v = Z[base + row0 + j];
        if (t > 0 && j < s.lsz) {
          const cx<TB> *cr = Ct + (long long)j * cb;
          for (int k = 0; k < cb; ++k) {
            const int col = band_col(s, t, j, k, P, dim);
            if (col >= 0) {
              const cx<TB> l = cr[k];
              const cx<T> y = V[base + col];
              v.re -= (T)l.re * y.re - (T)l.im * y.im;
              v.im -= (T)l.re * y.im + (T)l.im * y.re;
            }
          }
        }
      }
      x[j * RC + q] = v;
    }
  }
  __syncthreads();
  const int a = a0 + threadIdx.x;
  if (a >= m) return;
  const cx<TB> *g = B + slab_goff(s, t, P) + a;
  cx<T> acc[RC];
#pragma unroll
  for (int q = 0; q < RC; ++q) acc[q] = {0, 0};
#pragma unroll 8
  for (int b = 0; b < m; ++b) {
    const cx<T> gv = ccast<T>(ld_stream(g + (long long)b * m));
#pragma unroll
    for (int q = 0; q < RC; ++q) cmac(acc[q], gv, x[b * RC + q]);
  }
#pragma unroll
  for (int q = 0; q < RC; ++q)
    if (q < nq) V[(long long)(r0 + q) * xrows + s.xoff + row0 + a] = acc[q];
}

// Backward step of slab t < nsl - 1: w = L_{t+1}^T x_{t+1}[first layer] in LDS
// (for a node b of slab t the first-layer nodes of slab t + 1 within P
// positions, read from their coupling bands), then x_t = y_t - G_t w.
template <typename TB, typename T, int RC>
__global__ __launch_bounds__(64) void k_slab_bwd(const Sub *__restrict__ subs,
                                                 const cx<TB> *__restrict__ B,
                                                 cx<T> *__restrict__ V, long long xrows, int nrhs,
                                                 int t, int P, int dim) {
  extern __shared__ __align__(16) char slab_smem[];
  cx<T> *w = (cx<T> *)slab_smem;  // [m][RC]
  const Sub s = subs[blockIdx.x];
  if (t >= s.nsl - 1) return;  // uniform
  const int m = P * s.lsz;
  const int a0 = blockIdx.y * 64;
  if (a0 >= m) return;  // uniform
  const int r0 = blockIdx.z * RC, nq = min(RC, nrhs - r0);
  const long long row0 = (long long)t * P * s.lsz, rn = (long long)(t + 1) * P * s.lsz;
  const int cb = band_width(P, dim);
  const int W2 = 2 * P + 1;
  const cx<TB> *Cn = B + s.coff + (long long)t * s.lsz * cb;  // couplings of slab t + 1
  for (int j = threadIdx.x; j < m; j += 64) {
    const int lb = j / s.lsz, ib = j % s.lsz;
    const int xb = ib % s.nox, yb = dim == 3 ? ib / s.nox : 0;
#pragma unroll
    for (int q = 0; q < RC; ++q) {
      cx<T> v = {0, 0};
      if (q < nq) {
        const long long base = (long long)(r0 + q) * xrows + s.xoff + rn;
        for (int jy = 0; jy < (dim == 3 ? W2 : 1); ++jy) {
          const int ya = dim == 3 ? yb + P - jy : 0;  // jy = yb - ya + P
          if (ya < 0 || (dim == 3 && ya >= s.noy)) continue;
          for (int jx = 0; jx < W2; ++jx) {
            const int xa = xb + P - jx;  // jx = xb - xa + P
            if (xa < 0 || xa >= s.nox) continue;
            const int a = ya * s.nox + xa;
            const cx<TB> l = Cn[(long long)a * cb + (jy * W2 + jx) * P + lb];
            const cx<T> xv = V[base + a];
            v.re += (T)l.re * xv.re - (T)l.im * xv.im;
            v.im += (T)l.re * xv.im + (T)l.im * xv.re;
          }
        }
      }
      w[j * RC + q] = v;
    }
  }
  __syncthreads();
  const int a = a0 + threadIdx.x;
  if (a >= m) return;
  const cx<TB> *g = B + slab_goff(s, t, P) + a;
  cx<T> acc[RC];
#pragma unroll
  for (int q = 0; q < RC; ++q) acc[q] = {0, 0};
#pragma unroll 8
  for (int b = 0; b < m; ++b) {
    const cx<T> gv = ccast<T>(ld_stream(g + (long long)b * m));
#pragma unroll
    for (int q = 0; q < RC; ++q) cmac(acc[q], gv, w[b * RC + q]);
  }
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

template <typename TB, typename T, int RC>
static int slab_sweeps_t(const th_ctx *c, int nrhs, hipStream_t s) {
  const unsigned nsub = (unsigned)c->subs.size();
  const size_t shm = (size_t)c->max_slab_rows * RC * sizeof(cx<T>);
  const dim3 grid(nsub, (unsigned)ceil_div(c->max_slab_rows, 64), (unsigned)ceil_div(nrhs, RC));
  const cx<TB> *B = (const cx<TB> *)c->d_B;
  for (int t = 0; t < c->max_nsl; ++t)
    hipLaunchKernelGGL((k_slab_fwd<TB, T, RC>), grid, dim3(64), shm, s, c->d_subs, B,
                       (const cx<T> *)c->w_x, (cx<T> *)c->w_z, c->x_rows, nrhs, t, c->P, c->dim);
  for (int t = c->max_nsl - 2; t >= 0; --t)
    hipLaunchKernelGGL((k_slab_bwd<TB, T, RC>), grid, dim3(64), shm, s, c->d_subs, B,
                       (cx<T> *)c->w_z, c->x_rows, nrhs, t, c->P, c->dim);
  return 0;
}

// right-hand sides per sweep pass: the slab's right-hand sides must fit in 48 KiB of LDS
template <typename TB, typename T>
static int slab_apply_t(const th_ctx *c, const void *r, void *y, int nrhs, hipStream_t s) {
  const unsigned nsub = (unsigned)c->subs.size();
  hipLaunchKernelGGL((k_slab_gather<T>), dim3(ceil_div(c->max_nom, 256), nsub, nrhs), dim3(256), 0,
                     s, c->d_subs, (const cx<T> *)r, (cx<T> *)c->w_x, c->P, c->n1, c->nf,
                     c->x_rows);
  const size_t row_bytes = (size_t)c->max_slab_rows * sizeof(cx<T>);
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
