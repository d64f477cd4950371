// Matrix-free fine operator: out = f + sgn * (A u) for the Q_p Galerkin matrix
// of a(u, v) = int grad u . grad v - int kappa u v - int_{Gamma_abs} i k u v
// (eq. bilin_form; kappa = k^2 + i eps, or the shifted coefficient of A_s,
// Sec. 4.1) on the 2-D N x N mesh.
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
// reads one extra cell layer on the low sides.
#include "ctx.hpp"

namespace th {

template <int P> struct TileOf;
template <> struct TileOf<2> { static constexpr int TC = 16; };
template <> struct TileOf<4> { static constexpr int TC = 8; };
template <> struct TileOf<6> { static constexpr int TC = 5; };
template <> struct TileOf<8> { static constexpr int TC = 4; };

template <int P, typename T>
__global__ __launch_bounds__(256) void k_apply2d(FineOp op, Ref1D ref, const cx<T> *__restrict__ u,
                                                 const cx<T> *__restrict__ f,
                                                 cx<T> *__restrict__ out, T sgn) {
  constexpr int TC = TileOf<P>::TC;
  constexpr int NP = P + 1;
  constexpr int NROW = (TC + 1) * P + 1;
  constexpr int NCC = TC + 1;
  __shared__ cx<T> WX[NROW * NCC * NP];
  __shared__ cx<T> ZX[NROW * NCC * NP];
  __shared__ T sK[NP * NP], sM[NP * NP];

  const int N = op.N, n1 = op.n1;
  const long long rb = (long long)blockIdx.z * op.nf;
  u += rb;
  out += rb;
  if (f) f += rb;

  const int cx0 = blockIdx.x * TC, cy0 = blockIdx.y * TC;
  const int cxs = max(cx0 - 1, 0), cxe = min(cx0 + TC, N);
  const int cys = max(cy0 - 1, 0), cye = min(cy0 + TC, N);
  const int ncx = cxe - cxs;
  const int nrow = (cye - cys) * P + 1;

  for (int i = threadIdx.x; i < NP * NP; i += blockDim.x) {
    sK[i] = (T)ref.K[i];
    sM[i] = (T)ref.M[i];
  }

  // x pass
  for (int it = threadIdx.x; it < nrow * ncx; it += blockDim.x) {
    const int jr = it / ncx, cc = it - jr * ncx;
    const int jy = cys * P + jr, c = cxs + cc;
    const cx<T> *urow = u + (long long)jy * n1 + c * P;
    cx<T> uv[NP];
#pragma unroll
    for (int b = 0; b < NP; ++b) uv[b] = urow[b];
#pragma unroll
    for (int a = 0; a < NP; ++a) {
      cx<T> w = {0, 0}, z = {0, 0};
#pragma unroll
      for (int b = 0; b < NP; ++b) {
        rmac(w, (T)ref.M[a * NP + b], uv[b]);
        rmac(z, (T)ref.K[a * NP + b], uv[b]);
      }
      WX[(jr * NCC + cc) * NP + a] = w;
      ZX[(jr * NCC + cc) * NP + a] = z;
    }
  }
  __syncthreads();

  // y pass over owned nodes
  const int NPn = N * P;
  const int ix0 = cx0 * P, iy0 = cy0 * P;
  const int ix1 = (cx0 + TC >= N) ? NPn + 1 : (cx0 + TC) * P;
  const int iy1 = (cy0 + TC >= N) ? NPn + 1 : (cy0 + TC) * P;
  const int nox = ix1 - ix0, noy = iy1 - iy0;
  const T h = (T)op.h, h2 = (T)(op.h * op.h);

  for (int it = threadIdx.x; it < nox * noy; it += blockDim.x) {
    const int jy = it / nox, jx = it - jy * nox;
    const int ix = ix0 + jx, iy = iy0 + jy;
    const int chx = min(ix / P, N - 1), chy = min(iy / P, N - 1);
    const int ncellx = (ix % P == 0 && ix > 0 && ix < NPn) ? 2 : 1;
    const int ncelly = (iy % P == 0 && iy > 0 && iy < NPn) ? 2 : 1;
    cx<T> acc = {0, 0};
    for (int qy = ncelly - 1; qy >= 0; --qy) {
      const int cyq = chy - qy;
      const int ay = iy - cyq * P;
      const int rbase = (cyq - cys) * P;
      for (int qx = ncellx - 1; qx >= 0; --qx) {
        const int cxq = chx - qx;
        const int ax = ix - cxq * P;
        const int cc = cxq - cxs;
        const c64 kd = op.kap[(long long)cyq * N + cxq];
        const cx<T> kh = {(T)kd.re * h2, (T)kd.im * h2};
#pragma unroll
        for (int by = 0; by < NP; ++by) {
          const cx<T> w = WX[((rbase + by) * NCC + cc) * NP + ax];
          const cx<T> z = ZX[((rbase + by) * NCC + cc) * NP + ax];
          const T ky = sK[ay * NP + by], my = sM[ay * NP + by];
          rmac(acc, ky, w);
          cx<T> t = z - kh * w;
          rmac(acc, my, t);
        }
      }
    }
    // absorbing boundary terms: -i k h (M1 along the side) u
    if (op.robin) {
      cx<T> s = {0, 0};
      if ((ix == 0 && (op.robin & 1)) || (ix == NPn && (op.robin & 2))) {
        const int cxq = (ix == 0) ? 0 : N - 1;
        for (int qy = ncelly - 1; qy >= 0; --qy) {
          const int cyq = chy - qy, ay = iy - cyq * P;
          const T kk = (T)op.kr[(long long)cyq * N + cxq];
          cx<T> m = {0, 0};
          for (int by = 0; by < NP; ++by)
            rmac(m, sM[ay * NP + by], u[(long long)(cyq * P + by) * n1 + ix]);
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
            rmac(m, sM[ax * NP + bx], u[(long long)iy * n1 + cxq * P + bx]);
          rmac(s, kk, m);
        }
      }
      // -i h s = (h s.im, -h s.re)
      acc.re += h * s.im;
      acc.im -= h * s.re;
    }
    const long long g = (long long)iy * n1 + ix;
    cx<T> o = f ? f[g] : cx<T>{0, 0};
    o.re = fma(sgn, acc.re, o.re);
    o.im = fma(sgn, acc.im, o.im);
    out[g] = o;
  }
}

template <int P, typename T>
static int launch_apply_t(const FineOp &op, const Ref1D &ref, const void *u, const void *f,
                          void *out, int nrhs, double sgn, hipStream_t s) {
  constexpr int TC = TileOf<P>::TC;
  dim3 grid(ceil_div(op.N, TC), ceil_div(op.N, TC), nrhs);
  hipLaunchKernelGGL((k_apply2d<P, T>), grid, dim3(256), 0, s, op, ref, (const cx<T> *)u,
                     (const cx<T> *)f, (cx<T> *)out, (T)sgn);
  TH_HIP_CHECK_RET(hipGetLastError());
  return 0;
}

int launch_apply(const FineOp &op, const Ref1D &ref, const void *u, const void *f, void *out,
                 int nrhs, bool f32, double sgn, hipStream_t s) {
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
