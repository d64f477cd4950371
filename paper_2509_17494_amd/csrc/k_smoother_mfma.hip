// Batched subdomain solves on the matrix cores (BF16 storage, FP32
// accumulation) for many right-hand sides: Y_i = B_i X_i for all subdomains
// and all right-hand sides in one launch (Alg. 2 with n_dd = 1: w_i =
// (A_s^(i))^{-1} R_i r, pre-weighted by 1/L_j as in the FP64 path).
//
// B_i (n_U x n_Omega complex) is stored as BF16 re/im planes in the operand
// layout of v_mfma_f32_16x16x32_bf16: for every 16-row block rb and 32-column
// block kb, 2 planes x 64 lanes x 8 values, lane l holding row rb*16 + l%16,
// columns kb*32 + (l/16)*8 + [0, 8).  A wavefront therefore loads each operand
// fragment as one contiguous 1 KiB.  X_i is gathered from the residual,
// rounded to BF16 and staged in LDS per chunk of columns as re/im planes
// [rhs][k] (row stride padded against bank conflicts).  A complex product is
// four real MFMAs: Re += Br Xr + (-Bi) Xi, Im += Br Xi + Bi Xr.
//
// The grid is persistent: every workgroup loops over (subdomain, group of
// row blocks) work items, so the launch holds all subdomains and all
// right-hand sides; the waves per workgroup, the column chunk and the grid
// size are tunables chosen by the setup autotuner.
#include "ctx.hpp"

namespace th {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int MF_KB = 32;        // columns per MFMA step
constexpr int MF_RB = 16;        // rows per MFMA tile
constexpr int MF_NT = 16;        // right-hand sides per MFMA tile
constexpr int MF_RHS_GROUP = 64; // right-hand sides staged together

__device__ __forceinline__ unsigned short f2bf(float x) {
  // round to nearest even (finite inputs)
  unsigned int u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}

// Element offset (in bf16 units) of fragment (rb, kb, plane) of subdomain s.
__host__ __device__ __forceinline__ long long mf_frag(const Sub &s, int rb, int kb, int plane) {
  const int nkb = (s.nOm + MF_KB - 1) / MF_KB;
  return s.boff + (((long long)rb * nkb + kb) * 2 + plane) * 512;
}

template <typename T, int WAVES, int KCH>
__global__ __launch_bounds__(64 * WAVES) void k_dd_mfma(const Sub *__restrict__ subs, int nsub,
                                                        int max_groups,
                                                        const unsigned short *__restrict__ B,
                                                        const cx<T> *__restrict__ r,
                                                        cx<T> *__restrict__ Y, int P, int n1,
                                                        long long nf, long long yrows, int nrhs) {
  constexpr int KC = KCH * MF_KB;       // columns staged per chunk
  constexpr int LDR = KC + 8;           // padded row stride (bf16)
  __shared__ __attribute__((aligned(16))) unsigned short Xs[2][MF_RHS_GROUP][LDR];
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int total = nsub * max_groups;
  for (int item = blockIdx.x; item < total; item += gridDim.x) {
    const int si = item / max_groups, grp = item - si * max_groups;
    const Sub s = subs[si];
    const int nrb = (s.nU + MF_RB - 1) / MF_RB;
    if (grp * WAVES >= nrb) continue;  // uniform over the workgroup
    const int rb = grp * WAVES + wave;
    const bool live = rb < nrb;          // uniform per wavefront
    const int nkb = (s.nOm + MF_KB - 1) / MF_KB;
    for (int r0 = 0; r0 < nrhs; r0 += MF_RHS_GROUP) {
      const int nr = min(MF_RHS_GROUP, nrhs - r0);
      const int ntile = (nr + MF_NT - 1) / MF_NT;
      f32x4 are[MF_RHS_GROUP / MF_NT], aim[MF_RHS_GROUP / MF_NT];
#pragma unroll
      for (int t = 0; t < MF_RHS_GROUP / MF_NT; ++t) {
        are[t] = f32x4{0, 0, 0, 0};
        aim[t] = f32x4{0, 0, 0, 0};
      }
      for (int kb0 = 0; kb0 < nkb; kb0 += KCH) {
        const int k0 = kb0 * MF_KB;
        __syncthreads();
        // stage X chunk: columns [k0, k0 + KC) for the right-hand sides of the
        // ntile MFMA tiles in use; a thread keeps one column (its patch node
        // index computed once) and steps over right-hand sides, consecutive
        // threads take consecutive columns (coalesced loads)
        constexpr int NT = 64 * WAVES;
        constexpr int QG = NT >= KC ? NT / KC : 1;
        const int nrp = ntile * MF_NT;
        for (int t = threadIdx.x; t < KC * QG; t += NT) {
          const int kk = t % KC, qg = t / KC;
          const int k = k0 + kk;
          const bool valid = k < s.nOm;
          const long long g = valid ? om_node(s, k, P, n1) : 0;
          for (int q = qg; q < nrp; q += QG) {
            unsigned short vr = 0, vi = 0;
            if (valid && q < nr) {
              const cx<T> v = r[(long long)(r0 + q) * nf + g];
              vr = f2bf((float)v.re);
              vi = f2bf((float)v.im);
            }
            Xs[0][q][kk] = vr;
            Xs[1][q][kk] = vi;
          }
        }
        __syncthreads();
        if (live) {
          const int kbe = min(KCH, nkb - kb0);
          for (int kq = 0; kq < kbe; ++kq) {
            const unsigned short *fr = B + mf_frag(s, rb, kb0 + kq, 0) + lane * 8;
            const unsigned short *fi = B + mf_frag(s, rb, kb0 + kq, 1) + lane * 8;
            const u32x4 ur = __builtin_nontemporal_load((const u32x4 *)fr);
            const u32x4 ui = __builtin_nontemporal_load((const u32x4 *)fi);
            const u32x4 uin = ui ^ u32x4{0x80008000u, 0x80008000u, 0x80008000u, 0x80008000u};
            const bf16x8 br = __builtin_bit_cast(bf16x8, ur);
            const bf16x8 bi = __builtin_bit_cast(bf16x8, ui);
            const bf16x8 bin = __builtin_bit_cast(bf16x8, uin);
            const int kl = kq * MF_KB + (lane / 16) * 8;
#pragma unroll
            for (int t = 0; t < MF_RHS_GROUP / MF_NT; ++t) {
              if (t < ntile) {
                const int q = t * MF_NT + lane % 16;
                const bf16x8 xr = __builtin_bit_cast(bf16x8, *(const u32x4 *)&Xs[0][q][kl]);
                const bf16x8 xi = __builtin_bit_cast(bf16x8, *(const u32x4 *)&Xs[1][q][kl]);
                are[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(br, xr, are[t], 0, 0, 0);
                are[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bin, xi, are[t], 0, 0, 0);
                aim[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(br, xi, aim[t], 0, 0, 0);
                aim[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bi, xr, aim[t], 0, 0, 0);
              }
            }
          }
        }
      }
      if (live) {
#pragma unroll
        for (int t = 0; t < MF_RHS_GROUP / MF_NT; ++t) {
          const int q = t * MF_NT + lane % 16;
          if (t < ntile && q < nr) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const int row = rb * MF_RB + (lane / 16) * 4 + i;
              if (row < s.nU)
                Y[(long long)(r0 + q) * yrows + s.yoff + row] = cx<T>{(T)are[t][i], (T)aim[t][i]};
            }
          }
        }
      }
    }
  }
}

// Setup: B_i in the MFMA layout from the FP64 inverse (row-major, ld), the
// weights 1/L_j applied, rounded to BF16.  One thread per (rb, kb, lane).
__global__ __launch_bounds__(256) void k_extract_b_mfma(const Sub *__restrict__ subs, int s0,
                                                        const c64 *__restrict__ A, int ld,
                                                        long long stride,
                                                        const int *__restrict__ nblk,
                                                        unsigned short *__restrict__ B, int P) {
  const Sub s = subs[s0 + blockIdx.y];
  const c64 *Ab = A + blockIdx.y * stride;
  const int nrb = (s.nU + MF_RB - 1) / MF_RB, nkb = (s.nOm + MF_KB - 1) / MF_KB;
  const long long nthreads = (long long)nrb * nkb * 64;
  for (long long t = blockIdx.x * 256LL + threadIdx.x; t < nthreads; t += (long long)gridDim.x * 256) {
    const int lane = (int)(t % 64);
    const long long f = t / 64;
    const int kb = (int)(f % nkb), rb = (int)(f / nkb);
    const int row = rb * MF_RB + lane % 16;
    unsigned short vr[8], vi[8];
    for (int e = 0; e < 8; ++e) {
      const int k = kb * MF_KB + (lane / 16) * 8 + e;
      vr[e] = vi[e] = 0;
      if (row < s.nU && k < s.nOm) {
        int gn[3], uj;
        u_node(s, row, P, gn, uj);
        const double invL =
            1.0 / (double)(nblk[2 * gn[0] + 1] * nblk[2 * gn[1] + 1] * nblk[2 * gn[2] + 1]);
        const c64 v = Ab[(long long)uj * ld + k];
        vr[e] = f2bf((float)(v.re * invL));
        vi[e] = f2bf((float)(v.im * invL));
      }
    }
    unsigned short *pr = B + mf_frag(s, rb, kb, 0) + lane * 8;
    unsigned short *pi = B + mf_frag(s, rb, kb, 1) + lane * 8;
    for (int e = 0; e < 8; ++e) {
      pr[e] = vr[e];
      pi[e] = vi[e];
    }
  }
}

int launch_extract_b_mfma(const th_ctx *c, int s0, int nb, const c64 *work, int ld,
                          long long stride, hipStream_t s) {
  hipLaunchKernelGGL(k_extract_b_mfma, dim3(512, nb), dim3(256), 0, s, c->d_subs, s0, work, ld,
                     stride, c->d_nblk, (unsigned short *)c->d_B, c->P);
  TH_HIP_CHECK_RET(hipGetLastError());
  return 0;
}

long long mfma_store_elems(const Sub &s) {
  const long long nrb = (s.nU + MF_RB - 1) / MF_RB, nkb = (s.nOm + MF_KB - 1) / MF_KB;
  return nrb * nkb * 2 * 512;
}

template <typename T, int WAVES, int KCH>
static int launch_mfma_t(const th_ctx *c, const void *r, void *y, int nrhs, int grid,
                         hipStream_t s) {
  int max_nrb = 0;
  for (const Sub &sb : c->subs) max_nrb = std::max(max_nrb, (sb.nU + MF_RB - 1) / MF_RB);
  const int max_groups = ceil_div(max_nrb, WAVES);
  const int nsub = (int)c->subs.size();
  const int total = nsub * max_groups;
  const int g = grid > 0 ? std::min(grid, total) : total;
  hipLaunchKernelGGL((k_dd_mfma<T, WAVES, KCH>), dim3(g), dim3(64 * WAVES), 0, s, c->d_subs, nsub,
                     max_groups, (const unsigned short *)c->d_B, (const cx<T> *)r, (cx<T> *)y,
                     c->P, c->n1, c->nf, c->y_rows, nrhs);
  TH_HIP_CHECK_RET(hipGetLastError());
  return 0;
}

// tunable configurations: (waves per workgroup, column blocks per chunk)
static const int kMfmaCfg[][2] = {{4, 4}, {4, 8}, {2, 4}, {8, 4}, {2, 8}};
int mfma_num_configs() { return (int)(sizeof(kMfmaCfg) / sizeof(kMfmaCfg[0])); }

int launch_dd_mfma(const th_ctx *c, const void *r, void *y, int nrhs, bool f32, int cfg, int grid,
                   hipStream_t s) {
#define TH_MF(W, K)                                                                         \
  if (kMfmaCfg[cfg][0] == W && kMfmaCfg[cfg][1] == K)                                     \
    return f32 ? launch_mfma_t<float, W, K>(c, r, y, nrhs, grid, s)                       \
               : launch_mfma_t<double, W, K>(c, r, y, nrhs, grid, s);
  TH_MF(4, 4) TH_MF(4, 8) TH_MF(2, 4) TH_MF(8, 4) TH_MF(2, 8)
#undef TH_MF
  set_error("bad matrix-core smoother configuration");
  return TH_EINVAL;
}

}  // namespace th
