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
//
// Staged form (k_dd_mfx, for patches small enough to sit in LDS whole: n_Omega
// up to 448 columns with 64 right-hand sides, 896 with 32, 1792 with 16): one
// workgroup per (subdomain, group of row blocks).  Each wavefront first
// issues the loads of its first operand fragments, then the whole workgroup
// gathers the patch X_i once (node offsets from an LDS table, two columns per
// thread, rounded to BF16) into LDS planes [plane][rhs][k] (row stride
// n_Omega + 8: conflict-free 16-byte fragment reads), and after one barrier
// every wavefront streams its row blocks' fragments from memory, four deep in
// registers, through the MFMAs.  The workgroups of one subdomain are g * nsub
// + si, so with nsub a multiple of 8 they land on the same XCD and share its
// L2 for the patch.  Results go to the colour planes of the Y scratch: plane
// c = parity of the subdomain's block index per direction, at the global node
// position, so that subdomains of one colour never share a node and the
// averaged update reads every contribution with coalesced loads.
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

// ---------------------------------------------------------------------------
// Staged form.
constexpr int MFX_LDS_ELEMS = 2 * 64 * 456;  // bf16 elements of the staged patch planes
constexpr int MFX_KMAX = 1792;               // largest staged patch (columns)
constexpr int MFX_PF = 4;                    // operand fragments in flight per wavefront

// Columns of the largest patch the staged form holds for RHSG right-hand sides.
__host__ __device__ constexpr int mfx_kcap(int rhsg) {
  return ((MFX_LDS_ELEMS / (2 * rhsg) - 8) / MF_KB) * MF_KB < MFX_KMAX
             ? ((MFX_LDS_ELEMS / (2 * rhsg) - 8) / MF_KB) * MF_KB
             : MFX_KMAX;
}

template <typename T, int WAVES, int RHSG>
__global__ __launch_bounds__(64 * WAVES) void k_dd_mfx(const Sub *__restrict__ subs, int nsub,
                                                       int rbg, int M,
                                                       const unsigned short *__restrict__ B,
                                                       const cx<T> *__restrict__ r,
                                                       cx<T> *__restrict__ Yc, int P, int n1,
                                                       long long nf, int nrhs) {
  constexpr int NT = 64 * WAVES, NTILE = RHSG / MF_NT;
  __shared__ __attribute__((aligned(16))) unsigned short Xs[MFX_LDS_ELEMS];
  __shared__ int gofs[MFX_KMAX];
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int si = blockIdx.x % nsub, grp = blockIdx.x / nsub;
  const Sub s = subs[si];
  const int nrb = (s.nU + MF_RB - 1) / MF_RB;
  const int rb0 = grp * rbg, rb1 = min(nrb, rb0 + rbg);
  if (rb0 >= rb1) return;  // uniform over the workgroup
  const int nkb = (s.nOm + MF_KB - 1) / MF_KB, K = nkb * MF_KB, LD = K + 8;
  const long long base = om_node(s, 0, P, n1);
  for (int k = threadIdx.x; k < K; k += NT)
    gofs[k] = k < s.nOm ? (int)(om_node(s, k, P, n1) - base) : -1;
  const int bx = si % M, by = (si / M) % M, bz = si / (M * M);
  const int color = (bx & 1) | ((by & 1) << 1) | ((bz & 1) << 2);
  // this wavefront's row blocks rb0 + wave + j WAVES, flattened with the column blocks
  const int nmine = (rb0 + wave < rb1) ? (rb1 - rb0 - wave + WAVES - 1) / WAVES : 0;
  const int nit = nmine * nkb;
  auto frag = [&](int it, int plane) {
    const int rb = rb0 + wave + (it / nkb) * WAVES, kb = it % nkb;
    return (const u32x4 *)(B + mf_frag(s, rb, kb, plane) + lane * 8);
  };
  for (int r0 = 0; r0 < nrhs; r0 += RHSG) {
    const int nr = min(RHSG, nrhs - r0);
    u32x4 fr[MFX_PF], fi[MFX_PF];
#pragma unroll
    for (int j = 0; j < MFX_PF; ++j)
      if (j < nit) {
        fr[j] = __builtin_nontemporal_load(frag(j, 0));
        fi[j] = __builtin_nontemporal_load(frag(j, 1));
      }
    __syncthreads();  // offset table written; the previous group's reads of Xs done
    // gather X_i: two consecutive columns per thread, right-hand sides slowest
    const cx<T> *rg = r + (long long)r0 * nf + base;
    for (int t = threadIdx.x; t < (K / 2) * RHSG; t += NT) {
      const int k = 2 * (t % (K / 2)), q = t / (K / 2);
      unsigned int vr = 0, vi = 0;
      if (q < nr) {
        const int g0 = gofs[k], g1 = gofs[k + 1];
        const cx<T> a = g0 >= 0 ? rg[(long long)q * nf + g0] : cx<T>{0, 0};
        const cx<T> b = g1 >= 0 ? rg[(long long)q * nf + g1] : cx<T>{0, 0};
        vr = (unsigned int)f2bf((float)a.re) | ((unsigned int)f2bf((float)b.re) << 16);
        vi = (unsigned int)f2bf((float)a.im) | ((unsigned int)f2bf((float)b.im) << 16);
      }
      *(unsigned int *)&Xs[(long long)q * LD + k] = vr;
      *(unsigned int *)&Xs[(long long)(RHSG + q) * LD + k] = vi;
    }
    __syncthreads();
    f32x4 are[NTILE], aim[NTILE];
    for (int it0 = 0; it0 < nit; it0 += MFX_PF) {
#pragma unroll
      for (int j = 0; j < MFX_PF; ++j) {
        const int it = it0 + j;
        if (it < nit) {  // uniform per wavefront
          const int kb = it % nkb;
          if (kb == 0) {
#pragma unroll
            for (int t = 0; t < NTILE; ++t) {
              are[t] = f32x4{0, 0, 0, 0};
              aim[t] = f32x4{0, 0, 0, 0};
            }
          }
          const u32x4 uin = fi[j] ^ u32x4{0x80008000u, 0x80008000u, 0x80008000u, 0x80008000u};
          const bf16x8 br = __builtin_bit_cast(bf16x8, fr[j]);
          const bf16x8 bi = __builtin_bit_cast(bf16x8, fi[j]);
          const bf16x8 bin = __builtin_bit_cast(bf16x8, uin);
          const int kl = kb * MF_KB + (lane / 16) * 8;
#pragma unroll
          for (int t = 0; t < NTILE; ++t) {
            const int q = t * MF_NT + lane % 16;
            const bf16x8 xr = __builtin_bit_cast(bf16x8, *(const u32x4 *)&Xs[(long long)q * LD + kl]);
            const bf16x8 xi =
                __builtin_bit_cast(bf16x8, *(const u32x4 *)&Xs[(long long)(RHSG + q) * LD + kl]);
            are[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(br, xr, are[t], 0, 0, 0);
            are[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bin, xi, are[t], 0, 0, 0);
            aim[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(br, xi, aim[t], 0, 0, 0);
            aim[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bi, xr, aim[t], 0, 0, 0);
          }
          if (it + MFX_PF < nit) {
            fr[j] = __builtin_nontemporal_load(frag(it + MFX_PF, 0));
            fi[j] = __builtin_nontemporal_load(frag(it + MFX_PF, 1));
          }
          if (kb == nkb - 1) {
            const int rb = rb0 + wave + (it / nkb) * WAVES;
            long long gn[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const int row = rb * MF_RB + (lane / 16) * 4 + i;
              gn[i] = row < s.nU ? u_global(s, row, P, n1) : -1;
            }
#pragma unroll
            for (int t = 0; t < NTILE; ++t) {
              const int q = t * MF_NT + lane % 16;
              if (q < nr) {
                cx<T> *yq = Yc + ((long long)color * nrhs + r0 + q) * nf;
#pragma unroll
                for (int i = 0; i < 4; ++i)
                  if (gn[i] >= 0) yq[gn[i]] = cx<T>{(T)are[t][i], (T)aim[t][i]};
              }
            }
          }
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Two-pass form (any patch size): a gather pass rounds every patch X_i to BF16
// once and stores it in the B-operand layout of v_mfma_f32_16x16x32_bf16 --
// for every subdomain, 32-column block kb and tile of 16 right-hand sides,
// re and im planes of 64 lanes x 8 values, lane l holding right-hand side
// 16 t + l % 16 and patch columns 32 kb + 8 (l / 16) + [0, 8) -- with one
// thread per (column block, tile, lane) and eight independent loads per
// thread.  The product pass then streams both operands from memory with no
// LDS and no barrier: a workgroup owns one 16-row block of one subdomain, its
// wavefronts one tile of right-hand sides each (the B_i fragment is shared
// through the cache), fragments prefetched PF column blocks ahead; workgroups
// of one subdomain sit on one XCD (its patch stays in one L2).  Results go to
// the colour planes, as in the staged form, in the same MFMA order, so every
// form gives the same bits.
// Gather pass: workgroup (column block kb, subdomain); the 32 patch columns
// of every right-hand side are read with consecutive lanes on consecutive
// columns (coalesced along the patch's grid lines), transposed through LDS,
// rounded to BF16 and written as whole 1 KiB fragment planes.
template <typename T>
__global__ __launch_bounds__(256) void k_mfp_gather(const Sub *__restrict__ subs,
                                                    const cx<T> *__restrict__ r,
                                                    unsigned short *__restrict__ Xp, int P,
                                                    int n1, long long nf, int nrhs, int ntmax) {
  constexpr int QP = 64;  // right-hand sides staged per pass (four tiles)
  __shared__ cx<T> tile[QP][MF_KB + 1];
  __shared__ long long gofs[MF_KB];
  const Sub s = subs[blockIdx.y];
  const int kb = blockIdx.x;
  const int nkb = (s.nOm + MF_KB - 1) / MF_KB;
  if (kb >= nkb) return;  // uniform
  if (threadIdx.x < MF_KB) {
    const int k = kb * MF_KB + threadIdx.x;
    gofs[threadIdx.x] = k < s.nOm ? om_node(s, k, P, n1) : -1;
  }
  const int ntile = (nrhs + MF_NT - 1) / MF_NT;
  for (int q0 = 0; q0 < nrhs; q0 += QP) {
    __syncthreads();  // offsets written; the previous pass's reads of the tile done
    for (int t = threadIdx.x; t < QP * MF_KB; t += 256) {
      const int kk = t % MF_KB, qq = t / MF_KB, q = q0 + qq;
      const long long g = gofs[kk];
      tile[qq][kk] = (q < nrhs && g >= 0) ? r[(long long)q * nf + g] : cx<T>{0, 0};
    }
    __syncthreads();
    // fragment planes of the tiles of this pass: one thread per (tile, lane)
    const int nt = min(QP / MF_NT, ntile - q0 / MF_NT);
    for (int t = threadIdx.x; t < nt * 64; t += 256) {
      const int lane = t % 64, tt = t / 64;
      const int qq = tt * MF_NT + lane % 16, k0 = (lane / 16) * 8;
      u32x4 pr, pi;
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        const cx<T> a = tile[qq][k0 + 2 * h], c = tile[qq][k0 + 2 * h + 1];
        pr[h] = (unsigned int)f2bf((float)a.re) | ((unsigned int)f2bf((float)c.re) << 16);
        pi[h] = (unsigned int)f2bf((float)a.im) | ((unsigned int)f2bf((float)c.im) << 16);
      }
      unsigned short *o = Xp + (((s.xoff + kb) * ntmax + q0 / MF_NT + tt) * 2) * 512 + lane * 8;
      *(u32x4 *)o = pr;
      *(u32x4 *)(o + 512) = pi;
    }
  }
}

template <typename T, int PF>
__global__ __launch_bounds__(256) void k_mfp_gemm(const Sub *__restrict__ subs, int nsub, int nrb,
                                                  const unsigned short *__restrict__ B,
                                                  const unsigned short *__restrict__ Xp,
                                                  cx<T> *__restrict__ Yc, int P, int n1, int M,
                                                  long long nf, int nrhs, int ntmax) {
  // XCD-aware mapping: workgroup b runs on XCD b % 8; subdomain si on XCD si % 8
  const int b = blockIdx.x;
  const int si = (b & 7) + 8 * ((b >> 3) / nrb), rb = (b >> 3) % nrb;
  if (si >= nsub) return;
  const Sub s = subs[si];
  if (rb * MF_RB >= s.nU) return;  // uniform
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int nkb = (s.nOm + MF_KB - 1) / MF_KB, ntile = (nrhs + MF_NT - 1) / MF_NT;
  const int bx = si % M, by = (si / M) % M, bz = si / (M * M);
  const int color = (bx & 1) | ((by & 1) << 1) | ((bz & 1) << 2);
  const u32x4 sgn = u32x4{0x80008000u, 0x80008000u, 0x80008000u, 0x80008000u};
  long long gn[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int row = rb * MF_RB + (lane / 16) * 4 + i;
    gn[i] = row < s.nU ? u_global(s, row, P, n1) : -1;
  }
  for (int t = wave; t < ntile; t += nw) {
    const unsigned short *xb = Xp + ((s.xoff * ntmax + t) * 2) * 512 + lane * 8;
    const long long xstep = (long long)ntmax * 2 * 512;  // next column block
    u32x4 fr[PF], fi[PF], xr[PF], xi[PF];
#pragma unroll
    for (int j = 0; j < PF; ++j)
      if (j < nkb) {
        fr[j] = *(const u32x4 *)(B + mf_frag(s, rb, j, 0) + lane * 8);
        fi[j] = *(const u32x4 *)(B + mf_frag(s, rb, j, 1) + lane * 8);
        xr[j] = *(const u32x4 *)(xb + j * xstep);
        xi[j] = *(const u32x4 *)(xb + j * xstep + 512);
      }
    f32x4 are = {0, 0, 0, 0}, aim = {0, 0, 0, 0};
    for (int k0 = 0; k0 < nkb; k0 += PF) {
#pragma unroll
      for (int j = 0; j < PF; ++j) {
        const int kb = k0 + j;
        if (kb < nkb) {  // uniform
          const bf16x8 br = __builtin_bit_cast(bf16x8, fr[j]);
          const bf16x8 bi = __builtin_bit_cast(bf16x8, fi[j]);
          const bf16x8 bin = __builtin_bit_cast(bf16x8, fi[j] ^ sgn);
          const bf16x8 vr = __builtin_bit_cast(bf16x8, xr[j]);
          const bf16x8 vi = __builtin_bit_cast(bf16x8, xi[j]);
          are = __builtin_amdgcn_mfma_f32_16x16x32_bf16(br, vr, are, 0, 0, 0);
          are = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bin, vi, are, 0, 0, 0);
          aim = __builtin_amdgcn_mfma_f32_16x16x32_bf16(br, vi, aim, 0, 0, 0);
          aim = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bi, vr, aim, 0, 0, 0);
          const int kn = kb + PF;
          if (kn < nkb) {
            fr[j] = *(const u32x4 *)(B + mf_frag(s, rb, kn, 0) + lane * 8);
            fi[j] = *(const u32x4 *)(B + mf_frag(s, rb, kn, 1) + lane * 8);
            xr[j] = *(const u32x4 *)(xb + kn * xstep);
            xi[j] = *(const u32x4 *)(xb + kn * xstep + 512);
          }
        }
      }
    }
    const int q = t * MF_NT + lane % 16;
    if (q < nrhs) {
      cx<T> *yq = Yc + ((long long)color * nrhs + q) * nf;
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (gn[i] >= 0) yq[gn[i]] = cx<T>{(T)are[i], (T)aim[i]};
    }
  }
}

// Two-pass product, one wavefront per 16-row block with all tiles of right-hand
// sides (up to four per pass): the B_i fragment is loaded once and used for
// every tile; a workgroup holds four row blocks of one subdomain.
template <typename T, int PF>
__global__ __launch_bounds__(256) void k_mfp_gemm_all(const Sub *__restrict__ subs, int nsub,
                                                      int ng, const unsigned short *__restrict__ B,
                                                      const unsigned short *__restrict__ Xp,
                                                      cx<T> *__restrict__ Yc, int P, int n1,
                                                      int M, long long nf, int nrhs, int ntmax) {
  constexpr int TT = 4;  // tiles per pass
  const int b = blockIdx.x;
  const int si = (b & 7) + 8 * ((b >> 3) / ng), g = (b >> 3) % ng;
  if (si >= nsub) return;
  const Sub s = subs[si];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int rb = 4 * g + wave;
  if (rb * MF_RB >= s.nU) return;  // uniform per wavefront; no barrier follows
  const int nkb = (s.nOm + MF_KB - 1) / MF_KB, ntile = (nrhs + MF_NT - 1) / MF_NT;
  const int bx = si % M, by = (si / M) % M, bz = si / (M * M);
  const int color = (bx & 1) | ((by & 1) << 1) | ((bz & 1) << 2);
  const u32x4 sgn = u32x4{0x80008000u, 0x80008000u, 0x80008000u, 0x80008000u};
  long long gn[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int row = rb * MF_RB + (lane / 16) * 4 + i;
    gn[i] = row < s.nU ? u_global(s, row, P, n1) : -1;
  }
  const long long xstep = (long long)ntmax * 2 * 512;
  for (int t0 = 0; t0 < ntile; t0 += TT) {
    const int nt = min(TT, ntile - t0);
    const unsigned short *xb = Xp + ((s.xoff * ntmax + t0) * 2) * 512 + lane * 8;
    u32x4 fr[PF], fi[PF], xr[PF][TT], xi[PF][TT];
    auto load = [&](int j, int kb) {
      fr[j] = __builtin_nontemporal_load((const u32x4 *)(B + mf_frag(s, rb, kb, 0) + lane * 8));
      fi[j] = __builtin_nontemporal_load((const u32x4 *)(B + mf_frag(s, rb, kb, 1) + lane * 8));
#pragma unroll
      for (int t = 0; t < TT; ++t)
        if (t < nt) {
          xr[j][t] = *(const u32x4 *)(xb + kb * xstep + t * 1024);
          xi[j][t] = *(const u32x4 *)(xb + kb * xstep + t * 1024 + 512);
        }
    };
#pragma unroll
    for (int j = 0; j < PF; ++j)
      if (j < nkb) load(j, j);
    f32x4 are[TT], aim[TT];
#pragma unroll
    for (int t = 0; t < TT; ++t) {
      are[t] = f32x4{0, 0, 0, 0};
      aim[t] = f32x4{0, 0, 0, 0};
    }
    for (int k0 = 0; k0 < nkb; k0 += PF) {
#pragma unroll
      for (int j = 0; j < PF; ++j) {
        const int kb = k0 + j;
        if (kb < nkb) {  // uniform
          const bf16x8 br = __builtin_bit_cast(bf16x8, fr[j]);
          const bf16x8 bi = __builtin_bit_cast(bf16x8, fi[j]);
          const bf16x8 bin = __builtin_bit_cast(bf16x8, fi[j] ^ sgn);
#pragma unroll
          for (int t = 0; t < TT; ++t)
            if (t < nt) {
              const bf16x8 vr = __builtin_bit_cast(bf16x8, xr[j][t]);
              const bf16x8 vi = __builtin_bit_cast(bf16x8, xi[j][t]);
              are[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(br, vr, are[t], 0, 0, 0);
              are[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bin, vi, are[t], 0, 0, 0);
              aim[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(br, vi, aim[t], 0, 0, 0);
              aim[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bi, vr, aim[t], 0, 0, 0);
            }
          if (kb + PF < nkb) load(j, kb + PF);
        }
      }
    }
#pragma unroll
    for (int t = 0; t < TT; ++t) {
      const int q = (t0 + t) * MF_NT + lane % 16;
      if (t < nt && q < nrhs) {
        cx<T> *yq = Yc + ((long long)color * nrhs + q) * nf;
#pragma unroll
        for (int i = 0; i < 4; ++i)
          if (gn[i] >= 0) yq[gn[i]] = cx<T>{(T)are[t][i], (T)aim[t][i]};
      }
    }
  }
}

// Averaged update from the colour planes: v_j (assign) or u_j += sum over the
// closed U^(i) containing node j of (Y_i)_j, subdomains in ascending order (the
// order of k_dd_accumulate, so both give the same bits).
template <typename T>
__global__ __launch_bounds__(256) void k_dd_accum_col(const int *__restrict__ nblk,
                                                      const cx<T> *__restrict__ Yc,
                                                      cx<T> *__restrict__ u, int n1, long long nf,
                                                      int nrhs, int assign) {
  const long long rhs = blockIdx.y;
  for (long long g = blockIdx.x * (long long)blockDim.x + threadIdx.x; g < nf;
       g += (long long)gridDim.x * blockDim.x) {
    const int ix = (int)(g % n1);
    const long long t = g / n1;
    const int iy = (int)(t % n1), iz = (int)(t / n1);  // iz = 0 in 2-D
    const int bx0 = nblk[2 * ix], nbx = nblk[2 * ix + 1];
    const int by0 = nblk[2 * iy], nby = nblk[2 * iy + 1];
    const int bz0 = nblk[2 * iz], nbz = nblk[2 * iz + 1];
    cx<T> acc = {0, 0};
    for (int bz = bz0; bz < bz0 + nbz; ++bz)
      for (int by = by0; by < by0 + nby; ++by)
        for (int bx = bx0; bx < bx0 + nbx; ++bx) {
          const int color = (bx & 1) | ((by & 1) << 1) | ((bz & 1) << 2);
          acc = acc + Yc[((long long)color * nrhs + rhs) * nf + g];
        }
    cx<T> *up = u + rhs * nf + g;
    *up = assign ? acc : *up + acc;
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

template <typename T, int WAVES>
static int launch_mfx_t(const th_ctx *c, const void *r, int nrhs, int groups, hipStream_t s) {
  const int nsub = (int)c->subs.size();
  const int rbg = ceil_div(c->mfx_max_nrb, groups);
  const dim3 grid(nsub * groups);
  cx<T> *yc = (cx<T> *)c->w_yc;
  const unsigned short *B = (const unsigned short *)c->d_B;
  const cx<T> *rr = (const cx<T> *)r;
  const int rhsg = mfx_rhs_group(c->desc.max_rhs);
  if (rhsg == 16)
    hipLaunchKernelGGL((k_dd_mfx<T, WAVES, 16>), grid, dim3(64 * WAVES), 0, s, c->d_subs, nsub, rbg,
                       c->M, B, rr, yc, c->P, c->n1, c->nf, nrhs);
  else if (rhsg == 32)
    hipLaunchKernelGGL((k_dd_mfx<T, WAVES, 32>), grid, dim3(64 * WAVES), 0, s, c->d_subs, nsub, rbg,
                       c->M, B, rr, yc, c->P, c->n1, c->nf, nrhs);
  else
    hipLaunchKernelGGL((k_dd_mfx<T, WAVES, 64>), grid, dim3(64 * WAVES), 0, s, c->d_subs, nsub, rbg,
                       c->M, B, rr, yc, c->P, c->n1, c->nf, nrhs);
  TH_HIP_CHECK_RET(hipGetLastError());
  return 0;
}

template <typename T, int PF, bool ALL>
static int launch_mfp_t(const th_ctx *c, const void *r, int nrhs, hipStream_t s) {
  const int nsub = (int)c->subs.size();
  const int ntmax = mfp_tiles(c->desc.max_rhs), ntile = ceil_div(nrhs, MF_NT);
  int max_nkb = 0, nrb = 0;
  for (const Sub &sb : c->subs) {
    max_nkb = std::max(max_nkb, (sb.nOm + MF_KB - 1) / MF_KB);
    nrb = std::max(nrb, (sb.nU + MF_RB - 1) / MF_RB);
  }
  const int nw = std::min(4, ntile);
  unsigned short *xp = (unsigned short *)c->w_xp;
  hipLaunchKernelGGL((k_mfp_gather<T>), dim3(max_nkb, nsub), dim3(256), 0, s, c->d_subs,
                     (const cx<T> *)r, xp, c->P, c->n1, c->nf, nrhs, ntmax);
  const int groups = ceil_div(nsub, 8);
  if (ALL) {
    const int ng = ceil_div(nrb, 4);
    hipLaunchKernelGGL((k_mfp_gemm_all<T, PF>), dim3(8 * groups * ng), dim3(256), 0, s,
                       c->d_subs, nsub, ng, (const unsigned short *)c->d_B,
                       (const unsigned short *)xp, (cx<T> *)c->w_yc, c->P, c->n1, c->M, c->nf,
                       nrhs, ntmax);
  } else {
    hipLaunchKernelGGL((k_mfp_gemm<T, PF>), dim3(8 * groups * nrb), dim3(64 * nw), 0, s,
                       c->d_subs, nsub, nrb, (const unsigned short *)c->d_B,
                       (const unsigned short *)xp, (cx<T> *)c->w_yc, c->P, c->n1, c->M, c->nf,
                       nrhs, ntmax);
  }
  TH_HIP_CHECK_RET(hipGetLastError());
  return 0;
}

int mfp_tiles(int max_rhs) { return (max_rhs + MF_NT - 1) / MF_NT; }

// BF16 patch fragments of the two-pass form (bf16 elements)
long long mfp_patch_elems(const Sub &s, int max_rhs) {
  return (long long)((s.nOm + MF_KB - 1) / MF_KB) * mfp_tiles(max_rhs) * 2 * 512;
}

int mfx_rhs_group(int max_rhs) { return max_rhs <= 16 ? 16 : (max_rhs <= 32 ? 32 : 64); }

bool mfx_fits(int max_rhs, int max_nom) {
  return ceil_div(max_nom, MF_KB) * MF_KB <= mfx_kcap(mfx_rhs_group(max_rhs));
}

// tunable configurations: persistent chunked kernel (waves per workgroup,
// column blocks per chunk), then the staged kernel (waves per workgroup,
// workgroups per subdomain)
static const int kMfmaCfg[][2] = {{4, 4}, {4, 8}, {2, 4}, {8, 4}, {2, 8}};
static const int kMfxCfg[][2] = {{4, 4}, {8, 4}, {8, 2}, {4, 5}, {8, 3}, {4, 8}, {8, 1}};
// two-pass form: column blocks prefetched; 0: one wavefront per tile, 1: all tiles per wavefront
static const int kMfpCfg[][2] = {{2, 0}, {4, 0}, {2, 1}};
constexpr int kNumChunked = (int)(sizeof(kMfmaCfg) / sizeof(kMfmaCfg[0]));
constexpr int kNumStaged = (int)(sizeof(kMfxCfg) / sizeof(kMfxCfg[0]));
int mfma_num_configs() { return kNumChunked + kNumStaged + (int)(sizeof(kMfpCfg) / sizeof(kMfpCfg[0])); }
bool mfma_cfg_staged(int cfg) { return cfg >= kNumChunked; }
bool mfma_cfg_twopass(int cfg) { return cfg >= kNumChunked + kNumStaged; }
bool mfma_cfg_usable(const th_ctx *c, int cfg) {
  if (cfg < 0 || cfg >= mfma_num_configs()) return false;
  if (mfma_cfg_twopass(cfg)) return c->w_yc && c->w_xp;
  if (mfma_cfg_staged(cfg)) return c->w_yc && c->mfx_ok;
  return true;
}

int launch_dd_mfma(const th_ctx *c, const void *r, void *y, int nrhs, bool f32, int cfg, int grid,
                   hipStream_t s) {
  if (mfma_cfg_twopass(cfg) && cfg < mfma_num_configs()) {
    if (!c->w_yc || !c->w_xp) {
      set_error("two-pass matrix-core smoother selected without its colour planes");
      return TH_EINVAL;
    }
    const int pf = kMfpCfg[cfg - kNumChunked - kNumStaged][0];
    const bool all = kMfpCfg[cfg - kNumChunked - kNumStaged][1] != 0;
    if (all) return f32 ? launch_mfp_t<float, 2, true>(c, r, nrhs, s) : launch_mfp_t<double, 2, true>(c, r, nrhs, s);
    if (pf == 2) return f32 ? launch_mfp_t<float, 2, false>(c, r, nrhs, s) : launch_mfp_t<double, 2, false>(c, r, nrhs, s);
    return f32 ? launch_mfp_t<float, 4, false>(c, r, nrhs, s) : launch_mfp_t<double, 4, false>(c, r, nrhs, s);
  }
  if (cfg >= kNumChunked && cfg < mfma_num_configs()) {
    if (!c->w_yc || !c->mfx_ok) {
      set_error("staged matrix-core smoother selected without its colour planes or for patches "
                "too large for it");
      return TH_EINVAL;
    }
    const int w = kMfxCfg[cfg - kNumChunked][0], g = kMfxCfg[cfg - kNumChunked][1];
#define TH_MX(W)                                                                         \
  if (w == W) return f32 ? launch_mfx_t<float, W>(c, r, nrhs, g, s)                     \
                         : launch_mfx_t<double, W>(c, r, nrhs, g, s);
    TH_MX(4) TH_MX(8)
#undef TH_MX
  }
#define TH_MF(W, K)                                                                         \
  if (cfg < kNumChunked && kMfmaCfg[cfg][0] == W && kMfmaCfg[cfg][1] == K)                \
    return f32 ? launch_mfma_t<float, W, K>(c, r, y, nrhs, grid, s)                       \
               : launch_mfma_t<double, W, K>(c, r, y, nrhs, grid, s);
  TH_MF(4, 4) TH_MF(4, 8) TH_MF(2, 4) TH_MF(8, 4) TH_MF(2, 8)
#undef TH_MF
  set_error("bad matrix-core smoother configuration");
  return TH_EINVAL;
}

int launch_dd_accum_col(const th_ctx *c, void *u, int nrhs, bool f32, bool assign, hipStream_t s) {
  int blocks = (int)std::min<long long>(ceil_div_ll(c->nf, 256), 65535);
  if (f32)
    hipLaunchKernelGGL((k_dd_accum_col<float>), dim3(blocks, nrhs), dim3(256), 0, s, c->d_nblk,
                       (const cx<float> *)c->w_yc, (cx<float> *)u, c->n1, c->nf, nrhs,
                       assign ? 1 : 0);
  else
    hipLaunchKernelGGL((k_dd_accum_col<double>), dim3(blocks, nrhs), dim3(256), 0, s, c->d_nblk,
                       (const cx<double> *)c->w_yc, (cx<double> *)u, c->n1, c->nf, nrhs,
                       assign ? 1 : 0);
  TH_HIP_CHECK_RET(hipGetLastError());
  return 0;
}

}  // namespace th
