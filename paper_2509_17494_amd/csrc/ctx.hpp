// Library context and internal interfaces between the host code and the
// kernel launchers.
#pragma once

#include <string>
#include <vector>

#include "../../include/th.h"
#include "common.hpp"

namespace th {

// Block width of the batched Gauss-Jordan inversion; matrices handed to it are
// padded to a multiple of this.
constexpr int kGJBlock = 64;

// One subdomain: U = non-overlapping cell box, Om = U plus one cell layer
// clipped to the domain (Sec. 4.1, 4.4).  Boxes are half-open cell ranges.
// In 2-D the z extents are a single node layer (u0z = o0z = 0, nuz = noz = 1),
// so every index formula below serves both dimensions.
struct Sub {
  int u0x, u1x, u0y, u1y, u0z, u1z;  // U cell box
  int o0x, o1x, o0y, o1y, o0z, o1z;  // Omega cell box
  int nux, nuy, nuz, nox, noy, noz;  // node counts of closed U / Omega per direction
  int nU, nOm;                // nodes of closed U / Omega
  int ldb;                    // n_U padded to a multiple of 64 (rows of the stored B_i)
  int robin;                  // bit s set: absorbing term on side s of Omega (x-,x+,y-,y+,z-,z+)
  int dir;                    // bit s set: side s of Omega lies on a Dirichlet side of the domain
  long long boff;             // element offset of B_i in the operator store
  long long yoff;             // offset of this subdomain's rows in the Y scratch
  // symmetric-tile layout (FP64/FP32 operators): 64-row blocks of U, 64-column
  // blocks of the ring Omega \ U, ring node list and partial-sum rows
  int nrb, neb;
  long long eoff;             // offset of the ring node list (Omega-local indices)
  long long poff;             // offset of the transposed-tile partials
  long long xoff;             // offset of the gathered patch (U nodes, then ring nodes; the
                              // slab layout: Omega-local order)
  // slab-factor layout: slabs of P node layers along the slowest axis (y in
  // 2-D, z in 3-D), nodes per layer, and the offset of the coupling bands
  int nsl, lsz;
  long long coff;             // coupling bands (slab layout)
  long long ecoff;            // backward products E_t (slab layout)
};

constexpr int kSymTile = 64;

// Node (or vertex) index i along `axis` of a grid whose last index is `last`
// lies on a Dirichlet side (bit 2 axis: low side, bit 2 axis + 1: high side).
__host__ __device__ __forceinline__ bool on_dir(int dir, int axis, int i, int last) {
  return (i == 0 && ((dir >> (2 * axis)) & 1)) || (i == last && ((dir >> (2 * axis)) & 2));
}

// index of the upper tile (a, b), a <= b, among the nrb (nrb + 1) / 2 upper tiles
__host__ __device__ __forceinline__ int sym_tile(int a, int b, int nrb) {
  return a * nrb - a * (a - 1) / 2 + (b - a);
}

// global node index of local Omega node k of subdomain s
__host__ __device__ __forceinline__ long long om_node(const Sub &s, int k, int P, int n1) {
  const int kx = k % s.nox, t = k / s.nox;
  const int ky = t % s.noy, kz = t / s.noy;
  return ((long long)(s.o0z * P + kz) * n1 + (s.o0y * P + ky)) * n1 + s.o0x * P + kx;
}

// Local node j of closed U (x fastest): global node coordinates g[] and the
// position uj of the same node in the Omega numbering.
__host__ __device__ __forceinline__ void u_node(const Sub &s, int j, int P, int g[3], int &uj) {
  const int jx = j % s.nux, t = j / s.nux;
  const int jy = t % s.nuy, jz = t / s.nuy;
  g[0] = s.u0x * P + jx;
  g[1] = s.u0y * P + jy;
  g[2] = s.u0z * P + jz;
  uj = (((s.u0z - s.o0z) * P + jz) * s.noy + (s.u0y - s.o0y) * P + jy) * s.nox +
       (s.u0x - s.o0x) * P + jx;
}

// global node index of local node j of closed U
__host__ __device__ __forceinline__ long long u_global(const Sub &s, int j, int P, int n1) {
  int g[3], uj;
  u_node(s, j, P, g, uj);
  return ((long long)g[2] * n1 + g[1]) * n1 + g[0];
}

// Geometry and coefficients of the fine operator, passed to kernels by value.
struct FineOp {
  int dim;
  int N, P, n1;               // cells/dir, order, nodes/dir
  long long nf;               // nodes
  double h;
  int robin;                  // bit s: Robin on global side s (x-,x+,y-,y+,z-,z+)
  int dir;                    // bit s: Dirichlet on global side s (nodes eliminated)
  const c64 *kap;             // per cell volume coefficient (k^2 + i eps) or shifted
  const double *kr;           // per cell k for the absorbing term
};

// Nested-dissection coarse solve: one tree node (device descriptor).  The
// node's vertex list holds I (nI entries) followed by B (nB); its front
// positions (I, then B) carry two extend-add sources (update-vector entries of
// its two children, or -1); [G; -T] is stored column-major with leading
// dimension ldm (rows nI + nB), -W column-major over B with leading dimension
// ldw (rows nI); its own update vector has nB entries at uoff.
struct NDNode {
  int nI, nB, ldm, ldw;
  long long ioff, soff, moff, woff, uoff;
};

// Nodes of one tree level (equal height) and their workgroup tasks.
struct NDLevel {
  int n0 = 0, n1 = 0;     // nodes [n0, n1) in level order
  int f0 = 0, f1 = 0;     // forward tasks (node, first row)
  int b0 = 0, b1 = 0;     // backward tasks
  int maxI = 0, maxB = 0;
  long long fbytes = 0, bbytes = 0;  // factor bytes read by the level's forward / backward step
};

struct NDData {
  int levels = 0, nodes = 0;
  std::vector<NDLevel> lv;
  NDNode *d_nodes = nullptr;
  int *d_idx = nullptr;       // vertex lists (I then B per node)
  int *d_src = nullptr;       // extend-add sources, two per front position
  int2 *d_ftask = nullptr, *d_btask = nullptr;
  c64 *M = nullptr;           // [G; -T] per node
  c64 *Wm = nullptr;          // -W per node
  c64 *uvec = nullptr;        // update vectors [max_rhs][ulen]
  long long ulen = 0, bytes = 0, fwd_bytes = 0, bwd_bytes = 0;
  // iterative refinement: x += A_c^{-1}(r - A_c x) repeated `refine` times
  // for an exact solve (th_coarse_solve, th_twogrid), `refine_pc` times inside
  // the FP64 preconditioner of th_solve, with the stencil kept on the device
  // and two coarse work vectors per RHS
  int refine = 0, refine_pc = 0;
  c64 *st = nullptr;
  c64 *t = nullptr, *d = nullptr;
};

// The coarse grid is ordered in slabs along the slowest axis (lines of
// constant y in 2-D, planes of constant z in 3-D).  Every vertex couples to
// the previous / same / next slab through C = 3^(d-1) in-slab offsets.
struct CoarseData {
  int dim = 2;
  int nx = 0;                 // vertices per grid direction
  int L = 0;                  // vertices per slab (nx or nx^2)
  int ny = 0;                 // slabs
  int C = 3;                  // in-slab couplings per vertex (3 or 9)
  int nblk = 0;               // super-blocks of consecutive slabs
  int rc_chunk = 1;           // right-hand sides per sweep pass
  int mid = -1;               // twisted elimination: meeting super-block (-1: top-down only)
  std::vector<int> line0;     // first slab of every super-block (nblk + 1 entries)
  std::vector<int> ld;        // padded leading dimension of G_J
  std::vector<long long> goff;  // element offset of G_J
  c64 *G = nullptr;           // inverses of the Schur blocks S_J (symmetric), row-major
  c64 *st = nullptr;          // per vertex 3 x C couplings [slab offset + 1][in-slab code]
  c64 *tbuf = nullptr;        // staging of slab right-hand sides for large slabs
  c64 *pbuf = nullptr;        // column-chunk partial sums of the large-slab GEMV
  long long bytes = 0;
  int kind = 0;               // 0: block elimination over slabs, 1: nested dissection
  NDData nd;
  double check_err = -1.0;    // max |A_c^{-1} (A_c x) - x| of the setup probe (unit entries)
  double check_err_pc = -1.0; // the same at the preconditioner's refinement
};

}  // namespace th

struct th_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;

  bool fine_ready = false, coarse_ready = false;
  th_fine_desc desc{};
  int dim = 2, N = 0, P = 0, R = 0, n1 = 0, nc1 = 0;
  long long nf = 0, nc = 0;
  double h = 0;
  th::Ref1D ref{};

  // per-cell data
  th::c64 *d_kap = nullptr;    // k^2 + i eps
  th::c64 *d_kaps = nullptr;   // k^2 (1 + i alpha_s) + i eps
  double *d_k = nullptr;       // k
  std::vector<double> h_k, h_eps;

  // subdomains
  int dir = 0;                 // bit s: Dirichlet on global side s
  int max_nsl = 0;             // slab layout: most slabs of a subdomain
  int max_slab_rows = 0;       // slab layout: largest slab
  int slab_pk = 0;             // slab layout: G_t stored packed (lower block triangle)
  void *w_z = nullptr;         // slab layout: per-subdomain solutions [R][x_rows]
  int M = 0;                   // blocks per direction
  std::vector<int> blk_start;  // M+1 cell starts
  std::vector<th::Sub> subs;
  th::Sub *d_subs = nullptr;
  int *d_nblk = nullptr;       // per node index along an axis: first block, count (2 ints)
  void *d_B = nullptr;         // operator store (layout depends on gemm)
  long long b_entries = 0, b_bytes = 0, y_rows = 0;
  int layout = 0;              // 0 dense 64-row blocks, 1 symmetric tiles, 2 matrix-core BF16,
                               // 3 slab factors
  int *d_eidx = nullptr;       // ring node lists (symmetric layout)
  long long p_rows = 0;        // partial-sum rows per right-hand side (symmetric layout)
  long long x_rows = 0;        // gathered patch rows per right-hand side (symmetric layout)
  int max_pairs = 0;           // largest number of 64-row block pairs of a subdomain
  int max_ldb = 0, max_nom = 0, max_rowblocks = 0;

  // workspaces (fine vectors of max_rhs, both precisions as needed)
  void *w_r = nullptr;         // residual
  void *w_v = nullptr;         // DD update accumulator (n_dd > 1)
  void *w_rr = nullptr;        // shifted residual (n_dd > 1)
  void *w_y = nullptr;         // Y scratch [rhs][y_rows]
  void *w_rc = nullptr;        // coarse rhs (FP64)
  void *w_uc = nullptr;        // coarse solution (FP64)
  void *w_t = nullptr;         // coarse sweep temporaries
  void *w_p = nullptr;         // transposed-tile partial sums (symmetric layout)
  void *w_x = nullptr;         // gathered patches X_i (symmetric layout)
  void *w_yc = nullptr;        // colour planes [2^d][rhs][n_fine] of the staged matrix-core kernel
  void *w_xp = nullptr;        // BF16 patch fragments of the two-pass matrix-core kernel
  int mfx_max_nrb = 0;         // most 16-row blocks of a subdomain (staged matrix-core kernel)
  bool mfx_ok = false;         // patches fit the staged kernel's LDS
  size_t ws_bytes = 0;

  th::CoarseData coarse;
  void *noalloc_scratch = nullptr;  // this device's address of the no-allocation scratch array

  // solver workspaces (allocated lazily by th_solve)
  void *s_buf = nullptr;
  size_t s_bytes = 0;
  void *h_pinned = nullptr;    // pinned host staging of the Hessenberg column
  size_t h_pinned_bytes = 0;
  // Krylov basis V and preconditioned directions Z: blocks of a fixed number
  // of vectors (max_rhs x n_fine complex128 each), allocated as the Arnoldi
  // process reaches them and kept for later solves
  std::vector<void *> kv_V, kv_Z;
  size_t kv_vec_bytes = 0;

  // captured preconditioner graphs: (nrhs, f32, input, output) -> executable
  struct PrecGraph {
    int nrhs;
    bool f32;
    const void *in;
    void *out;
    hipGraphExec_t exec;
  };
  std::vector<PrecGraph> graphs;
  long long graph_launches = 0;

  double t_setup_fine = 0, t_setup_coarse = 0, t_stencil = 0;
  int n_fallback = 0;

  // matrix-core smoother tunables (chosen by the setup autotuner)
  int mfma_cfg = 0, mfma_grid = 0;
  std::string tune_report;

  // kernel timing (measurement only)
  bool timing = false;
  std::vector<hipEvent_t> ev_pool;                  // reusable events
  size_t ev_used = 0;
  std::vector<std::pair<int, std::pair<size_t, size_t>>> ev_marks;  // class, (start, stop)
};

namespace th {
// Records events around a launch sequence of one kernel class while timing is on.
struct KTimer {
  th_ctx *c;
  int cls;
  size_t start = (size_t)-1;
  KTimer(th_ctx *ctx, int k);
  ~KTimer();
};
}  // namespace th

namespace th {

// thread-local error text written by internal functions
void set_error(const std::string &msg);
const std::string &get_error();

// ref1d.cpp
void make_ref1d(int p, Ref1D &ref);
void gll_points(int p, std::vector<double> &x, std::vector<double> &w);

// k_operator.hip: out = f + sgn * (A u)   (f may be null); A carries unit rows
// and columns on the Dirichlet nodes (op.dir): u is read as zero there and
// out = f + sgn u.
int launch_apply(const FineOp &op, const Ref1D &ref, const void *u, const void *f, void *out,
                 int nrhs, bool f32, double sgn, hipStream_t s);

// k_transfer.hip; f32: complex64 fine vectors; coarse64: the coarse vector is
// complex128 even then (the two-grid step hands it to the FP64 coarse solve)
int launch_restrict(int dim, int N, int P, int dir, const Ref1D &ref, const void *r, void *rc, int nrhs,
                    bool f32, hipStream_t s, bool coarse64 = false);
int launch_prolong(int dim, int N, int P, int dir, const Ref1D &ref, const void *uc, void *u, double omega,
                   int nrhs, bool f32, hipStream_t s, bool coarse64 = false);

// k_smoother.hip
int launch_dd_apply(const th_ctx *c, const void *r, void *y, int nrhs, bool f32, hipStream_t s);
// right-hand sides of the gathered patches of the FP64 matrix-core apply (dense
// layout), 0 when max_rhs is below its threshold
int dd_mfma64_rhs_pad(int max_rhs);
// k_slab.hip: the slab-factor layout (apply, and its setup from the assembled
// subdomain matrices of one batch)
int launch_dd_slab(const th_ctx *c, const void *r, void *y, int nrhs, bool f32, hipStream_t s);
// packed slab factors: LDS bytes of the forward sweep for rhs_bytes bytes of
// right-hand sides per row (at most kSlabPkLds), and the largest slab
constexpr size_t kSlabPkLds = 64 * 1024;
size_t slab_pk_lds(const th_ctx *c, size_t rhs_bytes);
int slab_pk_max_rows();
int setup_slab_factors(th_ctx *c, int s0, int nb, const c64 *A, int npad, long long amat,
                       c64 *const W[3], c64 *T1, int ldw, int ldt, c64 *pws, hipStream_t s);
int launch_dd_accumulate(const th_ctx *c, const void *y, void *u, int nrhs, bool f32, bool assign,
                         hipStream_t s);

// k_dense.hip (setup)
int setup_subdomain_operators(th_ctx *c);

// k_smoother_mfma.hip
int launch_extract_b_mfma(const th_ctx *c, int s0, int nb, const c64 *work, int ld,
                          long long stride, hipStream_t s);
long long mfma_store_elems(const Sub &s);
int mfma_num_configs();
bool mfma_cfg_staged(int cfg);          // staged or two-pass form (colour-plane output)
bool mfma_cfg_twopass(int cfg);         // two-pass form (patch fragments gathered first)
bool mfma_cfg_usable(const th_ctx *c, int cfg);  // its workspaces exist and its limits hold
int mfp_tiles(int max_rhs);             // tiles of 16 right-hand sides of the patch fragments
long long mfp_patch_elems(const Sub &s, int max_rhs);  // bf16 elements of one patch's fragments
int mfx_rhs_group(int max_rhs);         // right-hand sides staged together by the staged kernel
bool mfx_fits(int max_rhs, int max_nom);  // patches small enough for the staged kernel
int launch_dd_accum_col(const th_ctx *c, void *u, int nrhs, bool f32, bool assign, hipStream_t s);
int launch_dd_mfma(const th_ctx *c, const void *r, void *y, int nrhs, bool f32, int cfg, int grid,
                   hipStream_t s);

// autotune.cpp
int autotune_mfma(th_ctx *c);

// dispersion.cpp (3-D compact stencil)
void fit27_from_radii(double eta, const double z[3], double qw[4]);
void plain_fit27_batch(const double *x, int n, double *e_out, double *q_out);

// mlp_api.cpp
int coarse_weights(int dim, int scheme, const th_mlp *m, double tau, const double *samples, int n,
                   double *q_out, int *n_fallback);

// k_coarse.hip
int setup_coarse_factors(th_ctx *c, const std::vector<c64> &stencil);
// Work vectors of a nested-dissection solve for nrhs right-hand sides: update
// vectors (nrhs x ulen) and the refinement residual and correction (nrhs x
// n_coarse each); null members mean the context's own.
struct CoarseScratch {
  c64 *uvec = nullptr, *t = nullptr, *d = nullptr;
};
// Accuracy asked of a coarse solve: rounded to complex64 afterwards (nested
// dissection skips its refinement), inside the FP64 preconditioner of
// th_solve (refined to a probe error of 1e-8), or exact (th_coarse_solve,
// th_twogrid: refined to the rounding level)
enum CoarseAccuracy { kCoarseRounded = 0, kCoarsePrecond = 1, kCoarseExact = 2 };
int launch_coarse_solve(th_ctx *c, const c64 *rc, c64 *uc, int nrhs, hipStream_t s, int accuracy,
                        const CoarseScratch *ws = nullptr);
// true when the line elimination's solve needs its large-slab staging buffers
bool coarse_lines_need_staging(const th_ctx *c);
// k_nd.hip: nested-dissection factorisation of the coarse stencil matrix, its
// solve, and the probe check of whichever coarse factorisation is set up
int setup_coarse_nd(th_ctx *c, const std::vector<c64> &stencil);
int launch_coarse_nd(const th_ctx *c, const c64 *rc, c64 *uc, int nrhs, hipStream_t s, int accuracy,
                     const CoarseScratch *ws);
void free_nd(NDData &nd);
int coarse_probe_check(th_ctx *c, const std::vector<c64> &stencil, double *err);
// modelled solve times (s) of both coarse factorisations for the context's grid
double coarse_model_lines(const th_ctx *c);
double coarse_model_nd(const th_ctx *c);
int gj_invert_batched(c64 *A, int n, int ld, long long stride, int batch, hipStream_t s,
                      c64 *ws);
// work space of gj_invert_batched for batches of up to `batch` matrices of size <= n:
// status words, inverted diagonal blocks, check vectors
size_t gj_ws_bytes(int batch, int n);
int gj_ws_reset(c64 *ws, hipStream_t s);   // clears the status words (before the first call)
// synchronises; TH_ENUMERIC (with the message naming `what`) when a pivot was zero, not
// finite or relatively small, or an inverse failed its one-vector check
int gj_ws_status(const c64 *ws, hipStream_t s, const char *what);

// k_blas.hip
int launch_convert(const void *in, void *out, long long n, bool in_f32, bool out_f32, hipStream_t s);
// the Arnoldi step's fused pair: partial dot products, then the axpy (or the
// normalisation) that finishes their sum itself and stores it
// One modified Gram-Schmidt step of the Arnoldi process in one launch (one
// workgroup per right-hand side): w -= sum_i h_i V_i in order with
// h_i = conj(V_i) . w into hcol[i][rhs], ||w||^2 into hcol[nv][rhs], w
// normalised.  For nrhs >= kMgsMinRhs, nv <= kMgsMax, n <= 18432 entries.
constexpr int kMgsMax = 32;
constexpr int kMgsMinRhs = 8;
struct MgsBasis {
  const c64 *v[kMgsMax];
};
bool mgs_step_fits(long long n, int nrhs, int nv);
int launch_mgs_step(const MgsBasis &B, int nv, c64 *w, c64 *hcol, long long n, int nrhs,
                    long long ld, hipStream_t s);
int launch_dot_partial(const c64 *x, const c64 *y, long long n, int nrhs, long long ldx,
                       long long ldy, c64 *partial, hipStream_t s);
int launch_axpy_partials(c64 *y, const c64 *x, const c64 *partial, c64 *coef, double sign,
                         long long n, int nrhs, long long ldy, long long ldx, hipStream_t s);
int launch_scale_partials(c64 *v, const c64 *partial, c64 *dot, long long n, int nrhs,
                          long long ld, hipStream_t s);
// the axpy of one projection fused with the partial dot products of the next
// (z = y: the squared norm); pin and pout are distinct partial buffers
int launch_axpy_dot_partials(c64 *y, const c64 *x, const c64 *z, const c64 *pin, c64 *coef,
                             double sign, long long n, int nrhs, long long ld, c64 *pout,
                             hipStream_t s);
int launch_dot(const c64 *x, const c64 *y, long long n, int nrhs, long long ldx, long long ldy,
               c64 *out, c64 *partial, hipStream_t s);
int launch_axpy_dev(c64 *y, const c64 *x, const c64 *coef, double sign, long long n, int nrhs,
                    long long ldy, long long ldx, hipStream_t s);
int launch_scale_dev(c64 *y, const c64 *x, const double *inv_norm, long long n, int nrhs,
                     long long ldy, long long ldx, hipStream_t s);
int launch_lincomb(c64 *x, const c64 *Z, const c64 *coef, int mcount, int cstride, long long n,
                   int nrhs, long long ldz_j, long long ldz_r, hipStream_t s);
int launch_add(void *u, const void *v, long long n_complex, bool f32, hipStream_t s);
int launch_inv_norm(const c64 *dots, double *inv, int n, hipStream_t s);
int launch_nan_check(const c64 *x, long long n, int *flag, hipStream_t s);

}  // namespace th
