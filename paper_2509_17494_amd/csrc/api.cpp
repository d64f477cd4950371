// Host side of the two-grid library: argument checking, setup orchestration,
// the two-grid step (Alg. 1) and the outer FP64 GMRES.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "ctx.hpp"

namespace th {

static thread_local std::string g_err;
void set_error(const std::string &msg) { g_err = msg; }
const std::string &get_error() { return g_err; }

int hip_fail(hipError_t e, const char *expr, const char *file, int line) {
  char buf[512];
  snprintf(buf, sizeof(buf), "HIP error %d (%s) in %s at %s:%d", (int)e, hipGetErrorString(e), expr,
           file, line);
  g_err = buf;
  return TH_EHIP;
}

static hipEvent_t take_event(th_ctx *c) {
  if (c->ev_used == c->ev_pool.size()) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    c->ev_pool.push_back(e);
  }
  return c->ev_pool[c->ev_used++];
}

KTimer::KTimer(th_ctx *ctx, int k) : c(ctx), cls(k) {
  if (c->timing) {
    start = c->ev_used;
    hipEvent_t e = take_event(c);
    if (e) (void)hipEventRecord(e, c->stream);
    else start = (size_t)-1;
  }
}

KTimer::~KTimer() {
  if (c->timing && start != (size_t)-1) {
    const size_t stop = c->ev_used;
    hipEvent_t e = take_event(c);
    if (!e) return;
    (void)hipEventRecord(e, c->stream);
    c->ev_marks.push_back({cls, {start, stop}});
  }
}

// ---------------------------------------------------------------------------
// QSFEM weights (Sec. 3.2, eq. P_QSFEM and eq. scaling_factor_QSFEM; Sec. 3.3
// element-wise q_gamma): eta = h_c k(c) on the coarse mesh.
static void qsfem_weights(double eta, double q[3]) {
  const double a1 = M_PI / 16.0, a2 = 3.0 * M_PI / 16.0;
  const double c1 = std::cos(eta * std::cos(a1)), s1 = std::cos(eta * std::sin(a1));
  const double c2 = std::cos(eta * std::cos(a2)), s2 = std::cos(eta * std::sin(a2));
  const double den = c2 * s2 * (c1 + s1) - c1 * s1 * (c2 + s2);
  const double P0 = 4.0;
  const double P1 = 2.0 * (c1 * s1 - c2 * s2) / den;
  const double P2 = (c2 + s2 - c1 - s1) / den;
  const double sigma0 = P0 + 4.0 * P1 + 4.0 * P2;  // symbol at xi = 0
  const double Nn = -eta * eta / sigma0;
  q[0] = Nn * P0 / 4.0;
  q[1] = Nn * P1 / 2.0;
  q[2] = Nn * P2;
}

}  // namespace th

using namespace th;

#define TH_TRY(expr)                   \
  do {                                 \
    int _rc = (expr);                  \
    if (_rc) return finish(ctx, _rc);  \
  } while (0)

static th_status finish(th_ctx *ctx, int rc) {
  if (rc && ctx) ctx->err = get_error();
  return (th_status)rc;
}
static th_status fail(th_ctx *ctx, th_status rc, const std::string &msg) {
  if (ctx) ctx->err = msg;
  return rc;
}

static bool is_f32(th_dtype dt) { return dt == TH_C64; }
static size_t csize(bool f32) { return f32 ? sizeof(c32) : sizeof(c64); }

static FineOp make_op(const th_ctx *c, bool shifted) {
  FineOp op;
  op.dim = c->dim;
  op.N = c->N;
  op.P = c->P;
  op.n1 = c->n1;
  op.nf = c->nf;
  op.h = c->h;
  op.robin = 0;
  for (int sd = 0; sd < 2 * c->dim; ++sd)
    if (c->desc.bc[sd] == TH_BC_ROBIN) op.robin |= 1 << sd;
  op.dir = c->dir;
  op.kap = shifted ? c->d_kaps : c->d_kap;
  op.kr = c->d_k;
  return op;
}

static void free_graphs(th_ctx *c) {
  for (auto &g : c->graphs) (void)hipGraphExecDestroy(g.exec);
  c->graphs.clear();
}

static void free_fine(th_ctx *c) {
  void *ptrs[] = {c->d_kap, c->d_kaps, c->d_k,  c->d_subs, c->d_nblk, c->d_B, c->w_r,
                  c->w_v,   c->w_rr,   c->w_y,  c->w_rc,   c->w_uc,   c->w_t,
                  c->d_eidx, c->w_p, c->w_x, c->w_z, c->w_yc, c->w_xp};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  c->d_kap = c->d_kaps = nullptr;
  c->d_k = nullptr;
  c->d_subs = nullptr;
  c->d_nblk = nullptr;
  c->d_B = c->w_r = c->w_v = c->w_rr = c->w_y = c->w_rc = c->w_uc = c->w_t = nullptr;
  c->d_eidx = nullptr;
  c->w_p = c->w_x = c->w_z = c->w_yc = c->w_xp = nullptr;
  c->mfx_max_nrb = 0;
  c->mfx_ok = false;
  c->max_nsl = c->max_slab_rows = 0;
  c->slab_pk = 0;
  c->fine_ready = false;
}

// nested-dissection coarse solve: probe error below which no further
// refinement step is taken for an exact solve (th_coarse_solve, th_twogrid),
// the same for the preconditioner inside th_solve, where the coarse solve may
// be approximate (Sec. 1): an order below the rounding of a complex64
// preconditioner, which takes no refinement at all, and whatever it perturbs,
// the solve stops only on the true FP64 residual; and the most steps
constexpr double kCoarseRefineTol = 1e-13;
constexpr double kCoarsePrecondTol = 1e-8;
constexpr int kCoarseMaxRefine = 3;

static void free_coarse(th_ctx *c) {
  free_graphs(c);  // graphs reference the coarse factors and workspaces
  void *ptrs[] = {c->coarse.G, c->coarse.st, c->coarse.tbuf, c->coarse.pbuf};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  free_nd(c->coarse.nd);
  c->coarse = CoarseData{};
  c->coarse_ready = false;
}

static void free_solver(th_ctx *c) {
  free_graphs(c);  // graphs reference the solver's staging buffers
  if (c->s_buf) (void)hipFree(c->s_buf);
  c->s_buf = nullptr;
  c->s_bytes = 0;
  for (auto *L : {&c->kv_V, &c->kv_Z}) {
    for (void *p : *L) (void)hipFree(p);
    L->clear();
  }
  c->kv_vec_bytes = 0;
}

// Device scratch of th_coarse_solve_noalloc: one fixed array per GPU, held
// until the process ends.  Host code never passes the array's name to a kernel
// (on the host it is a stand-in, not a device address); th_create looks up
// each device's address once, with that device current, and the entry point
// uses only that address.
constexpr size_t kNoAllocBytes = (size_t)64 << 20;
static __device__ __align__(256) c64 scratch[kNoAllocBytes / sizeof(c64)];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices] = {};

// the device address of `scratch` on the current device `dev`, looked up once
static hipError_t scratch_address(int dev, void **out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

extern "C" {

th_status th_create(th_ctx **out, int hip_device, void *hip_stream) {
  if (!out) return TH_EINVAL;
  *out = nullptr;
  th_ctx *c = new (std::nothrow) th_ctx();
  if (!c) return TH_ENOMEM;
  c->device = hip_device;
  c->stream = (hipStream_t)hip_stream;
  hipError_t e = hipSetDevice(hip_device);
  if (e == hipSuccess) e = scratch_address(hip_device, &c->noalloc_scratch);
  if (e != hipSuccess) {
    delete c;
    return TH_EHIP;
  }
  *out = c;
  return TH_OK;
}

void th_destroy(th_ctx *ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  else (void)hipDeviceSynchronize();
  free_solver(ctx);
  free_coarse(ctx);
  free_fine(ctx);
  for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
  if (ctx->h_pinned) (void)hipHostFree(ctx->h_pinned);
  delete ctx;
}

th_status th_timing_enable(th_ctx *ctx, int enable) {
  if (!ctx) return TH_EINVAL;
  ctx->err.clear();
  if (hipStreamSynchronize(ctx->stream) != hipSuccess) return fail(ctx, TH_EHIP, "synchronisation failed");
  ctx->ev_used = 0;
  ctx->ev_marks.clear();
  ctx->timing = enable != 0;
  return TH_OK;
}

th_status th_timing_get(th_ctx *ctx, int kernel_class, double *total_ms, long long *launches) {
  if (!ctx || !total_ms || !launches) return TH_EINVAL;
  if (kernel_class < 0 || kernel_class >= TH_KT_COUNT) return fail(ctx, TH_EINVAL, "bad kernel class");
  if (hipStreamSynchronize(ctx->stream) != hipSuccess) return fail(ctx, TH_EHIP, "synchronisation failed");
  double tot = 0.0;
  long long n = 0;
  for (auto &m : ctx->ev_marks) {
    if (m.first != kernel_class) continue;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, ctx->ev_pool[m.second.first], ctx->ev_pool[m.second.second]) !=
        hipSuccess)
      return fail(ctx, TH_EHIP, "hipEventElapsedTime failed");
    tot += ms;
    ++n;
  }
  *total_ms = tot;
  *launches = n;
  return TH_OK;
}

const char *th_last_error(const th_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

th_status th_get_info(const th_ctx *ctx, th_info *info) {
  if (!ctx || !info) return TH_EINVAL;
  std::memset(info, 0, sizeof(*info));
  info->n_fine = ctx->nf;
  info->n_coarse = ctx->nc;
  info->n_sub = (int)ctx->subs.size();
  info->b_entries = ctx->b_entries;
  info->b_bytes = ctx->b_bytes;
  info->coarse_bytes = ctx->coarse.bytes;
  info->t_setup_fine_s = ctx->t_setup_fine;
  info->t_setup_coarse_s = ctx->t_setup_coarse;
  info->smoother_cfg = ctx->mfma_cfg;
  info->smoother_grid = ctx->mfma_grid;
  info->coarse_lines = ctx->coarse.nblk > 0 ? ctx->coarse.line0[1] - ctx->coarse.line0[0] : 0;
  info->n_fallback_cells = ctx->n_fallback;
  info->t_stencil_s = ctx->t_stencil;
  info->smoother_layout = ctx->layout;
  info->coarse_solver = ctx->coarse.kind == 1 ? TH_CSOLVE_ND : TH_CSOLVE_LINES;
  info->coarse_levels = ctx->coarse.nd.levels;
  info->coarse_refine = ctx->coarse.nd.refine_pc;
  info->coarse_refine_exact = ctx->coarse.nd.refine;
  info->coarse_check = ctx->coarse.check_err;
  info->coarse_check_pc = ctx->coarse.check_err_pc;
  info->slab_packed = ctx->layout == 3 ? ctx->slab_pk : 0;
  return TH_OK;
}

th_status th_setup_fine(th_ctx *ctx, const th_fine_desc *d) {
  if (!ctx) return TH_EINVAL;
  ctx->err.clear();
  if (!d) return fail(ctx, TH_EINVAL, "null descriptor");
  if (d->dim != 2 && d->dim != 3) return fail(ctx, TH_EINVAL, "dim must be 2 or 3");
  if (d->n < 1) return fail(ctx, TH_EINVAL, "n must be >= 1");
  if (d->order < 2 || d->order > kMaxP || d->order % 2)
    return fail(ctx, TH_EINVAL, "order must be 2, 4, 6 or 8");
  if (d->dim == 3 && d->order > 4)
    return fail(ctx, TH_EUNSUPPORTED, "3-D problems support orders 2 and 4");
  if (!d->k) return fail(ctx, TH_EINVAL, "k is NULL");
  if (d->l_dd < 1 || d->n_dd < 1 || d->n_s < 1 || d->max_rhs < 1)
    return fail(ctx, TH_EINVAL, "l_dd, n_dd, n_s and max_rhs must be >= 1");
  if (!(d->alpha_s >= 0.0) || !std::isfinite(d->alpha_s) || !std::isfinite(d->omega_c))
    return fail(ctx, TH_EINVAL, "alpha_s must be finite and >= 0, omega_c finite");
  if (d->gemm != TH_GEMM_F64 && d->gemm != TH_GEMM_F32 && d->gemm != TH_GEMM_BF16)
    return fail(ctx, TH_EINVAL, "unknown subdomain operator storage");
  if (d->layout < TH_LAYOUT_AUTO || d->layout > TH_LAYOUT_SLAB)
    return fail(ctx, TH_EINVAL, "unknown subdomain solve layout");
  if (d->gemm == TH_GEMM_BF16 && d->layout != TH_LAYOUT_AUTO)
    return fail(ctx, TH_EINVAL, "BF16 storage has the matrix-core layout only");
  for (int sd = 0; sd < 2 * d->dim; ++sd)
    if (d->bc[sd] != TH_BC_ROBIN && d->bc[sd] != TH_BC_NEUMANN && d->bc[sd] != TH_BC_DIRICHLET)
      return fail(ctx, TH_EINVAL, "boundary condition must be Robin, Neumann or Dirichlet");
  const long long ncell = (long long)d->n * d->n * (d->dim == 3 ? d->n : 1);
  for (long long i = 0; i < ncell; ++i) {
    if (!(d->k[i] > 0.0) || !std::isfinite(d->k[i]))
      return fail(ctx, TH_EINVAL, "k must be finite and > 0 in every cell");
    if (d->eps && (!(d->eps[i] >= 0.0) || !std::isfinite(d->eps[i])))
      return fail(ctx, TH_EINVAL, "eps must be finite and >= 0 in every cell");
    // the subdomain factorisations run without pivoting; that rests on the
    // positive definite Hermitian part of i A_s^(i), which needs a positive
    // imaginary volume coefficient alpha_s k^2 + eps in every cell (Sec. 4.1)
    if (!(d->alpha_s * d->k[i] * d->k[i] + (d->eps ? d->eps[i] : 0.0) > 0.0))
      return fail(ctx, TH_EINVAL,
                  "alpha_s = 0 needs eps > 0 in every cell (shifted operator without pivoting)");
  }
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, TH_EHIP, "hipSetDevice failed");
  auto t0 = std::chrono::steady_clock::now();
  free_solver(ctx);
  free_coarse(ctx);
  free_fine(ctx);
  th_ctx *c = ctx;
  c->desc = *d;
  c->desc.k = nullptr;
  c->desc.eps = nullptr;
  c->dim = d->dim;
  c->N = d->n;
  c->P = d->order;
  c->R = d->order / 2;
  c->n1 = c->N * c->P + 1;
  c->nc1 = c->N * c->R + 1;
  c->nf = (long long)c->n1 * c->n1 * (c->dim == 3 ? c->n1 : 1);
  c->nc = (long long)c->nc1 * c->nc1 * (c->dim == 3 ? c->nc1 : 1);
  c->h = 1.0 / c->N;
  c->dir = 0;
  for (int sd = 0; sd < 2 * c->dim; ++sd)
    if (d->bc[sd] == TH_BC_DIRICHLET) c->dir |= 1 << sd;
  make_ref1d(c->P, c->ref);
  c->h_k.assign(d->k, d->k + ncell);
  c->h_eps.assign(ncell, 0.0);
  if (d->eps) c->h_eps.assign(d->eps, d->eps + ncell);

  // per-cell coefficients
  std::vector<c64> kap(ncell), kaps(ncell);
  for (long long i = 0; i < ncell; ++i) {
    const double k2 = c->h_k[i] * c->h_k[i];
    kap[i] = c64{k2, c->h_eps[i]};
    kaps[i] = c64{k2, d->alpha_s * k2 + c->h_eps[i]};
  }

  // subdomains: M balanced blocks per direction (larger ones first)
  const int N = c->N, P = c->P;
  const int M = (N + d->l_dd - 1) / d->l_dd;
  c->M = M;
  c->blk_start.assign(M + 1, 0);
  {
    const int base = N / M, rem = N % M;
    for (int b = 0; b < M; ++b) c->blk_start[b + 1] = c->blk_start[b] + base + (b < rem ? 1 : 0);
  }
  std::vector<int> nblk(2 * c->n1, 0);
  for (int i = 0; i < c->n1; ++i) {
    int b = 0;
    while (c->blk_start[b + 1] * P < i) ++b;
    const int cnt = (i == c->blk_start[b + 1] * P && b + 1 < M) ? 2 : 1;
    nblk[2 * i] = b;
    nblk[2 * i + 1] = cnt;
  }
  c->subs.clear();
  long long boff = 0, yoff = 0;
  int max_ldb = 0, max_nom = 0;
  const int Mz = c->dim == 3 ? M : 1;
  for (int bz = 0; bz < Mz; ++bz)
    for (int by = 0; by < M; ++by)
      for (int bx = 0; bx < M; ++bx) {
        Sub s{};
        s.u0x = c->blk_start[bx];
        s.u1x = c->blk_start[bx + 1];
        s.u0y = c->blk_start[by];
        s.u1y = c->blk_start[by + 1];
        s.o0x = std::max(s.u0x - 1, 0);
        s.o1x = std::min(s.u1x + 1, N);
        s.o0y = std::max(s.u0y - 1, 0);
        s.o1y = std::min(s.u1y + 1, N);
        if (c->dim == 3) {
          s.u0z = c->blk_start[bz];
          s.u1z = c->blk_start[bz + 1];
          s.o0z = std::max(s.u0z - 1, 0);
          s.o1z = std::min(s.u1z + 1, N);
        }
        s.nux = (s.u1x - s.u0x) * P + 1;
        s.nuy = (s.u1y - s.u0y) * P + 1;
        s.nuz = (s.u1z - s.u0z) * P + 1;  // 1 in 2-D
        s.nox = (s.o1x - s.o0x) * P + 1;
        s.noy = (s.o1y - s.o0y) * P + 1;
        s.noz = (s.o1z - s.o0z) * P + 1;
        s.nU = s.nux * s.nuy * s.nuz;
        s.nOm = s.nox * s.noy * s.noz;
        s.ldb = (s.nU + 63) / 64 * 64;
        s.robin = 0;
        const bool inner[6] = {s.o0x > 0, s.o1x < N, s.o0y > 0, s.o1y < N, s.o0z > 0, s.o1z < N};
        s.dir = 0;
        for (int sd = 0; sd < 2 * c->dim; ++sd) {
          if (inner[sd] || d->bc[sd] == TH_BC_ROBIN) s.robin |= 1 << sd;
          if (!inner[sd] && d->bc[sd] == TH_BC_DIRICHLET) s.dir |= 1 << sd;
        }
        s.nrb = (s.nU + kSymTile - 1) / kSymTile;
        s.neb = (s.nOm - s.nU + kSymTile - 1) / kSymTile;
        s.nsl = c->dim == 3 ? s.o1z - s.o0z : s.o1y - s.o0y;
        s.lsz = c->dim == 3 ? s.nox * s.noy : s.nox;
        s.yoff = yoff;
        yoff += s.nU;
        max_ldb = std::max(max_ldb, s.ldb);
        max_nom = std::max(max_nom, s.nOm);
        c->subs.push_back(s);
      }
  // storage layout.  Explicit inverse rows: the symmetric tiles (U x U block
  // of the symmetric inverse stored once) when they need at most 80 % of the
  // dense bytes.  Slab factors instead when their modelled apply time (their
  // bytes at a lower rate, plus about one launch per slab) is lower.
  auto sym_elems = [](const Sub &s) {
    return ((long long)s.nrb * (s.nrb + 1) / 2 + (long long)s.nrb * s.neb) * kSymTile * kSymTile;
  };
  const int cband = (c->dim == 3 ? (2 * P + 1) * (2 * P + 1) : 2 * P + 1) * P;
  // G_t, bands, E_t; stored rows padded to a multiple of 8 entries, regions
  // kept on 128-byte boundaries
  auto pad8 = [](long long x) { return (x + 7) & ~7LL; };
  // Packed G_t (each symmetric G_t stored once: skewed 64 x 64 tiles of the
  // lower block triangle plus a dense strip of the last m mod 64 rows) when
  // the largest slab is one work unit of the packed forward sweep and its LDS
  // holds a chunk of min(max_rhs, 4) FP64 right-hand sides (TH_SLAB_PACKED=0
  // or 1 overrides: whole G_t, or packed with one right-hand side per chunk).
  {
    int max_lsz = 0;
    for (const Sub &s : c->subs) max_lsz = std::max(max_lsz, s.lsz);
    const long long ml = (long long)(P + 1) * max_lsz;
    const int rc = d->max_rhs >= 4 ? 4 : (d->max_rhs >= 2 ? 2 : 1);
    auto lds = [&](int r) {
      return (size_t)std::max<long long>(2 * ml + 512 * ((ml + 63) / 64), 512) * r * sizeof(c64);
    };
    const char *env = std::getenv("TH_SLAB_PACKED");
    const bool want = env ? std::atoi(env) != 0 : true;
    c->slab_pk = want && ml <= slab_pk_max_rows() &&
                 lds(env ? 1 : rc) <= kSlabPkLds;
  }
  auto pk_size = [](long long m) {
    const long long nf = m / 64;
    return 64 * (33 * nf + 32 * nf * (nf - 1)) + (m - 64 * nf) * ((m + 7) & ~7LL);
  };
  auto slab_g = [&](const Sub &s) {
    const long long m = (long long)P * s.lsz, ml = (long long)(P + 1) * s.lsz;
    if (c->slab_pk) return (long long)(s.nsl - 1) * pk_size(m) + pk_size(ml);
    return (long long)(s.nsl - 1) * m * pad8(m) + ml * pad8(ml);
  };
  auto slab_bands = [&](const Sub &s) { return pad8((long long)(s.nsl - 1) * s.lsz * cband); };
  // E_t of the lower chain of the twisted elimination (slabs 0 .. (nsl - 1) / 2 - 1);
  // packed: also G_t[:, first layer] of the upper chain, indexed by slab
  auto slab_elems = [&](const Sub &s) {
    const long long m = (long long)P * s.lsz, ml = (long long)(P + 1) * s.lsz;
    if (c->slab_pk)
      return slab_g(s) + slab_bands(s) + (long long)(s.nsl - 1) * s.lsz * pad8(m) +
             s.lsz * pad8(ml);
    return slab_g(s) + slab_bands(s) + (long long)((s.nsl - 1) / 2) * s.lsz * pad8(m);
  };
  {
    long long dense = 0, sym = 0, slab = 0;
    int nsl = 0;
    for (const Sub &s : c->subs) {
      dense += (long long)s.nOm * s.ldb;
      sym += sym_elems(s);
      slab += slab_elems(s);
      nsl = std::max(nsl, s.nsl);
    }
    // modelled streaming rates (bytes/s) of the three apply paths, 8 us per launch
    const double es = d->gemm == TH_GEMM_F32 ? 8.0 : 16.0;
    const int rows = 10 * sym <= 8 * dense ? 1 : 0;
    const double t_rows = rows == 1 ? es * sym / 5.5e12 : es * dense / 6.5e12;
    const double t_slab = es * slab / 4.0e12 + (2 * (nsl / 2) + 3) * 8e-6;
    // the sweeps keep a slab's right-hand side (then, in the same space, up to
    // 512 partial sums) in 48 KiB of LDS
    int max_lsz = 0;
    for (const Sub &s : c->subs) max_lsz = std::max(max_lsz, s.lsz);
    const bool slab_fits = std::max<long long>((long long)(P + 1) * max_lsz, 512) * 16 <= 48 * 1024;
    if (d->gemm == TH_GEMM_BF16)
      c->layout = 2;
    else if (d->layout == TH_LAYOUT_DENSE)
      c->layout = 0;
    else if (d->layout == TH_LAYOUT_SYMMETRIC)
      c->layout = 1;
    else if (d->layout == TH_LAYOUT_SLAB && !slab_fits) {
      free_fine(c);
      return fail(ctx, TH_EUNSUPPORTED, "subdomain slabs too large for the slab layout");
    } else if (d->layout == TH_LAYOUT_SLAB)
      c->layout = 3;
    else
      c->layout = slab_fits && t_slab < t_rows ? 3 : rows;
    if (c->layout != 3) c->slab_pk = 0;
  }
  std::vector<int> eidx;
  long long poff = 0, xoff = 0;
  c->max_pairs = 0;
  for (Sub &s : c->subs) {
    s.boff = boff;
    // element offsets: complex entries (F64/F32) or bf16 values (matrix-core layout)
    if (c->layout == 3) {
      const long long ml = (long long)(P + 1) * s.lsz;
      s.coff = boff + slab_g(s);
      s.ecoff = s.coff + slab_bands(s);
      boff += slab_elems(s);
      c->max_nsl = std::max(c->max_nsl, s.nsl);
      c->max_slab_rows = std::max(c->max_slab_rows, (int)ml);
    } else {
      boff += c->layout == 2 ? mfma_store_elems(s)
                             : (c->layout == 1 ? sym_elems(s) : (long long)s.nOm * s.ldb);
    }
    s.eoff = (long long)eidx.size();
    s.poff = poff;
    s.xoff = xoff;
    if (c->layout == 1) {
      // ring nodes Omega \ U in Omega-local order
      const int ux0 = (s.u0x - s.o0x) * P, ux1 = (s.u1x - s.o0x) * P;
      const int uy0 = (s.u0y - s.o0y) * P, uy1 = (s.u1y - s.o0y) * P;
      const int uz0 = (s.u0z - s.o0z) * P, uz1 = (s.u1z - s.o0z) * P;
      for (int k = 0; k < s.nOm; ++k) {
        const int kx = k % s.nox, ky = (k / s.nox) % s.noy, kz = k / (s.nox * s.noy);
        const bool inU = kx >= ux0 && kx <= ux1 && ky >= uy0 && ky <= uy1 && kz >= uz0 && kz <= uz1;
        if (!inU) eidx.push_back(k);
      }
      if ((long long)eidx.size() - s.eoff != s.nOm - s.nU) {
        free_fine(c);
        return fail(ctx, TH_EINVAL, "internal error: ring node count");
      }
      poff += (long long)s.nrb * (s.nrb + 1) / 2 * kSymTile;
      xoff += s.nOm;
      c->max_pairs = std::max(c->max_pairs, (s.nrb + 1) / 2);
    } else if (c->layout == 3 || (c->layout == 0 && d->gemm == TH_GEMM_F64 &&
                                    dd_mfma64_rhs_pad(d->max_rhs) > 0)) {
      xoff += s.nOm;  // gathered patches (slab sweeps, FP64 matrix-core apply)
    } else if (c->layout == 2) {
      s.xoff = xoff;  // first 32-column block of the patch fragments (two-pass BF16 apply)
      xoff += (s.nOm + 31) / 32;
    }
  }
  c->p_rows = poff;
  c->x_rows = c->layout == 2 ? 0 : xoff;  // layout 2 counts column blocks, kept in the Subs
  c->max_ldb = max_ldb;
  c->max_nom = max_nom;
  c->max_rowblocks = (max_ldb + 255) / 256;
  c->y_rows = yoff;
  c->b_entries = 0;
  for (auto &s : c->subs) c->b_entries += (long long)s.nU * s.nOm;
  const size_t belem = (d->gemm == TH_GEMM_BF16) ? 2 : (d->gemm == TH_GEMM_F32) ? sizeof(c32)
                                                                                : sizeof(c64);
  c->b_bytes = boff * (long long)belem;

  hipStream_t st = c->stream;
  auto alloc = [&](void **p, size_t bytes) -> bool {
    if (bytes == 0) bytes = 16;
    return hipMalloc(p, bytes) == hipSuccess;
  };
  const size_t R = (size_t)d->max_rhs;
  bool ok = alloc((void **)&c->d_eidx, eidx.size() * sizeof(int)) &&
            alloc(&c->w_p, R * c->p_rows * sizeof(c64)) &&
            alloc(&c->w_x, std::max<size_t>(R, dd_mfma64_rhs_pad(d->max_rhs)) * c->x_rows *
                               sizeof(c64)) &&
            alloc((void **)&c->d_kap, ncell * sizeof(c64)) &&
            alloc((void **)&c->d_kaps, ncell * sizeof(c64)) &&
            alloc((void **)&c->d_k, ncell * sizeof(double)) &&
            alloc((void **)&c->d_subs, c->subs.size() * sizeof(Sub)) &&
            alloc((void **)&c->d_nblk, nblk.size() * sizeof(int)) && alloc(&c->d_B, c->b_bytes) &&
            alloc(&c->w_r, R * c->nf * sizeof(c64)) &&
            alloc(&c->w_y, R * c->y_rows * sizeof(c64));
  if (ok && d->n_dd > 1)
    ok = alloc(&c->w_v, R * c->nf * sizeof(c64)) && alloc(&c->w_rr, R * c->nf * sizeof(c64));
  if (ok && c->layout == 3) ok = alloc(&c->w_z, R * c->x_rows * sizeof(c64));
  if (ok && c->layout == 2) {
    // colour planes of the staged and two-pass matrix-core kernels (sized for
    // complex128 vectors) and the two-pass kernel's BF16 patch fragments
    const size_t yc = ((size_t)1 << c->dim) * R * c->nf * sizeof(c64);
    long long xp = 0;
    for (const Sub &sb : c->subs) xp += mfp_patch_elems(sb, d->max_rhs);
    if (yc <= ((size_t)4 << 30)) {
      ok = alloc(&c->w_yc, yc);
      c->mfx_ok = mfx_fits(d->max_rhs, max_nom);
      for (const Sub &sb : c->subs) c->mfx_max_nrb = std::max(c->mfx_max_nrb, (sb.nU + 15) / 16);
      if (ok && xp * 2 <= ((long long)4 << 30)) ok = alloc(&c->w_xp, (size_t)xp * 2);
    }
  }
  if (!ok) {
    free_fine(c);
    return fail(ctx, TH_ENOMEM, "device allocation failed in setup_fine");
  }
  if (hipMemcpyAsync(c->d_kap, kap.data(), ncell * sizeof(c64), hipMemcpyHostToDevice, st) ||
      hipMemcpyAsync(c->d_kaps, kaps.data(), ncell * sizeof(c64), hipMemcpyHostToDevice, st) ||
      hipMemcpyAsync(c->d_k, c->h_k.data(), ncell * sizeof(double), hipMemcpyHostToDevice, st) ||
      hipMemcpyAsync(c->d_subs, c->subs.data(), c->subs.size() * sizeof(Sub),
                     hipMemcpyHostToDevice, st) ||
      hipMemcpyAsync(c->d_nblk, nblk.data(), nblk.size() * sizeof(int), hipMemcpyHostToDevice,
                     st) ||
      (!eidx.empty() && hipMemcpyAsync(c->d_eidx, eidx.data(), eidx.size() * sizeof(int),
                                       hipMemcpyHostToDevice, st)) ||
      hipMemsetAsync(c->d_B, 0, c->b_bytes, st)) {
    free_fine(c);
    return fail(ctx, TH_EHIP, "upload failed in setup_fine");
  }
  int rc = setup_subdomain_operators(c);
  if (rc == 0 && d->gemm == TH_GEMM_BF16) rc = autotune_mfma(c);
  if (rc) {
    free_fine(c);
    return finish(ctx, rc);
  }
  if (hipStreamSynchronize(st) != hipSuccess) {
    free_fine(c);
    return fail(ctx, TH_EHIP, "synchronisation failed in setup_fine");
  }
  c->t_setup_fine = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  c->fine_ready = true;
  return TH_OK;
}

// Per-cell weights and the 9-point quasi-FE stencil on the 2-D coarse grid.
static th_status coarse_stencil_2d(th_ctx *c, const th_coarse_desc *d, std::vector<c64> &st) {
  const int Nc = c->N * c->R, nc1 = c->nc1;
  const double hc = 1.0 / Nc;
  // per coarse cell: k, eps of the fine cell containing it; weights q
  std::vector<double> qw((size_t)Nc * Nc * 3);
  const auto ts0 = std::chrono::steady_clock::now();
  c->n_fallback = 0;
  if (d->scheme == TH_COARSE_PLAINFIT || d->scheme == TH_COARSE_MLP) {
    // per-cell samples (eta_c = h_c k, p, eps / k^2)
    std::vector<double> smp((size_t)Nc * Nc * 3);
    for (int cy = 0; cy < Nc; ++cy)
      for (int cxx = 0; cxx < Nc; ++cxx) {
        const long long ci = (long long)cy * Nc + cxx;
        const long long fi = (long long)(cy / c->R) * c->N + cxx / c->R;
        const double kk = c->h_k[fi];
        smp[3 * ci] = hc * kk;
        smp[3 * ci + 1] = c->P;
        smp[3 * ci + 2] = c->h_eps[fi] / (kk * kk);
        if (!(smp[3 * ci] * c->P / 2.0 < M_PI))
          return fail(c, TH_EINVAL, "dispersion fit needs fine k h < pi in every cell");
      }
    int rc = coarse_weights(2, d->scheme, d->mlp, d->fallback_tau, smp.data(), Nc * Nc, qw.data(),
                            &c->n_fallback);
    if (rc) return finish(c, rc);
  } else {
    for (int cy = 0; cy < Nc; ++cy)
      for (int cxx = 0; cxx < Nc; ++cxx) {
        const long long ci = (long long)cy * Nc + cxx;
        const long long fi = (long long)(cy / c->R) * c->N + cxx / c->R;
        if (d->scheme == TH_COARSE_QSFEM) {
          qsfem_weights(hc * c->h_k[fi], &qw[3 * ci]);
        } else {
          for (int t = 0; t < 3; ++t) {
            qw[3 * ci + t] = d->q[3 * ci + t];
            if (!std::isfinite(qw[3 * ci + t])) return fail(c, TH_EINVAL, "non-finite weight q");
          }
        }
      }
  }
  c->t_stencil = std::chrono::duration<double>(std::chrono::steady_clock::now() - ts0).count();
  // 9-point quasi-FE stencil per coarse vertex (eq. element_wise_qsfem with the
  // -i eps Q1 mass and the absorbing Q1 boundary mass)
  st.assign((size_t)nc1 * nc1 * 9, c64{0, 0});
  const double m1[2][2] = {{1.0 / 3.0, 1.0 / 6.0}, {1.0 / 6.0, 1.0 / 3.0}};
  for (int cy = 0; cy < Nc; ++cy)
    for (int cxx = 0; cxx < Nc; ++cxx) {
      const long long ci = (long long)cy * Nc + cxx;
      const long long fi = (long long)(cy / c->R) * c->N + cxx / c->R;
      const double kk = c->h_k[fi], ee = c->h_eps[fi];
      for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) {
          const int ax = a & 1, ay = a >> 1, bx = b & 1, by = b >> 1;
          const int diff = (ax != bx) + (ay != by);
          c64 v = {qw[3 * ci + diff], -ee * hc * hc * m1[ay][by] * m1[ax][bx]};
          // absorbing sides: x- (cxx==0, ax=bx=0), x+ (ax=bx=1), y- (ay=by=0), y+
          if (cxx == 0 && ax == 0 && bx == 0 && c->desc.bc[0] == TH_BC_ROBIN)
            v.im -= kk * hc * m1[ay][by];
          if (cxx == Nc - 1 && ax == 1 && bx == 1 && c->desc.bc[1] == TH_BC_ROBIN)
            v.im -= kk * hc * m1[ay][by];
          if (cy == 0 && ay == 0 && by == 0 && c->desc.bc[2] == TH_BC_ROBIN)
            v.im -= kk * hc * m1[ax][bx];
          if (cy == Nc - 1 && ay == 1 && by == 1 && c->desc.bc[3] == TH_BC_ROBIN)
            v.im -= kk * hc * m1[ax][bx];
          const long long ga = (long long)(cy + ay) * nc1 + cxx + ax;
          const int dx = bx - ax, dy = by - ay;
          c64 &e = st[9 * ga + (dy + 1) * 3 + (dx + 1)];
          e = e + v;
        }
    }
  return TH_OK;
}

// Per-cell weights (q0, q_face, q_edge, q_corner) and the 27-point quasi-FE
// stencil on the 3-D coarse grid: the -i eps Q1 mass and the absorbing Q1
// face mass are added per coarse cell as in 2-D.  The weights are normalised
// to the 2-D element scale (symbol -eta^2 at 0); a 3-D cell stiffness scales
// as h_c, so a cell contributes h_c q.
static th_status coarse_stencil_3d(th_ctx *c, const th_coarse_desc *d, std::vector<c64> &st) {
  const int Nc = c->N * c->R, nc1 = c->nc1, R = c->R, N = c->N;
  const double hc = 1.0 / Nc;
  const long long ncc = (long long)Nc * Nc * Nc;
  auto fine_of = [&](long long cz, long long cy, long long cxx) {
    return ((cz / R) * N + cy / R) * N + cxx / R;
  };
  std::vector<double> qw((size_t)ncc * 4);
  const auto ts0 = std::chrono::steady_clock::now();
  c->n_fallback = 0;
  if (d->scheme == TH_COARSE_PLAINFIT || d->scheme == TH_COARSE_MLP) {
    std::vector<double> smp((size_t)ncc * 3);
    for (long long ci = 0; ci < ncc; ++ci) {
      const long long fi = fine_of(ci / ((long long)Nc * Nc), (ci / Nc) % Nc, ci % Nc);
      const double kk = c->h_k[fi];
      smp[3 * ci] = hc * kk;
      smp[3 * ci + 1] = c->P;
      smp[3 * ci + 2] = c->h_eps[fi] / (kk * kk);
      if (!(smp[3 * ci] * c->P / 2.0 < M_PI))
        return fail(c, TH_EINVAL, "dispersion fit needs fine k h < pi in every cell");
    }
    int rc = coarse_weights(3, d->scheme, d->mlp, d->fallback_tau, smp.data(), (int)ncc,
                            qw.data(), &c->n_fallback);
    if (rc) return finish(c, rc);
  } else {
    for (long long ci = 0; ci < ncc; ++ci) {
      if (d->scheme == TH_COARSE_QSFEM) {
        const long long fi = fine_of(ci / ((long long)Nc * Nc), (ci / Nc) % Nc, ci % Nc);
        const double eta = hc * c->h_k[fi];
        const double z[3] = {eta, eta, eta};
        fit27_from_radii(eta, z, &qw[4 * ci]);
      } else {
        for (int t = 0; t < 4; ++t) {
          qw[4 * ci + t] = d->q[4 * ci + t];
          if (!std::isfinite(qw[4 * ci + t])) return fail(c, TH_EINVAL, "non-finite weight q");
        }
      }
    }
  }
  c->t_stencil = std::chrono::duration<double>(std::chrono::steady_clock::now() - ts0).count();
  st.assign((size_t)nc1 * nc1 * nc1 * 27, c64{0, 0});
  const double m1[2][2] = {{1.0 / 3.0, 1.0 / 6.0}, {1.0 / 6.0, 1.0 / 3.0}};
  const double hc2 = hc * hc, hc3 = hc2 * hc;
  const bool rb[6] = {c->desc.bc[0] == TH_BC_ROBIN, c->desc.bc[1] == TH_BC_ROBIN,
                      c->desc.bc[2] == TH_BC_ROBIN, c->desc.bc[3] == TH_BC_ROBIN,
                      c->desc.bc[4] == TH_BC_ROBIN, c->desc.bc[5] == TH_BC_ROBIN};
  for (int cz = 0; cz < Nc; ++cz)
    for (int cy = 0; cy < Nc; ++cy)
      for (int cxx = 0; cxx < Nc; ++cxx) {
        const long long ci = ((long long)cz * Nc + cy) * Nc + cxx;
        const long long fi = fine_of(cz, cy, cxx);
        const double kk = c->h_k[fi], ee = c->h_eps[fi];
        for (int a = 0; a < 8; ++a)
          for (int b = 0; b < 8; ++b) {
            const int ax = a & 1, ay = (a >> 1) & 1, az = a >> 2;
            const int bx = b & 1, by = (b >> 1) & 1, bz = b >> 2;
            const int diff = (ax != bx) + (ay != by) + (az != bz);
            c64 v = {hc * qw[4 * ci + diff], -ee * hc3 * m1[az][bz] * m1[ay][by] * m1[ax][bx]};
            const double fx = kk * hc2 * m1[ay][by] * m1[az][bz];
            const double fy = kk * hc2 * m1[ax][bx] * m1[az][bz];
            const double fz = kk * hc2 * m1[ax][bx] * m1[ay][by];
            if (rb[0] && cxx == 0 && ax == 0 && bx == 0) v.im -= fx;
            if (rb[1] && cxx == Nc - 1 && ax == 1 && bx == 1) v.im -= fx;
            if (rb[2] && cy == 0 && ay == 0 && by == 0) v.im -= fy;
            if (rb[3] && cy == Nc - 1 && ay == 1 && by == 1) v.im -= fy;
            if (rb[4] && cz == 0 && az == 0 && bz == 0) v.im -= fz;
            if (rb[5] && cz == Nc - 1 && az == 1 && bz == 1) v.im -= fz;
            const long long ga = ((long long)(cz + az) * nc1 + cy + ay) * nc1 + cxx + ax;
            c64 &e = st[27 * ga + ((bz - az + 1) * 3 + (by - ay + 1)) * 3 + (bx - ax + 1)];
            e = e + v;
          }
      }
  return TH_OK;
}

// Dirichlet sides: the coarse vertices on them are eliminated like the fine
// nodes (unit rows and columns of the stencil matrix).
static void eliminate_dirichlet(const th_ctx *c, std::vector<c64> &st) {
  if (!c->dir) return;
  const int n = c->nc1, dim = c->dim, S = dim == 3 ? 27 : 9, nz = dim == 3 ? n : 1;
  auto on = [&](int x, int y, int z) {
    return on_dir(c->dir, 0, x, n - 1) || on_dir(c->dir, 1, y, n - 1) ||
           (dim == 3 && on_dir(c->dir, 2, z, n - 1));
  };
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < n; ++y)
      for (int x = 0; x < n; ++x) {
        c64 *row = &st[(size_t)S * (((long long)z * n + y) * n + x)];
        if (on(x, y, z)) {
          for (int t = 0; t < S; ++t) row[t] = c64{0, 0};
          row[S / 2] = c64{1.0, 0.0};
          continue;
        }
        for (int t = 0; t < S; ++t) {
          const int dx = t % 3 - 1, dy = (t / 3) % 3 - 1, dz = dim == 3 ? t / 9 - 1 : 0;
          const int xx = x + dx, yy = y + dy, zz = z + dz;
          if (xx < 0 || xx >= n || yy < 0 || yy >= n || zz < 0 || zz >= nz) continue;
          if (on(xx, yy, zz)) row[t] = c64{0, 0};
        }
      }
}

th_status th_setup_coarse(th_ctx *ctx, const th_coarse_desc *d) {
  if (!ctx) return TH_EINVAL;
  ctx->err.clear();
  if (!d) return fail(ctx, TH_EINVAL, "null descriptor");
  if (!ctx->fine_ready) return fail(ctx, TH_ESTATE, "th_setup_fine must succeed first");
  if (d->scheme != TH_COARSE_QSFEM && d->scheme != TH_COARSE_WEIGHTS &&
      d->scheme != TH_COARSE_PLAINFIT && d->scheme != TH_COARSE_MLP)
    return fail(ctx, TH_EINVAL, "unknown coarse scheme");
  if (d->solver != TH_CSOLVE_AUTO && d->solver != TH_CSOLVE_LINES && d->solver != TH_CSOLVE_ND)
    return fail(ctx, TH_EINVAL, "unknown coarse solver");
  if (d->scheme == TH_COARSE_WEIGHTS && !d->q) return fail(ctx, TH_EINVAL, "q is NULL");
  if (d->scheme == TH_COARSE_MLP && !d->mlp) return fail(ctx, TH_EINVAL, "mlp is NULL");
  if (d->scheme == TH_COARSE_MLP && !(d->fallback_tau >= 0.0))
    return fail(ctx, TH_EINVAL, "fallback_tau must be >= 0");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, TH_EHIP, "hipSetDevice failed");
  auto t0 = std::chrono::steady_clock::now();
  free_coarse(ctx);
  th_ctx *c = ctx;
  std::vector<c64> st;
  {
    const th_status sc = c->dim == 3 ? coarse_stencil_3d(c, d, st) : coarse_stencil_2d(c, d, st);
    if (sc) return sc;
    eliminate_dirichlet(c, st);
  }
  // nested dissection first (unless the caller asked for the line elimination);
  // AUTO falls back to the line elimination when it fails its probe check or
  // cannot get its memory
  int rc = 0;
  bool have = false;
  if (d->solver != TH_CSOLVE_LINES) {
    rc = setup_coarse_nd(c, st);
    double err = -1.0;
    if (rc == 0) rc = coarse_probe_check(c, st, &err);
    // refinement steps until the probe solve is at the rounding level (exact
    // solves) or within kCoarsePrecondTol (the FP64 preconditioner)
    int pc = err <= kCoarsePrecondTol ? 0 : -1;
    double err_pc = err;
    while (rc == 0 && !(err <= kCoarseRefineTol) && c->coarse.nd.refine < kCoarseMaxRefine) {
      ++c->coarse.nd.refine;
      rc = coarse_probe_check(c, st, &err);
      if (pc < 0 && err <= kCoarsePrecondTol) {
        pc = c->coarse.nd.refine;
        err_pc = err;
      }
    }
    c->coarse.nd.refine_pc = pc < 0 ? c->coarse.nd.refine : pc;
    c->coarse.check_err = err;
    c->coarse.check_err_pc = pc < 0 ? err : err_pc;
    const double tol = d->solver == TH_CSOLVE_ND ? 1e-6 : 1e-9;
    if (rc == 0 && err <= tol &&
        (d->solver == TH_CSOLVE_ND || coarse_model_nd(c) <= coarse_model_lines(c))) {
      have = true;
    } else if (d->solver == TH_CSOLVE_ND) {
      if (rc == 0) {
        char msg[160];
        std::snprintf(msg, sizeof msg, "nested-dissection coarse factors fail the probe check "
                      "(%.3e > %.0e)", err, tol);
        set_error(msg);
        rc = TH_ENUMERIC;
      }
    } else if (rc == 0 || rc == TH_ENOMEM || rc == TH_ENUMERIC) {
      rc = 0;  // AUTO: the line elimination instead
    }
    if (!have) {
      free_nd(c->coarse.nd);
      c->coarse = CoarseData{};
    }
  }
  if (!have && rc == 0) {
    rc = setup_coarse_factors(c, st);
    double err = -1.0;
    if (rc == 0) rc = coarse_probe_check(c, st, &err);
    c->coarse.check_err = c->coarse.check_err_pc = err;
  }
  if (rc) {
    free_coarse(c);
    return finish(ctx, rc);
  }
  const size_t R = (size_t)c->desc.max_rhs;
  if (!c->w_rc) {
    if (hipMalloc(&c->w_rc, R * c->nc * sizeof(c64)) != hipSuccess ||
        hipMalloc(&c->w_uc, R * c->nc * sizeof(c64)) != hipSuccess) {
      free_coarse(c);
      return fail(ctx, TH_ENOMEM, "device allocation failed in setup_coarse");
    }
  }
  c->t_setup_coarse = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  c->coarse_ready = true;
  return TH_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// internal steps (precision selected by f32)

namespace th {

static int add_inplace(th_ctx *c, void *u, const void *v, int nrhs, bool f32) {
  return launch_add(u, v, (long long)nrhs * c->nf, f32, c->stream);
}

// u <- CSDDSmoother(u, f) (Alg. 2).  u_zero: u holds zeros on entry (it is
// then assigned, not read).
static int smooth_impl(th_ctx *c, void *u, const void *f, int nrhs, bool f32, bool u_zero) {
  hipStream_t s = c->stream;
  const void *r = f;
  if (!u_zero) {
    KTimer kt(c, TH_KT_OPERATOR);
    int rc = launch_apply(make_op(c, false), c->ref, u, f, c->w_r, nrhs, f32, -1.0, s);
    if (rc) return rc;
    r = c->w_r;
  }
  int rc;
  {
    KTimer kt(c, TH_KT_DD_APPLY);
    rc = launch_dd_apply(c, r, c->w_y, nrhs, f32, s);
  }
  if (rc) return rc;
  if (c->desc.n_dd == 1) {
    KTimer kt(c, TH_KT_DD_ACCUM);
    return launch_dd_accumulate(c, c->w_y, u, nrhs, f32, u_zero, s);
  }
  // n_dd > 1: v accumulates the DD steps, DDStep(v, r; A_s):
  // v <- v + avg((A_s^(i))^{-1} R_i (r - A_s v))
  rc = launch_dd_accumulate(c, c->w_y, c->w_v, nrhs, f32, true, s);
  for (int it = 1; it < c->desc.n_dd && rc == 0; ++it) {
    rc = launch_apply(make_op(c, true), c->ref, c->w_v, r, c->w_rr, nrhs, f32, -1.0, s);
    if (!rc) rc = launch_dd_apply(c, c->w_rr, c->w_y, nrhs, f32, s);
    if (!rc) rc = launch_dd_accumulate(c, c->w_y, c->w_v, nrhs, f32, false, s);
  }
  if (rc) return rc;
  if (u_zero) {
    TH_HIP_CHECK_RET(hipMemcpyAsync(u, c->w_v, (size_t)nrhs * c->nf * csize(f32),
                                    hipMemcpyDeviceToDevice, s));
    return 0;
  }
  return add_inplace(c, u, c->w_v, nrhs, f32);
}

// accuracy: kCoarseExact (th_coarse_solve) or kCoarsePrecond (inside the
// two-grid preconditioner); a complex64 solve is always rounded
static int coarse_solve_impl(th_ctx *c, const void *rc_in, void *uc_out, int nrhs, bool f32,
                             int accuracy) {
  hipStream_t s = c->stream;
  const c64 *r64 = (const c64 *)rc_in;
  c64 *u64 = (c64 *)uc_out;
  if (f32) {
    int rc = launch_convert(rc_in, c->w_rc, (long long)nrhs * c->nc, true, false, s);
    if (rc) return rc;
    r64 = (const c64 *)c->w_rc;
    u64 = (c64 *)c->w_uc;
  }
  int rc;
  {
    KTimer kt(c, TH_KT_COARSE);
    rc = launch_coarse_solve(c, r64, u64, nrhs, s, f32 ? kCoarseRounded : accuracy);
  }
  if (rc) return rc;
  if (f32) return launch_convert(u64, uc_out, (long long)nrhs * c->nc, false, true, s);
  return 0;
}

// u <- TwoGridStep(u, f) (Alg. 1)
// accuracy of the coarse solve: kCoarseExact for th_twogrid, kCoarsePrecond
// for the preconditioner of th_solve
static int twogrid_impl(th_ctx *c, void *u, const void *f, int nrhs, bool f32, bool u_zero,
                        int accuracy) {
  hipStream_t s = c->stream;
  int rc = 0;
  for (int i = 0; i < c->desc.n_s && rc == 0; ++i) rc = smooth_impl(c, u, f, nrhs, f32, u_zero && i == 0);
  if (rc) return rc;
  {
    KTimer kt(c, TH_KT_OPERATOR);
    rc = launch_apply(make_op(c, false), c->ref, u, f, c->w_r, nrhs, f32, -1.0, s);
  }
  if (rc) return rc;
  // the coarse vectors stay complex128 for the FP64 coarse solve: a complex64
  // step restricts straight into them and prolongs straight from them
  {
    KTimer kt(c, TH_KT_RESTRICT);
    rc = launch_restrict(c->dim, c->N, c->P, c->dir, c->ref, c->w_r, c->w_rc, nrhs, f32, s, true);
  }
  if (!rc) {
    KTimer kt(c, TH_KT_COARSE);
    rc = launch_coarse_solve(c, (const c64 *)c->w_rc, (c64 *)c->w_uc, nrhs, s,
                             f32 ? kCoarseRounded : accuracy);
  }
  if (!rc) {
    KTimer kt(c, TH_KT_PROLONG);
    rc = launch_prolong(c->dim, c->N, c->P, c->dir, c->ref, c->w_uc, u, c->desc.omega_c, nrhs, f32,
                        s, true);
  }
  for (int i = 0; i < c->desc.n_s && rc == 0; ++i) rc = smooth_impl(c, u, f, nrhs, f32, false);
  return rc;
}

}  // namespace th

extern "C" {

static th_status check_vec_call(th_ctx *ctx, const void *a, const void *b, int nrhs, th_dtype dt,
                                bool need_coarse) {
  if (!ctx) return TH_EINVAL;
  ctx->err.clear();
  if (!ctx->fine_ready) return fail(ctx, TH_ESTATE, "th_setup_fine must succeed first");
  if (need_coarse && !ctx->coarse_ready)
    return fail(ctx, TH_ESTATE, "th_setup_coarse must succeed first");
  if (!a || !b) return fail(ctx, TH_EINVAL, "null vector pointer");
  if (nrhs < 1 || nrhs > ctx->desc.max_rhs) return fail(ctx, TH_EINVAL, "nrhs out of range");
  if (dt != TH_C128 && dt != TH_C64) return fail(ctx, TH_EINVAL, "unknown dtype");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, TH_EHIP, "hipSetDevice failed");
  return TH_OK;
}

th_status th_residual(th_ctx *ctx, const void *u, const void *f, void *r, int nrhs, th_dtype dt) {
  th_status st = check_vec_call(ctx, u, f, nrhs, dt, false);
  if (st) return st;
  if (!r) return fail(ctx, TH_EINVAL, "null vector pointer");
  return finish(ctx, launch_apply(make_op(ctx, false), ctx->ref, u, f, r, nrhs, is_f32(dt), -1.0,
                                  ctx->stream));
}

th_status th_smooth(th_ctx *ctx, void *u, const void *f, int nrhs, th_dtype dt) {
  th_status st = check_vec_call(ctx, u, f, nrhs, dt, false);
  if (st) return st;
  return finish(ctx, smooth_impl(ctx, u, f, nrhs, is_f32(dt), false));
}

th_status th_restrict(th_ctx *ctx, const void *r, void *rc, int nrhs, th_dtype dt) {
  th_status st = check_vec_call(ctx, r, rc, nrhs, dt, false);
  if (st) return st;
  return finish(ctx, launch_restrict(ctx->dim, ctx->N, ctx->P, ctx->dir, ctx->ref, r, rc, nrhs,
                                     is_f32(dt), ctx->stream));
}

th_status th_prolong(th_ctx *ctx, const void *uc, void *u, double omega_c, int nrhs, th_dtype dt) {
  th_status st = check_vec_call(ctx, uc, u, nrhs, dt, false);
  if (st) return st;
  if (!std::isfinite(omega_c)) return fail(ctx, TH_EINVAL, "omega_c must be finite");
  return finish(ctx, launch_prolong(ctx->dim, ctx->N, ctx->P, ctx->dir, ctx->ref, uc, u, omega_c,
                                    nrhs, is_f32(dt), ctx->stream));
}

th_status th_coarse_solve(th_ctx *ctx, const void *rc, void *uc, int nrhs, th_dtype dt) {
  th_status st = check_vec_call(ctx, rc, uc, nrhs, dt, true);
  if (st) return st;
  return finish(ctx, coarse_solve_impl(ctx, rc, uc, nrhs, is_f32(dt), kCoarseExact));
}

th_status th_coarse_solve_noalloc(th_ctx *ctx, const void *rc, void *uc, int nrhs, th_dtype dt) {
  th_status st = check_vec_call(ctx, rc, uc, nrhs, dt, true);
  if (st) return st;
  th_ctx *c = ctx;
  const bool f32 = is_f32(dt);
  const long long ncn = c->nc;
  // scratch: [FP64 staging of rc and uc (complex64 only)][update vectors][t][d]
  long long need = f32 ? 2LL * nrhs * ncn : 0;
  const bool nd = c->coarse.kind == 1;
  if (nd) need += (long long)nrhs * (c->coarse.nd.ulen + 2 * ncn);
  else if (coarse_lines_need_staging(c))
    return fail(ctx, TH_EUNSUPPORTED, "th_coarse_solve_noalloc: the line elimination of this "
                "grid stages slabs in context buffers; set up the nested-dissection solver");
  if (need * (long long)sizeof(c64) > (long long)kNoAllocBytes) {
    char msg[200];
    std::snprintf(msg, sizeof msg, "th_coarse_solve_noalloc: needs %lld bytes of scratch, the "
                  "limit is %zu (fewer right-hand sides per call)",
                  need * (long long)sizeof(c64), kNoAllocBytes);
    return fail(ctx, TH_EINVAL, msg);
  }
  c64 *w = (c64 *)c->noalloc_scratch;
  hipStream_t s = c->stream;
  const c64 *r64 = (const c64 *)rc;
  c64 *u64 = (c64 *)uc;
  int rcode = 0;
  if (f32) {
    rcode = launch_convert(rc, w, (long long)nrhs * ncn, true, false, s);
    r64 = w;
    u64 = w + (long long)nrhs * ncn;
    w += 2LL * nrhs * ncn;
  }
  CoarseScratch ws;
  if (nd) {
    ws.uvec = w;
    ws.t = w + (long long)nrhs * c->coarse.nd.ulen;
    ws.d = ws.t + (long long)nrhs * ncn;
  }
  if (!rcode) rcode = launch_coarse_solve(c, r64, u64, nrhs, s, f32 ? kCoarseRounded : kCoarseExact, &ws);
  if (!rcode && f32) rcode = launch_convert(u64, uc, (long long)nrhs * ncn, false, true, s);
  return finish(ctx, rcode);
}

th_status th_twogrid(th_ctx *ctx, void *u, const void *f, int nrhs, th_dtype dt) {
  th_status st = check_vec_call(ctx, u, f, nrhs, dt, true);
  if (st) return st;
  return finish(ctx, twogrid_impl(ctx, u, f, nrhs, is_f32(dt), false, kCoarseExact));
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Outer Krylov method (FP64)

namespace th {

using zc = std::complex<double>;

struct SolverWS {
  c64 *partial, *partial2, *hd, *tmp32a, *tmp32b, *coef, *res;
  double *scal;
  c64 *hcol;    // device: one Hessenberg column, (m + 2) x nrhs
  c64 *hcol_h;  // pinned host copy of it
};

// Vectors per block of the Krylov basis (V or Z).
static const int KV_CHUNK = 8;

// Basis vector j of V or Z (nrhs vectors of n_fine, consecutive), its block
// allocated on first use.
static int basis_vec(th_ctx *c, std::vector<void *> &blocks, int j, c64 **out) {
  while ((int)blocks.size() <= j / KV_CHUNK) {
    void *p = nullptr;
    if (hipMalloc(&p, (size_t)KV_CHUNK * c->kv_vec_bytes) != hipSuccess) {
      (void)hipGetLastError();
      set_error("cannot allocate Krylov basis vectors (" + std::to_string(j + 1) +
                " needed); lower th_solve_opts.restart");
      return TH_ENOMEM;
    }
    blocks.push_back(p);
  }
  *out = (c64 *)((char *)blocks[j / KV_CHUNK] + (size_t)(j % KV_CHUNK) * c->kv_vec_bytes);
  return 0;
}

static int ensure_solver_ws(th_ctx *c, int m, int nrhs, bool f32, SolverWS &w) {
  const size_t vec = (size_t)nrhs * c->nf * sizeof(c64);
  size_t need = 0;
  need += 2 * (size_t)nrhs * 256 * sizeof(c64);             // partial sums (two sets)
  need += (size_t)nrhs * sizeof(c64) * 2;                   // dot outputs
  need += 2 * vec;                                          // preconditioner staging
  need += (size_t)nrhs * (m + 1) * sizeof(c64);             // lincomb coefficients
  need += (size_t)nrhs * sizeof(double) * 2;                // scalars
  need += (size_t)nrhs * (m + 2) * sizeof(c64);             // Hessenberg column
  need += vec;                                              // true residual
  const size_t pinned = (size_t)nrhs * (m + 2) * sizeof(c64);
  if (pinned > c->h_pinned_bytes) {
    if (c->h_pinned) (void)hipHostFree(c->h_pinned);
    c->h_pinned = nullptr;
    c->h_pinned_bytes = 0;
    if (hipHostMalloc(&c->h_pinned, pinned, hipHostMallocDefault) != hipSuccess) {
      set_error("cannot allocate pinned host memory for the Krylov work space");
      return TH_ENOMEM;
    }
    c->h_pinned_bytes = pinned;
  }
  need += 4096;
  const size_t kv_vec = (size_t)c->desc.max_rhs * c->nf * sizeof(c64);
  if (need > c->s_bytes || kv_vec != c->kv_vec_bytes) {
    free_solver(c);
    if (hipMalloc(&c->s_buf, need) != hipSuccess) {
      set_error("cannot allocate the Krylov work space");
      return TH_ENOMEM;
    }
    c->s_bytes = need;
    c->kv_vec_bytes = kv_vec;
  }
  char *p = (char *)c->s_buf;
  auto take = [&](size_t bytes) {
    char *q = p;
    p += (bytes + 255) / 256 * 256;
    return q;
  };
  w.partial = (c64 *)take((size_t)nrhs * 256 * sizeof(c64));
  w.partial2 = (c64 *)take((size_t)nrhs * 256 * sizeof(c64));
  w.hd = (c64 *)take((size_t)nrhs * sizeof(c64) * 2);
  // staging of the preconditioner input/output (complex64 copies, or FP64
  // copies at fixed addresses for graph replay)
  w.tmp32a = (c64 *)take(vec);
  w.tmp32b = (c64 *)take(vec);
  (void)f32;
  w.coef = (c64 *)take((size_t)nrhs * (m + 1) * sizeof(c64));
  w.scal = (double *)take((size_t)nrhs * sizeof(double) * 2);
  w.hcol = (c64 *)take((size_t)nrhs * (m + 2) * sizeof(c64));
  w.res = (c64 *)take(vec);
  w.hcol_h = (c64 *)c->h_pinned;
  return 0;
}

// z = TwoGridStep(0, v) in the requested precision; v, z FP64
// out = TwoGridStep(0, in) replayed from a HIP graph captured on first use for
// this (nrhs, precision, in, out); the graph holds every kernel of the step.
static int twogrid_graph(th_ctx *c, void *out, const void *in, int nrhs, bool f32) {
  for (auto &g : c->graphs)
    if (g.nrhs == nrhs && g.f32 == f32 && g.in == in && g.out == out) {
      TH_HIP_CHECK_RET(hipGraphLaunch(g.exec, c->stream));
      ++c->graph_launches;
      return 0;
    }
  hipGraph_t graph = nullptr;
  TH_HIP_CHECK_RET(hipStreamBeginCapture(c->stream, hipStreamCaptureModeRelaxed));
  int rc = twogrid_impl(c, out, in, nrhs, f32, true, kCoarsePrecond);
  hipError_t e = hipStreamEndCapture(c->stream, &graph);
  if (rc) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc;
  }
  if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture", __FILE__, __LINE__);
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate", __FILE__, __LINE__);
  c->graphs.push_back({nrhs, f32, in, out, exec});
  TH_HIP_CHECK_RET(hipGraphLaunch(exec, c->stream));
  ++c->graph_launches;
  return 0;
}

static int precond(th_ctx *c, const c64 *v, c64 *z, int nrhs, bool f32, SolverWS &w,
                   bool use_graph) {
  const bool graph = use_graph && c->stream != nullptr && !c->timing;
  const long long n = (long long)nrhs * c->nf;
  if (!f32) {
    if (!graph) return twogrid_impl(c, z, v, nrhs, false, true, kCoarsePrecond);
    TH_HIP_CHECK_RET(hipMemcpyAsync(w.tmp32a, v, n * sizeof(c64), hipMemcpyDeviceToDevice, c->stream));
    int rc = twogrid_graph(c, w.tmp32b, w.tmp32a, nrhs, false);
    if (rc) return rc;
    TH_HIP_CHECK_RET(hipMemcpyAsync(z, w.tmp32b, n * sizeof(c64), hipMemcpyDeviceToDevice, c->stream));
    return 0;
  }
  int rc = launch_convert(v, w.tmp32a, n, false, true, c->stream);
  if (!rc) rc = graph ? twogrid_graph(c, w.tmp32b, w.tmp32a, nrhs, true)
                      : twogrid_impl(c, w.tmp32b, w.tmp32a, nrhs, true, true, kCoarsePrecond);
  if (!rc) rc = launch_convert(w.tmp32b, z, n, true, false, c->stream);
  return rc;
}

static int dot_to_host(th_ctx *c, const c64 *x, const c64 *y, int nrhs, SolverWS &w,
                       std::vector<zc> &out) {
  int rc = launch_dot(x, y, c->nf, nrhs, c->nf, c->nf, w.hd, w.partial, c->stream);
  if (rc) return rc;
  std::vector<c64> h(nrhs);
  TH_HIP_CHECK_RET(hipMemcpyAsync(h.data(), w.hd, nrhs * sizeof(c64), hipMemcpyDeviceToHost,
                                  c->stream));
  TH_HIP_CHECK_RET(hipStreamSynchronize(c->stream));
  out.resize(nrhs);
  for (int r = 0; r < nrhs; ++r) out[r] = zc(h[r].re, h[r].im);
  return 0;
}

static void givens(zc a, zc b, zc &cs, zc &sn, zc &rr) {
  if (b == 0.0) {
    cs = 1.0;
    sn = 0.0;
    rr = a;
    return;
  }
  if (a == 0.0) {
    cs = 0.0;
    sn = std::conj(b) / std::abs(b);
    rr = std::abs(b);
    return;
  }
  const double t = std::sqrt(std::norm(a) + std::norm(b));
  const zc ph = a / std::abs(a);
  cs = std::abs(a) / t;
  sn = ph * std::conj(b) / t;
  rr = ph * t;
}

// Right-preconditioned GMRES storing the preconditioned directions (flexible
// GMRES), x0 = 0, modified Gram-Schmidt, complex Givens rotations, all
// right-hand sides advancing together.  A right-hand side leaves the current
// cycle when its recurrence residual |g_{j+1}| / ||f|| reaches rtol; at the
// end of every cycle the true FP64 residual f - A x is formed and decides:
// a right-hand side is converged only when ||f - A x|| / ||f|| <= rtol, the
// others start a new cycle from that residual until maxit.
static int solve_gmres(th_ctx *c, const c64 *f, c64 *u, int nrhs, const th_solve_opts *o,
                       th_solve_stats *stats) {
  hipStream_t s = c->stream;
  const bool f32 = o->precond_dtype == TH_C64;
  const int maxit = o->maxit;
  const int m = (o->restart > 0) ? std::min(o->restart, maxit) : maxit;
  SolverWS w;
  int rc = ensure_solver_ws(c, m, nrhs, f32, w);
  if (rc) return rc;
  const size_t vbytes = (size_t)nrhs * c->nf * sizeof(c64);
  const long long nf = c->nf;
  const long long ldj = (long long)(c->kv_vec_bytes / sizeof(c64));  // stride between basis vectors
  std::vector<c64 *> Vp, Zp;  // basis vectors reached so far
  auto Vj = [&](int j) { return Vp[j]; };
  auto Zj = [&](int j) { return Zp[j]; };
  auto reach = [&](std::vector<c64 *> &P, std::vector<void *> &blocks, int j) -> int {
    while ((int)P.size() <= j) {
      c64 *q = nullptr;
      int e = basis_vec(c, blocks, (int)P.size(), &q);
      if (e) return e;
      P.push_back(q);
    }
    return 0;
  };

  std::vector<zc> fn2;
  rc = dot_to_host(c, f, f, nrhs, w, fn2);
  if (rc) return rc;
  std::vector<double> fnorm(nrhs);
  for (int r = 0; r < nrhs; ++r) {
    fnorm[r] = std::sqrt(std::max(fn2[r].real(), 0.0));
    if (!std::isfinite(fnorm[r])) {
      set_error("right-hand side contains NaN or Inf");
      return TH_ENUMERIC;
    }
  }
  TH_HIP_CHECK_RET(hipMemsetAsync(u, 0, vbytes, s));
  // x0 = 0: the first residual is f itself
  TH_HIP_CHECK_RET(hipMemcpyAsync(w.res, f, vbytes, hipMemcpyDeviceToDevice, s));
  std::vector<double> beta(fnorm);        // true residual norms of the current iterate
  std::vector<int> done(nrhs, 0), it_r(nrhs, 0);
  for (int r = 0; r < nrhs; ++r) done[r] = fnorm[r] == 0.0 || beta[r] <= o->rtol * fnorm[r];
  int total = 0;
  long long nprec = 0;
  std::vector<double> hscal(nrhs);
  auto all_done = [&]() {
    for (int r = 0; r < nrhs; ++r)
      if (!done[r]) return false;
    return true;
  };
  while (!all_done() && total < maxit) {
    rc = reach(Vp, c->kv_V, 0);
    if (rc) return rc;
    // V_0 = r / beta for the right-hand sides still running, 0 for the others
    for (int r = 0; r < nrhs; ++r) hscal[r] = (!done[r] && beta[r] > 0.0) ? 1.0 / beta[r] : 0.0;
    TH_HIP_CHECK_RET(hipMemcpyAsync(w.scal, hscal.data(), nrhs * sizeof(double),
                                    hipMemcpyHostToDevice, s));
    rc = launch_scale_dev(Vj(0), w.res, w.scal, nf, nrhs, nf, nf, s);
    if (rc) return rc;
    // rotated Hessenberg (upper triangular R) stored by columns as they grow:
    // H[r][q][i] = R(i, q), i <= q
    std::vector<std::vector<std::vector<zc>>> H(nrhs);
    std::vector<std::vector<zc>> g(nrhs, std::vector<zc>(m + 1, 0.0)), cs(nrhs, std::vector<zc>(m)),
        sn(nrhs, std::vector<zc>(m));
    std::vector<int> jend(nrhs, 0), active(nrhs);
    for (int r = 0; r < nrhs; ++r) {
      g[r][0] = beta[r];
      active[r] = !done[r];
    }
    int j = 0;
    bool cycle_done = false;
    for (j = 0; j < m && !cycle_done; ++j) {
      rc = reach(Vp, c->kv_V, j + 1);
      if (!rc) rc = reach(Zp, c->kv_Z, j);
      if (rc) return rc;
      rc = precond(c, Vj(j), Zj(j), nrhs, f32, w, o->use_graph != 0);
      if (rc) return rc;
      nprec += nrhs;
      {
        KTimer kt(c, TH_KT_OPERATOR);
        rc = launch_apply(make_op(c, false), c->ref, Zj(j), nullptr, Vj(j + 1), nrhs, false, 1.0, s);
      }
      if (rc) return rc;
      // modified Gram-Schmidt: coefficients stay on the device (column j of
      // the Hessenberg matrix in w.hcol), the new vector is normalised by a
      // device-computed 1/norm, and one copy brings the column to the host;
      // short vectors with many right-hand sides take the whole step in one
      // launch (a workgroup per right-hand side); otherwise each projection
      // is one launch, the axpy that finishes the fixed-order sum of its
      // partial dot products fused with the partial dot products of the next
      // projection (after the last one: of the squared norm)
      std::vector<std::vector<zc>> hcol(nrhs, std::vector<zc>(j + 2, 0.0));
      if (mgs_step_fits(nf, nrhs, j + 1)) {
        // short vectors, many right-hand sides: the whole step in one launch
        KTimer kt(c, TH_KT_KRYLOV);
        MgsBasis B{};
        for (int i = 0; i <= j; ++i) B.v[i] = Vj(i);
        rc = launch_mgs_step(B, j + 1, Vj(j + 1), w.hcol, nf, nrhs, nf, s);
      } else {
        KTimer kt(c, TH_KT_KRYLOV);
        c64 *pin = w.partial, *pout = w.partial2;
        rc = launch_dot_partial(Vj(0), Vj(j + 1), nf, nrhs, nf, nf, pin, s);
        for (int i = 0; i <= j && rc == 0; ++i) {
          rc = launch_axpy_dot_partials(Vj(j + 1), Vj(i), i < j ? Vj(i + 1) : Vj(j + 1), pin,
                                        w.hcol + (size_t)i * nrhs, -1.0, nf, nrhs, nf, pout, s);
          std::swap(pin, pout);
        }
        if (!rc)
          rc = launch_scale_partials(Vj(j + 1), pin, w.hcol + (size_t)(j + 1) * nrhs, nf, nrhs,
                                     nf, s);
      }
      if (rc) return rc;
      TH_HIP_CHECK_RET(hipMemcpyAsync(w.hcol_h, w.hcol, (size_t)(j + 2) * nrhs * sizeof(c64),
                                      hipMemcpyDeviceToHost, s));
      TH_HIP_CHECK_RET(hipStreamSynchronize(s));
      for (int r = 0; r < nrhs; ++r) {
        for (int i = 0; i <= j; ++i) {
          const c64 v = w.hcol_h[(size_t)i * nrhs + r];
          hcol[r][i] = zc(v.re, v.im);
        }
        hcol[r][j + 1] = std::sqrt(std::max(w.hcol_h[(size_t)(j + 1) * nrhs + r].re, 0.0));
      }
      ++total;
      bool cycle_finished = true;
      for (int r = 0; r < nrhs; ++r) {
        if (!active[r]) continue;
        std::vector<zc> &h = hcol[r];
        const double hsub = std::abs(h[j + 1]);  // before the rotation zeroes it
        if (!std::isfinite(hsub)) {
          set_error("NaN or Inf in the Arnoldi process");
          return TH_ENUMERIC;
        }
        for (int i = 0; i < j; ++i) {
          zc t = cs[r][i] * h[i] + sn[r][i] * h[i + 1];
          h[i + 1] = -std::conj(sn[r][i]) * h[i] + std::conj(cs[r][i]) * h[i + 1];
          h[i] = t;
        }
        zc rr;
        givens(h[j], h[j + 1], cs[r][j], sn[r][j], rr);
        h[j] = rr;
        h[j + 1] = 0.0;
        g[r][j + 1] = -std::conj(sn[r][j]) * g[r][j];
        g[r][j] = cs[r][j] * g[r][j];
        H[r].emplace_back(h.begin(), h.begin() + j + 1);
        jend[r] = j + 1;
        it_r[r] = total;
        const double rel = std::abs(g[r][j + 1]) / fnorm[r];
        if (rel <= o->rtol || hsub == 0.0)
          active[r] = 0;  // leaves this cycle; the true residual decides below
        else
          cycle_finished = false;
      }
      if (cycle_finished || total >= maxit) cycle_done = true;
    }
    // x += Z y for every right-hand side of this cycle
    std::vector<c64> coef((size_t)nrhs * m, c64{0, 0});
    for (int r = 0; r < nrhs; ++r) {
      const int je = jend[r];
      std::vector<zc> y(je, 0.0);
      for (int i = je - 1; i >= 0; --i) {
        zc acc = g[r][i];
        for (int q = i + 1; q < je; ++q) acc -= H[r][q][i] * y[q];
        y[i] = acc / H[r][i][i];
      }
      for (int i = 0; i < je; ++i) coef[(size_t)r * m + i] = c64{y[i].real(), y[i].imag()};
    }
    TH_HIP_CHECK_RET(hipMemcpyAsync(w.coef, coef.data(), coef.size() * sizeof(c64),
                                    hipMemcpyHostToDevice, s));
    for (int b = 0; b * KV_CHUNK < j; ++b) {
      const int cnt = std::min(KV_CHUNK, j - b * KV_CHUNK);
      rc = launch_lincomb(u, Zj(b * KV_CHUNK), w.coef + b * KV_CHUNK, cnt, m, nf, nrhs, ldj, nf, s);
      if (rc) return rc;
    }
    // true FP64 residual of the new iterate: the convergence test and the
    // start of the next cycle
    rc = launch_apply(make_op(c, false), c->ref, u, f, w.res, nrhs, false, -1.0, s);
    if (rc) return rc;
    std::vector<zc> rn;
    rc = dot_to_host(c, w.res, w.res, nrhs, w, rn);
    if (rc) return rc;
    for (int r = 0; r < nrhs; ++r) {
      beta[r] = std::sqrt(std::max(rn[r].real(), 0.0));
      if (!std::isfinite(beta[r])) {
        set_error("NaN or Inf in the residual");
        return TH_ENUMERIC;
      }
      done[r] = fnorm[r] == 0.0 || beta[r] <= o->rtol * fnorm[r];
    }
  }
  double worst = 0.0;
  int maxits = 0;
  for (int r = 0; r < nrhs; ++r) {
    worst = std::max(worst, fnorm[r] > 0 ? beta[r] / fnorm[r] : 0.0);
    maxits = std::max(maxits, it_r[r]);
  }
  if (stats) {
    stats->iters = maxits;
    stats->rel_res = worst;
    stats->n_precond = nprec;
  }
  if (!all_done()) {
    set_error("GMRES reached maxit before the true residual met the tolerance");
    return TH_ENOTCONV;
  }
  return 0;
}

static int solve_stationary(th_ctx *c, const c64 *f, c64 *u, int nrhs, const th_solve_opts *o,
                            th_solve_stats *stats) {
  hipStream_t s = c->stream;
  const bool f32 = o->precond_dtype == TH_C64;
  SolverWS w;
  int rc = ensure_solver_ws(c, 1, nrhs, f32, w);
  if (rc) return rc;
  const long long nf = c->nf;
  const size_t vbytes = (size_t)nrhs * nf * sizeof(c64);
  c64 *zdir = nullptr;
  rc = basis_vec(c, c->kv_Z, 0, &zdir);
  if (rc) return rc;
  std::vector<zc> fn2;
  rc = dot_to_host(c, f, f, nrhs, w, fn2);
  if (rc) return rc;
  std::vector<double> fnorm(nrhs);
  for (int r = 0; r < nrhs; ++r) {
    fnorm[r] = std::sqrt(std::max(fn2[r].real(), 0.0));
    if (!std::isfinite(fnorm[r])) {
      set_error("right-hand side contains NaN or Inf");
      return TH_ENUMERIC;
    }
  }
  TH_HIP_CHECK_RET(hipMemsetAsync(u, 0, vbytes, s));
  int it = 0;
  double worst = 0.0;
  while (it < o->maxit) {
    // u <- u + B (f - A u)  (= TwoGridStep(u, f) for the linear two-grid map)
    rc = launch_apply(make_op(c, false), c->ref, u, f, w.res, nrhs, false, -1.0, s);
    if (!rc) rc = precond(c, w.res, zdir, nrhs, f32, w, o->use_graph != 0);
    if (rc) return rc;
    c64 one = {1.0, 0.0};
    std::vector<c64> ones(nrhs, one);
    TH_HIP_CHECK_RET(hipMemcpyAsync(w.hd, ones.data(), nrhs * sizeof(c64), hipMemcpyHostToDevice, s));
    rc = launch_axpy_dev(u, zdir, w.hd, 1.0, nf, nrhs, nf, nf, s);
    if (rc) return rc;
    ++it;
    rc = launch_apply(make_op(c, false), c->ref, u, f, w.res, nrhs, false, -1.0, s);
    if (rc) return rc;
    std::vector<zc> rn;
    rc = dot_to_host(c, w.res, w.res, nrhs, w, rn);
    if (rc) return rc;
    worst = 0.0;
    for (int r = 0; r < nrhs; ++r)
      worst = std::max(worst, fnorm[r] > 0 ? std::sqrt(std::max(rn[r].real(), 0.0)) / fnorm[r] : 0.0);
    if (!std::isfinite(worst)) {
      set_error("stationary iteration diverged to NaN/Inf");
      return TH_ENUMERIC;
    }
    if (worst <= o->rtol) break;
  }
  if (stats) {
    stats->iters = it;
    stats->rel_res = worst;
    stats->n_precond = (long long)it * nrhs;
  }
  if (worst > o->rtol) {
    set_error("stationary iteration reached maxit before the tolerance");
    return TH_ENOTCONV;
  }
  return 0;
}

}  // namespace th

extern "C" th_status th_solve(th_ctx *ctx, const void *f, void *u, int nrhs,
                              const th_solve_opts *opts, th_solve_stats *stats) {
  th_status st = check_vec_call(ctx, f, u, nrhs, TH_C128, true);
  if (st) return st;
  if (!opts) return fail(ctx, TH_EINVAL, "null options");
  if (!(opts->rtol > 0.0) || opts->maxit < 1) return fail(ctx, TH_EINVAL, "rtol > 0 and maxit >= 1 required");
  if (opts->precond_dtype != TH_C128 && opts->precond_dtype != TH_C64)
    return fail(ctx, TH_EINVAL, "unknown preconditioner dtype");
  if (stats) std::memset(stats, 0, sizeof(*stats));
  auto t0 = std::chrono::steady_clock::now();
  int rc;
  if (opts->krylov == TH_KRYLOV_GMRES_RIGHT || opts->krylov == TH_KRYLOV_FGMRES)
    rc = solve_gmres(ctx, (const c64 *)f, (c64 *)u, nrhs, opts, stats);
  else if (opts->krylov == TH_KRYLOV_STATIONARY)
    rc = solve_stationary(ctx, (const c64 *)f, (c64 *)u, nrhs, opts, stats);
  else
    return fail(ctx, TH_EINVAL, "unknown Krylov method");
  if (hipStreamSynchronize(ctx->stream) != hipSuccess && rc == 0) rc = TH_EHIP;
  if (stats) {
    stats->t_solve_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    stats->t_cycle_s = stats->iters > 0 ? stats->t_solve_s / stats->iters : 0.0;
    stats->n_fallback_cells = ctx->n_fallback;
  }
  return finish(ctx, rc);
}
