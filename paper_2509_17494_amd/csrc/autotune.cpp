// Autotuner of the matrix-core smoother: at setup every candidate
// (waves per workgroup, column chunk, persistent grid size) is timed with HIP
// events on the real subdomain operators and max_rhs right-hand sides, and the
// fastest is kept.  Results are cached per problem shape and device in the
// text file named by the environment variable TH_AUTOTUNE_CACHE (if set), one
// line "key cfg grid ms" per shape.  TH_MFMA_CFG=<index>[,<grid>] skips the
// search and takes that configuration when it applies to the problem.
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <sstream>
#include <string>

#include "ctx.hpp"

namespace th {

static std::string shape_key(const th_ctx *c) {
  int max_nu = 0, max_no = 0;
  for (const Sub &s : c->subs) {
    max_nu = std::max(max_nu, s.nU);
    max_no = std::max(max_no, s.nOm);
  }
  hipDeviceProp_t prop{};
  (void)hipGetDeviceProperties(&prop, c->device);
  std::ostringstream k;
  k << prop.gcnArchName << "/cu" << prop.multiProcessorCount << "/s" << c->subs.size() << "/u"
    << max_nu << "/o" << max_no << "/r" << c->desc.max_rhs;
  std::string key = k.str();
  for (char &ch : key)
    if (ch == ' ' || ch == ':') ch = '_';
  return key;
}

static bool cache_lookup(const std::string &key, int &cfg, int &grid, double &ms) {
  const char *path = std::getenv("TH_AUTOTUNE_CACHE");
  if (!path) return false;
  std::ifstream in(path);
  std::string k;
  int c0, g0;
  double t0;
  bool found = false;
  while (in >> k >> c0 >> g0 >> t0)
    if (k == key && c0 >= 0 && c0 < mfma_num_configs() && g0 >= 0) {
      cfg = c0;
      grid = g0;
      ms = t0;
      found = true;
    }
  return found;
}

static void cache_store(const std::string &key, int cfg, int grid, double ms) {
  const char *path = std::getenv("TH_AUTOTUNE_CACHE");
  if (!path) return;
  std::ofstream out(path, std::ios::app);
  out << key << " " << cfg << " " << grid << " " << ms << "\n";
}

// Every candidate is timed as the smoother's subdomain step: the batched
// apply followed by the averaged update that reads its output (the staged
// kernel writes colour planes, the chunked kernels the packed Y rows).
int autotune_mfma(th_ctx *c) {
  hipStream_t s = c->stream;
  const int nrhs = c->desc.max_rhs;
  const std::string key = shape_key(c);
  int cfg = 0, grid = 0;
  double best = 0;
  // TH_MFMA_CFG=<index>[,<grid>] forces a configuration (tests and measurements)
  if (const char *force = std::getenv("TH_MFMA_CFG")) {
    int f = -1, g = 0;
    if (std::sscanf(force, "%d,%d", &f, &g) >= 1 && g >= 0 && mfma_cfg_usable(c, f)) {
      c->mfma_cfg = f;
      c->mfma_grid = mfma_cfg_staged(f) ? 0 : g;
      c->tune_report = "forced";
      return 0;
    }
  }
  if (cache_lookup(key, cfg, grid, best) && mfma_cfg_usable(c, cfg)) {
    c->mfma_cfg = cfg;
    c->mfma_grid = grid;
    c->tune_report = "cache " + key;
    return 0;
  }
  TH_HIP_CHECK_RET(hipMemsetAsync(c->w_r, 0, (size_t)nrhs * c->nf * sizeof(c32), s));
  void *uout = nullptr;
  if (hipMalloc(&uout, (size_t)nrhs * c->nf * sizeof(c32)) != hipSuccess) {
    set_error("cannot allocate the autotuner's output vector");
    return TH_ENOMEM;
  }
  hipDeviceProp_t prop{};
  TH_HIP_CHECK_RET(hipGetDeviceProperties(&prop, c->device));
  const int cu = prop.multiProcessorCount;
  const int grids[] = {0, cu, 2 * cu, 4 * cu};
  hipEvent_t e0, e1;
  TH_HIP_CHECK_RET(hipEventCreate(&e0));
  TH_HIP_CHECK_RET(hipEventCreate(&e1));
  best = 1e300;
  std::ostringstream rep;
  rep << key << ":";
  int rc = 0;
  const int saved = c->mfma_cfg;
  auto step = [&](int cf, int g) {
    c->mfma_cfg = cf;  // selects the matching averaged update
    int e = launch_dd_mfma(c, c->w_r, c->w_y, nrhs, true, cf, g, s);
    if (!e) e = launch_dd_accumulate(c, c->w_y, uout, nrhs, true, true, s);
    return e;
  };
  for (int cf = 0; cf < mfma_num_configs() && rc == 0; ++cf) {
    if (!mfma_cfg_usable(c, cf)) continue;
    for (int g : grids) {
      if (mfma_cfg_staged(cf) && g != 0) continue;  // one workgroup per item, no grid choice
      rc = step(cf, g);  // warm-up
      if (rc) break;
      (void)hipEventRecord(e0, s);
      const int reps = 3;
      for (int i = 0; i < reps && rc == 0; ++i) rc = step(cf, g);
      (void)hipEventRecord(e1, s);
      if (hipEventSynchronize(e1) != hipSuccess) {
        rc = TH_EHIP;
        set_error("event synchronisation failed in the autotuner");
        break;
      }
      float ms = 0;
      (void)hipEventElapsedTime(&ms, e0, e1);
      const double t = ms / reps;
      rep << " cfg" << cf << "/g" << g << "=" << t;
      if (t < best) {
        best = t;
        cfg = cf;
        grid = g;
      }
    }
  }
  c->mfma_cfg = saved;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipStreamSynchronize(s);
  (void)hipFree(uout);
  if (rc) return rc;
  c->mfma_cfg = cfg;
  c->mfma_grid = grid;
  rep << " -> cfg" << cfg << "/g" << grid;
  c->tune_report = rep.str();
  cache_store(key, cfg, grid, best);
  return 0;
}

}  // namespace th
