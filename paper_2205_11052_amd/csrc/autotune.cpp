// Launch-shape autotuner of the stage kernel.
//
// Every implemented launch shape -- the node-per-thread kernel with each
// elements-per-work-group value x work-groups per compute unit of the
// persistent grid (0 meaning one work-group per block of elements), and the
// lane-per-field kernel where it supports the order -- is timed with HIP events on the
// context's stream over real stage launches of the context's own workload,
// writing into scratch buffers so the solver state is untouched.  The fastest
// shape is kept; with a cache path the choice is stored in a flat JSON object
// keyed by order, precision, element count and shot count, and read back on
// later calls instead of timing again.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <fstream>
#include <map>
#include <sstream>
#include <string>

#include "../../include/dgw.h"
#include "dgw_ctx.h"

using namespace dgw;

namespace {

std::map<std::string, long> read_cache(const char *path) {
  std::map<std::string, long> out;
  std::ifstream f(path);
  if (!f) return out;
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string s = ss.str();
  size_t p = 0;
  while ((p = s.find('"', p)) != std::string::npos) {
    const size_t q = s.find('"', p + 1);
    if (q == std::string::npos) break;
    const std::string key = s.substr(p + 1, q - p - 1);
    size_t colon = s.find(':', q);
    if (colon == std::string::npos) break;
    long v = 0;
    if (std::sscanf(s.c_str() + colon + 1, " %ld", &v) == 1) out[key] = v;
    p = colon + 1;
  }
  return out;
}

bool write_cache(const char *path, const std::map<std::string, long> &m) {
  std::ofstream f(path);
  if (!f) return false;
  f << "{";
  bool first = true;
  for (const auto &kv : m) {
    f << (first ? "" : ",") << "\n  \"" << kv.first << "\": " << kv.second;
    first = false;
  }
  f << "\n}\n";
  return (bool)f;
}


}  // namespace

struct Shape {
  int kernel, be, wpc;
  long code() const { return kernel * 1000000L + be * 1000L + wpc; }
};

extern "C" int dgw_autotune(dgw_ctx *c, const char *cache_path, int *kernel,
                            int *elems_per_block, int *wgs_per_cu) {
  if (!c) return DGW_EINVAL;
  RoctxRange range("dgw_autotune");
  if (!c->have_mesh || !c->have_mat || !c->have_dt)
    return c->fail(DGW_ESTATE, "mesh, material and dt must be set first");
  char key[128];
  std::snprintf(key, sizeof key, "N%d_fp%d_K%lld_S%d%s", c->R.N, c->precision,
                (long long)c->mesh.K, c->nshots, c->have_aniso ? "_aniso" : "");
  std::vector<Shape> opts;
  for (int kv : {0, 1})
    for (int be : stage_block_choices(kv, c->R.N, c->precision))
      for (int w : {0, 1, 2, 3, 4, 8, 16}) opts.push_back({kv, be, w});
  // the minimal-form kernel: one shape (16 elements, one work-group each)
  if (!c->have_aniso)
    for (int be : stage_block_choices(2, c->R.N, c->precision)) opts.push_back({2, be, 0});
  auto report = [&](const Shape &o) {
    if (kernel) *kernel = o.kernel;
    if (elems_per_block) *elems_per_block = o.be;
    if (wgs_per_cu) *wgs_per_cu = o.wpc;
  };
  std::map<std::string, long> cache;
  if (cache_path) {
    cache = read_cache(cache_path);
    auto it = cache.find(key);
    if (it != cache.end())
      for (const auto &o : opts)
        if (o.code() == it->second) {
          int rc = dgw_set_launch(c, o.kernel, o.be, o.wpc);
          report(o);
          return rc;
        }
  }
  const size_t n = (size_t)c->nshots * c->mesh.K * 9 * c->R.Np * c->real_size();
  void *out = c->dalloc(n), *res = c->dalloc(n);
  if (!out || !res) {
    c->dfree(out);
    c->dfree(res);
    return c->fail(DGW_ENOMEM, "device allocation failed (autotune scratch)");
  }
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  Shape best = opts[0];
  float best_ms = 1e30f;
  int rc = DGW_OK;
  // two passes over the candidates, each shape's best time counting: the
  // first shapes of a single pass run while the clocks are still rising
  for (int pass = 0; pass < 2 && rc == DGW_OK; ++pass) {
    for (const auto &o : opts) {
      hipError_t err = hipSuccess;
      const int reps = 10;
      for (int r = 0; r < reps + 2 && err == hipSuccess; ++r) {
        if (r == 2) (void)hipEventRecord(e0, c->stream);
        // every stage index in turn (the first stage reads no residual),
        // each twice over the reps
        const int si = r % 5;
        if (c->precision == 64) {
          StageArgs<double> a;
          stage_args(c, a, c->d_q[c->cur], out, res, c->d_step, si);
          err = launch_stage(o.kernel, c->R.N, 64, o.be, o.wpc, c->ncu, c->nshots, &a,
                             c->stream);
        } else {
          StageArgs<float> a;
          stage_args(c, a, c->d_q[c->cur], out, res, c->d_step, si);
          err = launch_stage(o.kernel, c->R.N, 32, o.be, o.wpc, c->ncu, c->nshots, &a,
                             c->stream);
        }
      }
      if (err != hipSuccess) {
        rc = c->hipfail(err, "autotune launch");
        break;
      }
      (void)hipEventRecord(e1, c->stream);
      (void)hipEventSynchronize(e1);
      float ms = 0;
      (void)hipEventElapsedTime(&ms, e0, e1);
      ms /= reps;
      if (ms < best_ms) {
        best_ms = ms;
        best = o;
      }
    }
  }
  (void)hipStreamSynchronize(c->stream);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  c->dfree(out);
  c->dfree(res);
  if (rc) return rc;
  if ((rc = dgw_set_launch(c, best.kernel, best.be, best.wpc))) return rc;
  report(best);
  if (cache_path) {
    cache[key] = best.code();
    if (!write_cache(cache_path, cache))
      return c->fail(DGW_EINVAL, std::string("cannot write ") + cache_path);
  }
  return DGW_OK;
}
