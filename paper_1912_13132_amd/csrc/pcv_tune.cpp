// Autotuner for the launch shapes and the schedule of a theta-evaluation:
// times pcv_eval under the candidate choices that change one of this
// problem's launches and keeps the fastest; choices are cached in a text
// file keyed by the device, the runtime, this library's build and the
// problem's padded sizes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "pcv_host.h"

using pcv::fail;

namespace pcv {
namespace {

struct Cfg {
  int32_t small_npad, max_wg;
  bool two_groups;
};

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

uint64_t fnv1a(uint64_t h, const void* data, size_t n) {
  const unsigned char* b = static_cast<const unsigned char*>(data);
  for (size_t i = 0; i < n; ++i) {
    h ^= b[i];
    h *= 1099511628211ull;
  }
  return h;
}

// Cache key: architecture, runtime version, library build, precision,
// refinement sweeps and the padded sizes of the evaluated subsets in LPT
// order (they fix every launch's shape and the schedule groups).
std::string cache_key(const pcv_problem* p) {
  hipDeviceProp_t prop;
  std::string arch = "unknown";
  if (hipGetDeviceProperties(&prop, p->device) == hipSuccess) arch = prop.gcnArchName;
  int rt = 0;
  (void)hipRuntimeGetVersion(&rt);
  uint64_t h = 1469598103934665603ull;
  const int32_t head[3] = {p->opt.prec, p->opt.max_refine, p->n_cu};
  h = fnv1a(h, head, sizeof(head));
  for (int32_t i : p->order_eval) h = fnv1a(h, &p->desc[i].npad, sizeof(int32_t));
  char buf[96];
  std::snprintf(buf, sizeof(buf), "%016llx", (unsigned long long)h);
  std::string key = arch + "|hip" + std::to_string(rt) + "|" + __DATE__ "_" __TIME__ + "|S" +
                    std::to_string(p->n_active) + "|" + buf;
  for (char& c : key)  // one whitespace-free field of the cache line
    if (c == ' ' || c == '\t' || c == '\n' || c == '\r') c = '_';
  return key;
}

bool cache_lookup(const char* path, const std::string& key, Cfg& c) {
  if (!path || !*path) return false;
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  bool found = false;
  char line[512];
  while (std::fgets(line, sizeof(line), f)) {
    char k[400];
    int a = 0, b = 0, g = 0;
    if (std::sscanf(line, "%399s %d %d %d", k, &a, &b, &g) == 4 && key == k && a >= 0 && b >= 0 && b <= 8) {
      c = Cfg{a, b, g != 0};  // the last matching line wins
      found = true;
    }
  }
  std::fclose(f);
  return found;
}

void cache_store(const char* path, const std::string& key, const Cfg& c, double best_s) {
  if (!path || !*path) return;
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "%s %d %d %d %.6e\n", key.c_str(), c.small_npad, c.max_wg, c.two_groups ? 1 : 0, best_s);
  std::fclose(f);
}

// The launches a configuration produces: per schedule group, its size and
// shape, and the sharing plan of the first launch.  Candidates with the same
// signature launch the same work and are timed once.
std::vector<int64_t> signature(pcv_problem* p, const Cfg& c) {
  const int32_t s0 = p->tune_small_npad, w0 = p->opt.max_wg_per_subset;
  const bool g0 = p->tune_two_groups;
  p->tune_small_npad = c.small_npad;
  p->tune_two_groups = c.two_groups;
  p->opt.max_wg_per_subset = c.max_wg;
  std::vector<int64_t> sig;
  const bool mixed = p->opt.prec == PCV_PREC_MIXED;
  const int K = c.two_groups && p->groups.size() > 1 ? (int)p->groups.size() : 1;
  for (int k = 0; k < K; ++k) {
    const pcv_group& G = K > 1 ? p->groups[k] : p->g_all;
    const int32_t np = G.cnt > 0 ? p->desc[p->order_eval[G.o0]].npad : 0;
    sig.push_back(G.cnt);
    sig.push_back(mixed && np <= c.small_npad ? 256 : 512);
  }
  // sharing plan (as plan_coop makes it), only where the first launch can share
  std::vector<int32_t> co = p->coop_order, ci = p->coop_info;
  const int32_t cb = p->coop_blocks, cs = p->coop_slots, cg = p->coop_group_cnt;
  plan_coop(p);
  const bool first_wide = !mixed || sig[1] == 512;
  if (first_wide)
    for (int32_t v : p->coop_info) sig.push_back(v);
  p->coop_order = co;
  p->coop_info = ci;
  p->coop_blocks = cb;
  p->coop_slots = cs;
  p->coop_group_cnt = cg;
  p->tune_small_npad = s0;
  p->tune_two_groups = g0;
  p->opt.max_wg_per_subset = w0;
  return sig;
}

}  // namespace

pcv_status autotune_impl(pcv_problem* p, const pcv_theta& th, const char* cache_path, int32_t reps,
                         pcv_tune_report* rep) {
  const double t_start = now_s();
  if (p->served) return fail(PCV_ERR_STATE, "pcv_autotune: the problem is held by a server");
  pcv_tune_report r;
  std::memset(&r, 0, sizeof(r));
  const std::string key = cache_key(p);
  Cfg best{p->tune_small_npad, p->opt.max_wg_per_subset ? p->opt.max_wg_per_subset : 8, p->tune_two_groups};
  if (cache_lookup(cache_path, key, best)) {
    pcv_status s = apply_tuning(p, best.small_npad, best.max_wg, best.two_groups);
    if (s != PCV_OK) return s;
    r.from_cache = 1;
  } else {
    // on an error the problem goes back to the configuration it had
    const Cfg orig = best;
    auto restore = [&](pcv_status s) {
      (void)apply_tuning(p, orig.small_npad, orig.max_wg, orig.two_groups);
      return s;
    };
    std::vector<std::vector<int64_t>> seen;
    std::vector<double> seen_t;
    auto time_cfg = [&](const Cfg& c, double* out) -> pcv_status {
      const std::vector<int64_t> sig = signature(p, c);
      for (size_t k = 0; k < seen.size(); ++k)
        if (seen[k] == sig) {
          *out = seen_t[k];
          return PCV_OK;
        }
      pcv_status s = apply_tuning(p, c.small_npad, c.max_wg, c.two_groups);
      if (s != PCV_OK) return s;
      double loss = 0.0;
      s = eval_impl(p, th, &loss, nullptr);  // warm-up: captures the graph
      if (s != PCV_OK) return s;
      std::vector<double> t;
      for (int i = 0; i < reps; ++i) {
        const double t0 = now_s();
        s = eval_impl(p, th, &loss, nullptr);
        if (s != PCV_OK) return s;
        t.push_back(now_s() - t0);
      }
      std::sort(t.begin(), t.end());
      *out = t[t.size() / 2];
      seen.push_back(sig);
      seen_t.push_back(*out);
      ++r.n_timed;
      return PCV_OK;
    };
    double best_t = 0.0;
    pcv_status s = time_cfg(best, &best_t);
    if (s != PCV_OK) return restore(s);
    r.default_s = best_t;
    const bool mixed = p->opt.prec == PCV_PREC_MIXED;
    if (mixed)
      for (int32_t sn : {0, 1024, 1408, 1536, 2048, 3072, 4096}) {
        Cfg c = best;
        c.small_npad = sn;
        double t = 0.0;
        if ((s = time_cfg(c, &t)) != PCV_OK) return restore(s);
        if (t < best_t) best = c, best_t = t;
      }
    for (int32_t w : {1, 2, 3, 4, 6, 8}) {
      Cfg c = best;
      c.max_wg = w;
      double t = 0.0;
      if ((s = time_cfg(c, &t)) != PCV_OK) return restore(s);
      if (t < best_t) best = c, best_t = t;
    }
    if (p->groups.size() > 1)
      for (bool g : {true, false}) {
        Cfg c = best;
        c.two_groups = g;
        double t = 0.0;
        if ((s = time_cfg(c, &t)) != PCV_OK) return restore(s);
        if (t < best_t) best = c, best_t = t;
      }
    if ((s = apply_tuning(p, best.small_npad, best.max_wg, best.two_groups)) != PCV_OK) return restore(s);
    r.best_s = best_t;
    cache_store(cache_path, key, best, best_t);
  }
  r.small_npad = p->tune_small_npad;
  r.max_wg_per_subset = p->opt.max_wg_per_subset;
  r.two_groups = p->tune_two_groups ? 1 : 0;
  r.tuning_s = now_s() - t_start;
  if (rep) *rep = r;
  return PCV_OK;
}

}  // namespace pcv
