// Call sequences of the C ABI run against the CPU stand-in of the HIP
// runtime (hip_stub.cpp), under AddressSanitizer / UBSan: problem creation
// with two schedule groups and shared launches planned, graph capture and
// replay, eager and profiled evaluations, batched and grid evaluations,
// factorisation, prediction, GLS, a server that toggles the problem's
// served mode, forced fallbacks, the memory cap, and the tuner with its
// cache, each repeated on fresh problems.  After every problem is
// destroyed the stand-in must hold no allocation, pinned buffer, stream or
// event more than before it was created.
//
// usage: driver <scenario> [cache path]
//   scenario: sequence | oom | tune
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <string>
#include <vector>

#include "pcv.h"

extern "C" {
int64_t stub_live_allocations();
int64_t stub_live_pinned();
int64_t stub_live_streams();
int64_t stub_live_events();
void stub_report(const char* tag);
void stub_fail_malloc_after(int64_t n);
void stub_fail_launch_after(int64_t n);
}

#define CHECK(x)                                                                                   \
  do {                                                                                             \
    pcv_status s_ = (x);                                                                           \
    if (s_ != PCV_OK) {                                                                            \
      std::fprintf(stderr, "%s:%d %s -> %s: %s\n", __FILE__, __LINE__, #x, pcv_status_string(s_), \
                   pcv_last_error());                                                              \
      std::exit(1);                                                                                \
    }                                                                                              \
  } while (0)
#define EXPECT(c)                                                                  \
  do {                                                                             \
    if (!(c)) {                                                                    \
      std::fprintf(stderr, "%s:%d expectation failed: %s\n", __FILE__, __LINE__, #c); \
      std::exit(1);                                                                \
    }                                                                              \
  } while (0)

struct Data {
  int64_t n = 0;
  std::vector<double> locs, y, rect;
  std::vector<int64_t> tptr{0}, vptr{0};
  std::vector<int32_t> tidx, vidx;
  int32_t S = 0;
};

// S independent subsets; subset i lives in [i, i+1) x [0, 1).  A few large
// ones (padded to >= 2,048 rows) so that the first launch shares them; more
// subsets than compute units and not a whole number of rounds, so the
// evaluation runs as two schedule groups.
Data make_data(int S, unsigned seed) {
  Data d;
  std::mt19937_64 r(seed);
  std::uniform_real_distribution<double> u(0.0, 1.0);
  std::normal_distribution<double> g;
  for (int i = 0; i < S; ++i) {
    const int nt = i == 0 ? 3000 : i == 1 ? 2500 : i == 2 ? 2100 : 40 + (int)(u(r) * 150);
    const int nv = i == 5 ? 0 : 1 + (int)(u(r) * 10);
    for (int k = 0; k < nt + nv; ++k) {
      d.locs.push_back(i + u(r));
      d.locs.push_back(u(r));
      d.y.push_back(g(r));
      if (k < nt)
        d.tidx.push_back((int32_t)d.n);
      else
        d.vidx.push_back((int32_t)d.n);
      ++d.n;
    }
    d.tptr.push_back((int64_t)d.tidx.size());
    d.vptr.push_back((int64_t)d.vidx.size());
    d.rect.insert(d.rect.end(), {(double)i, 0.0, (double)i + 1, 1.0});
  }
  d.S = S;
  return d;
}

pcv_theta th(double range, double lam) { return pcv_theta{PCV_COV_EXP, range, lam, 1.0}; }

pcv_problem* create(const Data& d, const pcv_options& o) {
  pcv_problem* p = nullptr;
  CHECK(pcv_problem_create(&p, d.n, d.locs.data(), d.y.data(), d.S, d.tptr.data(), d.tidx.data(),
                           d.vptr.data(), d.vidx.data(), d.rect.data(), &o));
  return p;
}

struct Live {
  int64_t a, p, s, e;
  static Live now() { return {stub_live_allocations(), stub_live_pinned(), stub_live_streams(), stub_live_events()}; }
  bool operator==(const Live& o) const { return a == o.a && p == o.p && s == o.s && e == o.e; }
};

void evals(pcv_problem* p, int k) {
  for (int i = 0; i < k; ++i) {
    double loss = -1;
    pcv_eval_report rep;
    std::memset(&rep, 0, sizeof(rep));
    std::vector<double> z(4096), ld(4096);
    rep.per_subset_sspe = z.data();
    rep.per_subset_logdet = ld.data();
    const pcv_theta t = th(0.3 + 0.01 * i, 0.1);
    CHECK(pcv_eval(p, &t, &loss, &rep));
    EXPECT(loss == 0.0);
  }
}

void sequence(const Data& d, int rep) {
  const Live base = Live::now();
  pcv_options o;
  pcv_default_options(&o);
  o.est_error = rep % 2;  // every other cycle with the error estimate's extra pass
  pcv_problem* p = create(d, o);
  evals(p, 3);
  std::vector<pcv_theta> ths;
  for (int k = 0; k < 70; ++k) ths.push_back(th(0.2 + 0.003 * k, 0.05 + 0.001 * k));
  std::vector<double> losses(70);
  CHECK(pcv_eval_batch(p, 70, ths.data(), losses.data()));
  CHECK(pcv_eval_batch(p, 9, ths.data(), losses.data()));
  std::vector<double> zg(9 * (size_t)d.S);
  std::vector<int32_t> best(d.S);
  CHECK(pcv_eval_grid(p, 9, ths.data(), losses.data(), zg.data(), best.data()));
  CHECK(pcv_factor(p, &ths[0]));
  std::vector<double> q, mean(300), var(300);
  std::mt19937_64 r(7 + rep);
  std::uniform_real_distribution<double> u(-0.5, d.S + 0.5);
  for (int k = 0; k < 300; ++k) {
    q.push_back(u(r));
    q.push_back(u(r) / d.S);
  }
  std::vector<int32_t> owner(300);
  CHECK(pcv_predict(p, 300, q.data(), mean.data(), var.data(), 0, owner.data()));
  CHECK(pcv_predict_noalloc(p, 120, q.data(), mean.data(), nullptr, 1, nullptr));
  std::vector<pcv_theta> loc(d.S, th(0.25, 0.08));
  CHECK(pcv_factor_local(p, loc.data()));
  std::vector<double> X(2 * (size_t)d.n, 1.0), beta(2 * (size_t)d.S);
  std::vector<int32_t> gst(d.S);
  CHECK(pcv_gls(p, 2, X.data(), beta.data(), gst.data()));
  // a server toggles the problem's served mode (drops and rebuilds the
  // captured evaluation and the post streams)
  for (int round = 0; round < 2; ++round) {
    pcv_server* srv = nullptr;
    CHECK(pcv_server_create(&srv, p, (size_t)64 << 20, 16));
    std::vector<pcv_ticket> tk;
    std::vector<std::vector<double>> outs;
    double l1 = -1, l2 = -1;
    for (int k = 0; k < 6; ++k) {
      const int nq = 1 + 40 * k;
      outs.emplace_back(2 * (size_t)nq);
      pcv_ticket t;
      CHECK(pcv_server_submit_predict(srv, nq, q.data(), outs.back().data(), outs.back().data() + nq, k & 1, &t));
      tk.push_back(t);
      if (k == 2) {
        CHECK(pcv_server_submit_eval(srv, &ths[3], &l1, &t));
        tk.push_back(t);
      }
    }
    pcv_ticket t;
    CHECK(pcv_server_submit_eval(srv, &ths[4], &l2, &t));
    tk.push_back(t);
    for (pcv_ticket x : tk) CHECK(pcv_server_wait(srv, x, -1.0));
    EXPECT(pcv_server_wait(srv, tk[0], 0.0) == PCV_ERR_INVALID);
    pcv_server_report sr;
    CHECK(pcv_server_report_get(srv, &sr));
    CHECK(pcv_server_destroy(srv));
    evals(p, 2);  // graph captured again after the served mode
  }
  CHECK(pcv_problem_destroy(p));
  // eager, profiled, forced fallback, device flag taken
  for (int variant = 0; variant < 4; ++variant) {
    pcv_options v;
    pcv_default_options(&v);
    if (variant == 0) v.graph = 0;
    if (variant == 1) v.profile = 1;
    if (variant == 2) v.debug_flags = 1;
    if (variant == 3) v.debug_flags = 2;
    pcv_problem* pv = create(d, v);
    evals(pv, 2);
    CHECK(pcv_eval_batch(pv, 5, ths.data(), losses.data()));
    CHECK(pcv_problem_destroy(pv));
  }
  const Live after = Live::now();
  if (!(after == base)) {
    stub_report("after sequence");
    std::fprintf(stderr, "resources left behind\n");
    std::exit(1);
  }
}

void oom(const Data& d) {
  const Live base = Live::now();
  for (size_t cap : {(size_t)4096, (size_t)1 << 20, (size_t)8 << 20}) {
    pcv_options o;
    pcv_default_options(&o);
    o.mem_cap_bytes = cap;
    pcv_problem* p = nullptr;
    const pcv_status s = pcv_problem_create(&p, d.n, d.locs.data(), d.y.data(), d.S, d.tptr.data(),
                                            d.tidx.data(), d.vptr.data(), d.vidx.data(), d.rect.data(), &o);
    EXPECT(s == PCV_ERR_OOM);
    EXPECT(p == nullptr);
    EXPECT(Live::now() == base);
  }
  std::printf("oom: rejected with nothing left behind\n");
}

// A device allocation that fails at every point of a multi-theta call:
// the call returns PCV_OK (the workspace or plan that did not fit is given
// up, the theta values go one at a time) or PCV_ERR_OOM (a single
// evaluation could not allocate), the problem's byte count matches what it
// holds, and the next call without the failure builds the workspace.
void oom_batch(const Data& d) {
  const Live base = Live::now();
  std::vector<pcv_theta> ths;
  for (int k = 0; k < 9; ++k) ths.push_back(th(0.2 + 0.01 * k, 0.05 + 0.005 * k));
  std::vector<double> losses(9);
  int ok = 0, oom = 0, dropped = 0;
  for (int64_t k = 0; k < 60; ++k) {
    pcv_options o;
    pcv_default_options(&o);
    pcv_problem* p = create(d, o);
    evals(p, 1);
    const int64_t a0 = stub_live_allocations();
    size_t b0 = 0;
    CHECK(pcv_problem_info(p, nullptr, nullptr, nullptr, &b0));
    stub_fail_malloc_after(k);
    const pcv_status s = pcv_eval_batch(p, 9, ths.data(), losses.data());
    stub_fail_malloc_after(-1);
    EXPECT(s == PCV_OK || s == PCV_ERR_OOM);
    if (s == PCV_OK) ++ok; else ++oom;
    size_t b1 = 0;
    CHECK(pcv_problem_info(p, nullptr, nullptr, nullptr, &b1));
    // nothing was allocated, or the workspace was kept (then more bytes)
    EXPECT((stub_live_allocations() == a0) == (b1 == b0));
    if (b1 == b0) ++dropped;
    CHECK(pcv_eval_batch(p, 9, ths.data(), losses.data()));
    CHECK(pcv_problem_destroy(p));
  }
  EXPECT(Live::now() == base);
  std::printf("oom_batch: %d calls ok, %d out of memory, %d gave the workspace up\n", ok, oom, dropped);
}

// Server creation failing at each device or pinned allocation in turn:
// PCV_ERR_OOM with the problem back as it was (its stream, not served, no
// resources left behind); a workspace no device holds fails the same way;
// the next creation works and serves.
void oom_server(const Data& d) {
  const Live base = Live::now();
  pcv_options o;
  pcv_default_options(&o);
  pcv_problem* p = create(d, o);
  pcv_theta t = th(0.2, 0.05);
  CHECK(pcv_factor(p, &t));
  evals(p, 1);
  const Live before = Live::now();
  int ok = 0, oom = 0;
  for (int64_t k = 0; k < 60; ++k) {
    pcv_server* srv = nullptr;
    stub_fail_malloc_after(k);
    const pcv_status s = pcv_server_create(&srv, p, (size_t)64 << 20, 4);
    stub_fail_malloc_after(-1);
    EXPECT(s == PCV_OK || s == PCV_ERR_OOM);
    if (s == PCV_OK) {
      ++ok;
      CHECK(pcv_server_destroy(srv));
    } else {
      ++oom;
      EXPECT(srv == nullptr);
    }
    evals(p, 1);  // the problem still evaluates on its own stream
    EXPECT(Live::now() == before);
  }
  pcv_server* srv = nullptr;
  for (size_t b : {(size_t)1, (size_t)1024, (size_t)7000, (size_t)3 * 64 * 40})
    EXPECT(pcv_server_create(&srv, p, b, 4) == PCV_ERR_INVALID);  // below one kriging item per slot
  EXPECT(pcv_server_create(&srv, p, (size_t)1 << 50, 4) == PCV_ERR_OOM);
  evals(p, 1);
  EXPECT(Live::now() == before);
  CHECK(pcv_server_create(&srv, p, (size_t)64 << 20, 4));
  std::vector<double> q = {0.3, 0.4, 0.7, 0.2}, out(4);
  pcv_ticket tk;
  CHECK(pcv_server_submit_predict(srv, 2, q.data(), out.data(), out.data() + 2, 0, &tk));
  CHECK(pcv_server_wait(srv, tk, -1.0));
  CHECK(pcv_server_destroy(srv));
  CHECK(pcv_problem_destroy(p));
  EXPECT(Live::now() == base);
  std::printf("oom_server: %d created, %d out of memory\n", ok, oom);
}

// The tuner's cycle on three problems in one process (tune, reuse of the
// cache on an identical problem, a new problem shape), with evaluations,
// batches and a server between, then tuning of a problem whose configuration
// changed under a server (refused) and after it.
void tune(const Data& d, const char* cache) {
  const Live base = Live::now();
  std::remove(cache);
  const Data d2 = make_data(290, 5);  // another shape
  pcv_theta t = th(0.3, 0.1);
  for (int k = 0; k < 3; ++k) {
    const Data& dk = k < 2 ? d : d2;
    for (int prec : {PCV_PREC_MIXED, PCV_PREC_FP64}) {
      pcv_options o;
      pcv_default_options(&o);
      o.prec = prec;
      pcv_problem* p = create(dk, o);
      evals(p, 1);
      pcv_tune_report r;
      CHECK(pcv_autotune(p, &t, cache, 2, &r));
      std::printf("tune problem %d prec %d: small_npad %d max_wg %d two_groups %d from_cache %d timed %d\n", k,
                  prec, r.small_npad, r.max_wg_per_subset, r.two_groups, r.from_cache, r.n_timed);
      EXPECT(r.from_cache == (k == 1 ? 1 : 0));
      EXPECT(r.from_cache || r.n_timed >= 2);
      evals(p, 2);
      std::vector<pcv_theta> ths(5, t);
      std::vector<double> losses(5);
      CHECK(pcv_eval_batch(p, 5, ths.data(), losses.data()));
      CHECK(pcv_factor(p, &t));
      pcv_server* srv = nullptr;
      CHECK(pcv_server_create(&srv, p, (size_t)64 << 20, 4));
      EXPECT(pcv_autotune(p, &t, cache, 2, &r) == PCV_ERR_STATE);
      double l = 0;
      pcv_ticket tk;
      CHECK(pcv_server_submit_eval(srv, &t, &l, &tk));
      CHECK(pcv_server_wait(srv, tk, -1.0));
      CHECK(pcv_server_destroy(srv));
      CHECK(pcv_autotune(p, &t, nullptr, 1, &r));  // again, no cache
      evals(p, 2);
      CHECK(pcv_problem_destroy(p));
    }
  }
  EXPECT(Live::now() == base);
}

// Tuning of a problem whose first evaluation happens inside the tuner,
// after a factorisation and a server that held it (and was refused tuning).
void tune_after_serving(const Data& d) {
  const Live base = Live::now();
  const pcv_theta t = th(0.4, 0.1);
  for (int rep = 0; rep < 3; ++rep) {
    pcv_options o;
    pcv_default_options(&o);
    pcv_problem* p = create(d, o);
    CHECK(pcv_factor(p, &t));
    pcv_server* srv = nullptr;
    CHECK(pcv_server_create(&srv, p, 0, 64));
    pcv_tune_report r;
    EXPECT(pcv_autotune(p, &t, nullptr, 3, &r) == PCV_ERR_STATE);
    CHECK(pcv_server_destroy(srv));
    CHECK(pcv_autotune(p, &t, nullptr, 1, &r));
    std::printf("tune after serving: small_npad %d max_wg %d two_groups %d timed %d\n", r.small_npad,
                r.max_wg_per_subset, r.two_groups, r.n_timed);
    evals(p, 1);
    CHECK(pcv_problem_destroy(p));
  }
  EXPECT(Live::now() == base);
}

// Tuning with a device or pinned allocation failing at each point in turn,
// on a problem whose first evaluation happens inside the tuner and on one
// evaluated and factored before: the tuner returns OK or the failure, the
// problem keeps evaluating, and nothing is left behind.
void oom_tune(const Data& d) {
  const Live base = Live::now();
  const pcv_theta t = th(0.4, 0.1);
  int ok = 0, failed = 0;
  for (int pre = 0; pre < 2; ++pre)
    for (int64_t k = 0; k < 40; ++k) {
      pcv_options o;
      pcv_default_options(&o);
      pcv_problem* p = create(d, o);
      if (pre) {
        evals(p, 1);
        CHECK(pcv_factor(p, &t));
      }
      pcv_tune_report r;
      stub_fail_malloc_after(k);
      const pcv_status s = pcv_autotune(p, &t, nullptr, 1, &r);
      stub_fail_malloc_after(-1);
      EXPECT(s == PCV_OK || s == PCV_ERR_OOM);
      if (s == PCV_OK) ++ok; else ++failed;
      evals(p, 2);
      CHECK(pcv_problem_destroy(p));
    }
  EXPECT(Live::now() == base);
  std::printf("oom_tune: %d tuned, %d out of memory\n", ok, failed);
}

// A kernel launch failing at each point in turn: of an evaluation (graph
// capture and the fallback paths included), of a multi-theta call, of a
// factorisation with a prediction, and of a server's kriging batches and
// evaluations.  The call reports PCV_ERR_DEVICE (or OK when it launched
// fewer kernels), nothing is left behind, and the next calls give the same
// results as before the failure.
void launch_fail(const Data& d) {
  const Live base = Live::now();
  const pcv_theta t = th(0.3, 0.1);
  std::vector<pcv_theta> ths;
  for (int k = 0; k < 5; ++k) ths.push_back(th(0.25 + 0.02 * k, 0.08));
  std::vector<double> q = {0.3, 0.4, 0.7, 0.2, 0.1, 0.9};
  int ok = 0, failed = 0;
  for (int mode = 0; mode < 4; ++mode)
    for (int64_t k = 0; k < 40; ++k) {
      pcv_options o;
      pcv_default_options(&o);
      o.est_error = k & 1;
      pcv_problem* p = create(d, o);
      double ref = 0, l = 0;
      std::vector<double> refb(ths.size()), lb(ths.size());
      std::vector<double> m0(3), v0(3), m1(3), v1(3);
      // every other round the failing call is the problem's first, so that
      // the failure can hit the graph captures and the first allocations
      const bool first = (k & 2) && mode < 2;
      if (!first) {
        CHECK(pcv_eval(p, &t, &ref, nullptr));
        CHECK(pcv_eval_batch(p, (int32_t)ths.size(), ths.data(), refb.data()));
        CHECK(pcv_factor(p, &t));
        CHECK(pcv_predict(p, 3, q.data(), m0.data(), v0.data(), 0, nullptr));
      }
      pcv_status s = PCV_OK;
      stub_fail_launch_after(k);
      if (mode == 0) {
        s = pcv_eval(p, &t, &l, nullptr);
      } else if (mode == 1) {
        s = pcv_eval_batch(p, (int32_t)ths.size(), ths.data(), lb.data());
      } else if (mode == 2) {
        s = pcv_factor(p, &t);
        if (s == PCV_OK) s = pcv_predict(p, 3, q.data(), m1.data(), v1.data(), 0, nullptr);
      } else {
        pcv_server* srv = nullptr;
        s = pcv_server_create(&srv, p, (size_t)64 << 20, 8);
        if (s == PCV_OK) {
          pcv_ticket a, b;
          const pcv_status sa = pcv_server_submit_predict(srv, 3, q.data(), m1.data(), v1.data(), 0, &a);
          const pcv_status sb = pcv_server_submit_eval(srv, &t, &l, &b);
          pcv_status wa = sa == PCV_OK ? pcv_server_wait(srv, a, -1.0) : sa;
          pcv_status wb = sb == PCV_OK ? pcv_server_wait(srv, b, -1.0) : sb;
          EXPECT(wa == PCV_OK || wa == PCV_ERR_DEVICE);
          EXPECT(wb == PCV_OK || wb == PCV_ERR_DEVICE);
          s = wa != PCV_OK ? wa : wb;
          stub_fail_launch_after(-1);
          // the server keeps serving after a failed batch or evaluation
          CHECK(pcv_server_submit_predict(srv, 3, q.data(), m1.data(), v1.data(), 0, &a));
          CHECK(pcv_server_wait(srv, a, -1.0));
          for (int i = 0; i < 3; ++i) EXPECT(m1[i] == m0[i] && v1[i] == v0[i]);
          CHECK(pcv_server_destroy(srv));
        }
      }
      stub_fail_launch_after(-1);
      EXPECT(s == PCV_OK || s == PCV_ERR_DEVICE);
      if (s == PCV_OK) ++ok; else ++failed;
      if (first) {
        CHECK(pcv_eval(p, &t, &ref, nullptr));
        CHECK(pcv_eval_batch(p, (int32_t)ths.size(), ths.data(), refb.data()));
        CHECK(pcv_factor(p, &t));
        CHECK(pcv_predict(p, 3, q.data(), m0.data(), v0.data(), 0, nullptr));
      }
      // the problem is usable and gives the same results
      CHECK(pcv_eval(p, &t, &l, nullptr));
      EXPECT(l == ref);
      CHECK(pcv_eval_batch(p, (int32_t)ths.size(), ths.data(), lb.data()));
      for (size_t i = 0; i < ths.size(); ++i) EXPECT(lb[i] == refb[i]);
      CHECK(pcv_factor(p, &t));
      CHECK(pcv_predict(p, 3, q.data(), m1.data(), v1.data(), 0, nullptr));
      for (int i = 0; i < 3; ++i) EXPECT(m1[i] == m0[i] && v1[i] == v0[i]);
      CHECK(pcv_problem_destroy(p));
    }
  EXPECT(Live::now() == base);
  std::printf("launch_fail: %d completed, %d failed\n", ok, failed);
}

int main(int argc, char** argv) {
  const std::string sc = argc > 1 ? argv[1] : "sequence";
  const Data d = make_data(300, 1);
  if (sc == "sequence") {
    for (int rep = 0; rep < 3; ++rep) sequence(d, rep);
    stub_report("sequence");
  } else if (sc == "oom") {
    oom(d);
    oom_batch(make_data(40, 3));
    oom_server(make_data(40, 4));
    oom_tune(make_data(120, 6));
    launch_fail(make_data(60, 7));
  } else if (sc == "tune_after_serving") {
    tune_after_serving(make_data(290, 2));
    stub_report("tune_after_serving");
  } else if (sc == "tune") {
    tune(d, argc > 2 ? argv[2] : "pcv_tune_cache.txt");
    stub_report("tune");
  } else {
    std::fprintf(stderr, "unknown scenario %s\n", sc.c_str());
    return 2;
  }
  std::printf("ok %s\n", sc.c_str());
  return 0;
}
