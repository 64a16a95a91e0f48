// CPU stand-in for the HIP runtime and for the library's kernel launchers,
// so that the library's host code (problem residency, evaluation schedules,
// graph capture and replay, batched evaluations, prediction, serving and
// tuning) can run its call sequences on the CPU under AddressSanitizer and
// UndefinedBehaviorSanitizer.  Test infrastructure only.
//
// What it checks, beyond what the sanitizers see:
//   * every stream, event, graph and executable graph is live when used
//     (a destroyed handle used again stops the process with a message);
//   * every device pointer a copy, fill or kernel launch touches lies in a
//     live device allocation, checked when the work runs, so a captured
//     graph replayed after its buffers were freed is caught;
//   * calls that the capture mode forbids (synchronisation, allocation,
//     synchronous copies) are not made by a thread while it captures;
//   * at the end, no device allocation, pinned buffer, stream or event is
//     left alive (stub_report()).
// Work runs when it is enqueued (streams are trivially ordered); while a
// stream captures, its work is recorded and runs at each graph launch.
// Kernels do no arithmetic: the buffers keep whatever they held (device
// allocations start zeroed), which the host code reads as "no subset failed".
#include <hip/hip_runtime_api.h>

#include <chrono>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <random>
#include <set>
#include <thread>
#include <vector>

#include "../../paper_1912_13132_amd/csrc/pcv_host.h"

struct Capture;
struct ihipStream_t {
  bool alive = true;
  Capture* cap = nullptr;
};
struct ihipEvent_t {
  bool alive = true;
  Capture* cap = nullptr;
};
struct ihipGraph {
  bool alive = true;
  std::vector<std::function<void()>> ops;
};
struct hipGraphExec {
  bool alive = true;
  std::vector<std::function<void()>> ops;
};
struct Capture {
  hipStream_t origin = nullptr;
  ihipGraph* graph = nullptr;
  std::set<hipStream_t> members;
};

namespace {

// The registries are never destroyed (no static destructors run before the
// leak check at exit), so destroyed handles kept in g_dead stay reachable.
std::recursive_mutex& g_mu = *new std::recursive_mutex;
// Failure injection: with g_fail_after >= 0, that many more hipMalloc calls
// succeed and the next ones report hipErrorOutOfMemory until it is reset.
int64_t g_fail_after = -1;
// The runtime's per-thread last error: a failed call sets it, hipGetLastError
// returns and clears it (the launch wrappers return it after each launch).
thread_local hipError_t g_last_error = hipSuccess;
// Launch failure injection: with g_fail_launch_after >= 0, that many more
// kernel launches succeed and the next one fails (hipErrorLaunchFailure as
// the launch's error; the kernel does not run).
int64_t g_fail_launch_after = -1;
constexpr size_t kStubMaxAlloc = (size_t)1 << 40;
struct Alloc {
  size_t size;
  bool pinned;
};
std::map<uintptr_t, Alloc>& g_live = *new std::map<uintptr_t, Alloc>;  // base -> allocation
// destroyed handles stay allocated (reachable) so a later use is detected
std::vector<void*>& g_dead = *new std::vector<void*>;
std::set<hipStream_t>& g_streams = *new std::set<hipStream_t>;
std::set<hipEvent_t>& g_events = *new std::set<hipEvent_t>;
thread_local int t_capturing = 0;
int64_t g_launches = 0, g_graph_launches = 0, g_captures = 0;

[[noreturn]] void die(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  std::fprintf(stderr, "hip-stub: ");
  std::vfprintf(stderr, fmt, ap);
  std::fprintf(stderr, "\n");
  va_end(ap);
  std::fflush(stderr);
  std::abort();
}

const Alloc* find(const void* p, uintptr_t* base) {
  const uintptr_t a = (uintptr_t)p;
  auto it = g_live.upper_bound(a);
  if (it == g_live.begin()) return nullptr;
  --it;
  if (a >= it->first + it->second.size && !(a == it->first && it->second.size == 0)) return nullptr;
  if (base) *base = it->first;
  return &it->second;
}

// [p, p + bytes) inside one live device allocation
void dev_range(const void* p, size_t bytes, const char* what) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  uintptr_t base = 0;
  const Alloc* a = find(p, &base);
  if (!a || a->pinned) die("%s: %p is not in a live device allocation", what, p);
  if ((uintptr_t)p + bytes > base + a->size)
    die("%s: %zu bytes at %p run past the end of their allocation (%zu bytes at %p)", what, bytes, p, a->size,
        (void*)base);
}
void dev_ptr(const void* p, const char* what) {
  if (p) dev_range(p, 1, what);
}
// host side of a copy: pinned buffers are range-checked, pageable memory is not ours to check
void host_range(const void* p, size_t bytes, const char* what) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  uintptr_t base = 0;
  const Alloc* a = find(p, &base);
  if (a && a->pinned && (uintptr_t)p + bytes > base + a->size)
    die("%s: %zu bytes at %p run past the end of a pinned buffer", what, bytes, p);
  if (a && !a->pinned) die("%s: %p is device memory, expected host memory", what, p);
}

void live_stream(hipStream_t s, const char* what) {
  if (!s) return;
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  if (!g_streams.count(s)) die("%s: stream %p is not live", what, (void*)s);
}
void live_event(hipEvent_t e, const char* what) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  if (!e || !g_events.count(e)) die("%s: event %p is not live", what, (void*)e);
}
void no_capture(const char* what) {
  if (t_capturing) die("%s called by a thread that is capturing a graph", what);
}

// run now, or record into the capture the stream belongs to
void enqueue(hipStream_t s, const char* what, std::function<void()> op) {
  live_stream(s, what);
  {
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    if (s && s->cap) {
      s->cap->graph->ops.push_back(std::move(op));
      return;
    }
  }
  op();
}

}  // namespace

extern "C" {

void stub_fail_malloc_after(int64_t n) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  g_fail_after = n;
}
void stub_fail_launch_after(int64_t n) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  g_fail_launch_after = n;
}

int64_t stub_live_allocations() {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  int64_t n = 0;
  for (auto& kv : g_live)
    if (!kv.second.pinned) ++n;
  return n;
}
int64_t stub_live_pinned() {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  int64_t n = 0;
  for (auto& kv : g_live)
    if (kv.second.pinned) ++n;
  return n;
}
int64_t stub_live_streams() {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  return (int64_t)g_streams.size();
}
int64_t stub_live_events() {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  return (int64_t)g_events.size();
}
void stub_report(const char* tag) {
  std::printf("[stub] %s: live device allocations %lld, pinned %lld, streams %lld, events %lld; "
              "launches %lld, captures %lld, graph launches %lld\n",
              tag, (long long)stub_live_allocations(), (long long)stub_live_pinned(),
              (long long)stub_live_streams(), (long long)stub_live_events(), (long long)g_launches,
              (long long)g_captures, (long long)g_graph_launches);
  std::fflush(stdout);
}

hipError_t hipMalloc(void** ptr, size_t size) {
  no_capture("hipMalloc");
  if (size > kStubMaxAlloc) {  // more than any device or host holds
    *ptr = nullptr;
    return g_last_error = hipErrorOutOfMemory;
  }
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  if (g_fail_after == 0) {
    *ptr = nullptr;
    return g_last_error = hipErrorOutOfMemory;
  }
  if (g_fail_after > 0) --g_fail_after;
  void* p = std::calloc(size ? size : 1, 1);
  if (!p) return hipErrorOutOfMemory;
  g_live[(uintptr_t)p] = Alloc{size, false};
  *ptr = p;
  return hipSuccess;
}
hipError_t hipFree(void* ptr) {
  no_capture("hipFree");
  if (!ptr) return hipSuccess;
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  auto it = g_live.find((uintptr_t)ptr);
  if (it == g_live.end() || it->second.pinned) die("hipFree(%p): not a live device allocation", ptr);
  g_live.erase(it);
  std::free(ptr);
  return hipSuccess;
}
hipError_t hipHostMalloc(void** ptr, size_t size, unsigned int) {
  no_capture("hipHostMalloc");
  if (size > kStubMaxAlloc) {  // more than any device or host holds
    *ptr = nullptr;
    return g_last_error = hipErrorOutOfMemory;
  }
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  if (g_fail_after == 0) {
    *ptr = nullptr;
    return g_last_error = hipErrorOutOfMemory;
  }
  if (g_fail_after > 0) --g_fail_after;
  void* p = std::calloc(size ? size : 1, 1);
  if (!p) return hipErrorOutOfMemory;
  g_live[(uintptr_t)p] = Alloc{size, true};
  *ptr = p;
  return hipSuccess;
}
hipError_t hipHostFree(void* ptr) {
  no_capture("hipHostFree");
  if (!ptr) return hipSuccess;
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  auto it = g_live.find((uintptr_t)ptr);
  if (it == g_live.end() || !it->second.pinned) die("hipHostFree(%p): not a live pinned buffer", ptr);
  g_live.erase(it);
  std::free(ptr);
  return hipSuccess;
}

static void copy_checked(void* dst, const void* src, size_t n, hipMemcpyKind kind, const char* what) {
  if (n == 0) return;
  switch (kind) {
    case hipMemcpyHostToDevice:
      dev_range(dst, n, what);
      host_range(src, n, what);
      break;
    case hipMemcpyDeviceToHost:
      dev_range(src, n, what);
      host_range(dst, n, what);
      break;
    case hipMemcpyDeviceToDevice:
      dev_range(src, n, what);
      dev_range(dst, n, what);
      break;
    default:
      die("%s: unsupported copy kind %d", what, (int)kind);
  }
  std::memmove(dst, src, n);
}
hipError_t hipMemcpy(void* dst, const void* src, size_t n, hipMemcpyKind kind) {
  no_capture("hipMemcpy");
  copy_checked(dst, src, n, kind, "hipMemcpy");
  return hipSuccess;
}
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t n, hipMemcpyKind kind, hipStream_t s) {
  enqueue(s, "hipMemcpyAsync", [=] { copy_checked(dst, src, n, kind, "hipMemcpyAsync"); });
  return hipSuccess;
}
hipError_t hipMemset(void* dst, int v, size_t n) {
  no_capture("hipMemset");
  if (n) dev_range(dst, n, "hipMemset");
  std::memset(dst, v, n);
  return hipSuccess;
}
hipError_t hipMemsetAsync(void* dst, int v, size_t n, hipStream_t s) {
  enqueue(s, "hipMemsetAsync", [=] {
    if (n) dev_range(dst, n, "hipMemsetAsync");
    std::memset(dst, v, n);
  });
  return hipSuccess;
}

hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned int) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  *s = new ihipStream_t();
  g_streams.insert(*s);
  return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  if (!s || !g_streams.count(s)) die("hipStreamDestroy(%p): not a live stream", (void*)s);
  if (s->cap) die("hipStreamDestroy(%p) while it captures", (void*)s);
  g_streams.erase(s);
  s->alive = false;
  g_dead.push_back(s);
  return hipSuccess;
}
// With STUB_JITTER=<seed> set, every stream synchronisation takes a random
// 0..300 microseconds, so that timing-driven choices (the tuner's) follow
// different paths from run to run.
static void jitter() {
  static const char* env = std::getenv("STUB_JITTER");
  if (!env) return;
  static std::mt19937_64 rng(std::strtoull(env, nullptr, 10));
  static std::mutex mu;
  int us;
  {
    std::lock_guard<std::mutex> lk(mu);
    us = (int)(rng() % 300);
  }
  std::this_thread::sleep_for(std::chrono::microseconds(us));
}
hipError_t hipStreamSynchronize(hipStream_t s) {
  live_stream(s, "hipStreamSynchronize");
  no_capture("hipStreamSynchronize");
  if (s && s->cap) die("hipStreamSynchronize on a capturing stream");
  jitter();
  return hipSuccess;
}
hipError_t hipDeviceSynchronize(void) {
  no_capture("hipDeviceSynchronize");
  return hipSuccess;
}
hipError_t hipEventCreate(hipEvent_t* e) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  *e = new ihipEvent_t();
  g_events.insert(*e);
  return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { return hipEventCreate(e); }
hipError_t hipEventDestroy(hipEvent_t e) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  if (!e || !g_events.count(e)) die("hipEventDestroy(%p): not a live event", (void*)e);
  g_events.erase(e);
  e->alive = false;
  g_dead.push_back(e);
  return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s) {
  live_event(e, "hipEventRecord");
  live_stream(s, "hipEventRecord");
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  e->cap = s ? s->cap : nullptr;
  return hipSuccess;
}
hipError_t hipEventSynchronize(hipEvent_t e) {
  live_event(e, "hipEventSynchronize");
  no_capture("hipEventSynchronize");
  return hipSuccess;
}
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b) {
  live_event(a, "hipEventElapsedTime");
  live_event(b, "hipEventElapsedTime");
  *ms = 1.0f;
  return hipSuccess;
}
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned int) {
  live_stream(s, "hipStreamWaitEvent");
  live_event(e, "hipStreamWaitEvent");
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  if (e->cap && s) {
    if (s->cap && s->cap != e->cap) die("hipStreamWaitEvent joins two captures");
    s->cap = e->cap;  // the stream joins the capture (fork)
    e->cap->members.insert(s);
  } else if (s && s->cap && !e->cap) {
    die("a capturing stream waits for an event recorded outside the capture");
  }
  return hipSuccess;
}
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode) {
  live_stream(s, "hipStreamBeginCapture");
  if (!s) die("hipStreamBeginCapture on the null stream");
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  if (s->cap) die("hipStreamBeginCapture: stream already captures");
  Capture* c = new Capture();
  c->origin = s;
  c->graph = new ihipGraph();
  c->members.insert(s);
  s->cap = c;
  ++t_capturing;
  ++g_captures;
  return hipSuccess;
}
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t* g) {
  live_stream(s, "hipStreamEndCapture");
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  if (!s || !s->cap || s->cap->origin != s) die("hipStreamEndCapture on a stream that did not begin one");
  Capture* c = s->cap;
  for (hipStream_t m : c->members) m->cap = nullptr;
  *g = c->graph;
  g_dead.push_back(c);
  --t_capturing;
  return hipSuccess;
}
hipError_t hipGraphInstantiate(hipGraphExec_t* x, hipGraph_t g, hipGraphNode_t*, char*, size_t) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  if (!g || !g->alive) die("hipGraphInstantiate: graph not live");
  hipGraphExec* e = new hipGraphExec();
  e->ops = g->ops;
  *x = e;
  return hipSuccess;
}
hipError_t hipGraphDestroy(hipGraph_t g) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  if (!g || !g->alive) die("hipGraphDestroy: graph not live");
  g->alive = false;
  g->ops.clear();
  g_dead.push_back(g);
  return hipSuccess;
}
hipError_t hipGraphExecDestroy(hipGraphExec_t x) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  if (!x || !x->alive) die("hipGraphExecDestroy: executable graph not live");
  x->alive = false;
  x->ops.clear();
  g_dead.push_back(x);
  return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t x, hipStream_t s) {
  std::vector<std::function<void()>> ops;
  {
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    if (!x || !x->alive) die("hipGraphLaunch: executable graph not live");
    ops = x->ops;
    ++g_graph_launches;
  }
  enqueue(s, "hipGraphLaunch", [ops] {
    for (auto& op : ops) op();
  });
  return hipSuccess;
}

hipError_t hipGetDevice(int* d) {
  *d = 0;
  return hipSuccess;
}
hipError_t hipSetDevice(int d) { return d == 0 ? hipSuccess : hipErrorInvalidDevice; }
hipError_t hipDeviceGetAttribute(int* v, hipDeviceAttribute_t a, int) {
  *v = a == hipDeviceAttributeMultiprocessorCount ? 256 : 0;
  return hipSuccess;
}
hipError_t hipGetDeviceProperties(hipDeviceProp_t* prop, int d) {
  if (d != 0) return hipErrorInvalidDevice;
  std::memset(prop, 0, sizeof(*prop));
  std::strcpy(prop->gcnArchName, "stub");
  prop->multiProcessorCount = 256;
  return hipSuccess;
}
hipError_t hipRuntimeGetVersion(int* v) {
  *v = 1;
  return hipSuccess;
}
hipError_t hipGetLastError(void) {
  const hipError_t e = g_last_error;
  g_last_error = hipSuccess;
  return e;
}
const char* hipGetErrorString(hipError_t e) { return e == hipSuccess ? "hipSuccess" : "hip-stub error"; }
hipError_t hipPointerGetAttributes(hipPointerAttribute_t* a, const void* p) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  const Alloc* al = find(p, nullptr);
  if (!al) return hipErrorInvalidValue;
  std::memset(a, 0, sizeof(*a));
  a->type = al->pinned ? hipMemoryTypeHost : hipMemoryTypeDevice;
  a->device = 0;
  a->devicePointer = const_cast<void*>(p);
  return hipSuccess;
}
hipError_t hipMemGetAddressRange(hipDeviceptr_t* base, size_t* size, hipDeviceptr_t p) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  uintptr_t b = 0;
  const Alloc* al = find(p, &b);
  if (!al) return hipErrorInvalidValue;
  *base = (hipDeviceptr_t)b;
  *size = al->size;
  return hipSuccess;
}

}  // extern "C"

// ---- the library's kernel launchers: argument checks, no arithmetic
namespace pcv {

static void launched(const char* what, std::function<void()> chk, hipStream_t s) {
  {
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    if (g_fail_launch_after == 0) {
      g_last_error = hipErrorLaunchFailure;
      return;
    }
    if (g_fail_launch_after > 0) --g_fail_launch_after;
    ++g_launches;
  }
  chk();  // arguments valid when the launch is enqueued
  enqueue(s, what, chk);  // and when it runs (graph replays)
}

static void potrf_checks(const Launch& L, const int32_t* order, int n, const void* cx, const void* cy,
                         const void* cv, double* zout, const void* Lb, double* Inv, double* logdet,
                         int32_t* status, const CoopPlan& c) {
  dev_ptr(L.desc, "potrf desc"); dev_ptr(L.theta, "potrf theta"); dev_range(order, 4 * (size_t)n, "potrf order");
  dev_ptr(cx, "potrf cx"); dev_ptr(cy, "potrf cy"); dev_ptr(cv, "potrf cv"); dev_ptr(zout, "potrf z");
  dev_ptr(Lb, "potrf L"); dev_ptr(Inv, "potrf Inv");
  dev_ptr(logdet, "potrf logdet"); dev_ptr(status, "potrf status");
  if (c.n_blocks > 0) {
    dev_range(c.info, 4 * (size_t)c.n_blocks, "potrf coop info");
    dev_range(c.sync, 16 * (size_t)c.n_slots, "potrf coop sync");
    if (cv) dev_range(c.subsets, 4 * (size_t)c.n_subsets, "potrf coop subsets");
  }
}
hipError_t launch_potrf_f32(const Launch& L, const int32_t* order, int n, int, const float* cx, const float* cy,
                            const float* cv, double* zout, float* Lb, double* Inv, double* logdet, int32_t* status,
                            const CoopPlan* cp, int, int) {
  if (cv && !zout) return hipErrorInvalidValue;
  if (n <= 0) return hipSuccess;
  const CoopPlan c = cp ? *cp : CoopPlan{};
  if (cv && c.n_blocks > 0 && (!c.subsets || c.n_subsets <= 0)) return hipErrorInvalidValue;
  launched("potrf_f32", [=] { potrf_checks(L, order, n, cx, cy, cv, zout, Lb, Inv, logdet, status, c); },
           L.stream);
  return hipGetLastError();  // like the launch wrappers: a pending error surfaces here
}
hipError_t launch_potrf_f64(const Launch& L, const int32_t* order, int n, const double* cx, const double* cy,
                            const double* cv, double* zout, double* Lb, double* Inv, double* logdet,
                            int32_t* status, const CoopPlan* cp) {
  if (cv && !zout) return hipErrorInvalidValue;
  if (n <= 0) return hipSuccess;
  const CoopPlan c = cp ? *cp : CoopPlan{};
  if (cv && c.n_blocks > 0 && (!c.subsets || c.n_subsets <= 0)) return hipErrorInvalidValue;
  launched("potrf_f64", [=] { potrf_checks(L, order, n, cx, cy, cv, zout, Lb, Inv, logdet, status, c); },
           L.stream);
  return hipGetLastError();  // like the launch wrappers: a pending error surfaces here
}
template <typename T>
static hipError_t trsv(const char* what, const Launch& L, const int32_t* order, int n, const T* Lb,
                       const double* Inv, const void* a, const void* b, const void* c, const void* d,
                       const int32_t* gate) {
  if (n <= 0) return hipSuccess;
  launched(what, [=] {
    dev_ptr(L.desc, what); dev_ptr(L.theta, what); dev_range(order, 4 * (size_t)n, what);
    dev_ptr(Lb, what); dev_ptr(Inv, what); dev_ptr(a, what); dev_ptr(b, what); dev_ptr(c, what); dev_ptr(d, what);
    dev_ptr(gate, what);
  }, L.stream);
  return hipGetLastError();  // like the launch wrappers: a pending error surfaces here
}
hipError_t launch_trsv_fwd_f32(const Launch& L, const int32_t* o, int n, int, const float* Lb, const double* Inv,
                               const double* rt, const double* rp, double* z, double* r2, const int32_t* g) {
  return trsv("trsv_fwd_f32", L, o, n, Lb, Inv, rt, rp, z, r2, g);
}
hipError_t launch_trsv_fwd_f64(const Launch& L, const int32_t* o, int n, int, const double* Lb, const double* Inv,
                               const double* rt, const double* rp, double* z, double* r2, const int32_t* g) {
  return trsv("trsv_fwd_f64", L, o, n, Lb, Inv, rt, rp, z, r2, g);
}
hipError_t launch_trsv_bwd_f32(const Launch& L, const int32_t* o, int n, int, const float* Lb, const double* Inv,
                               const double* z, double* x, double* acc, const int32_t* g) {
  return trsv("trsv_bwd_f32", L, o, n, Lb, Inv, z, x, acc, nullptr, g);
}
hipError_t launch_trsv_bwd_f64(const Launch& L, const int32_t* o, int n, int, const double* Lb, const double* Inv,
                               const double* z, double* x, double* acc, const int32_t* g) {
  return trsv("trsv_bwd_f64", L, o, n, Lb, Inv, z, x, acc, nullptr, g);
}
hipError_t launch_residual(const Launch& L, const int2* ti, int nt, const int2* ri, int nr, const double* tx,
                           const double* ty, const double* yT, const double* alpha, double* rrow, double* pcol,
                           double* r, const int32_t* gate) {
  if (nt <= 0 && nr <= 0) return hipSuccess;
  launched("residual", [=] {
    if (nt > 0) dev_range(ti, 8 * (size_t)nt, "residual tile items");
    if (nr > 0) dev_range(ri, 8 * (size_t)nr, "residual row items");
    for (const void* p : {(const void*)tx, (const void*)ty, (const void*)yT, (const void*)alpha, (const void*)rrow,
                          (const void*)pcol, (const void*)r, (const void*)gate})
      dev_ptr(p, "residual");
  }, L.stream);
  return hipGetLastError();  // like the launch wrappers: a pending error surfaces here
}
hipError_t launch_refine_gate(hipStream_t s, int n, const int32_t* order, int, int, const double* rhs2,
                              const double* ynorm2, double, int32_t* gate, int32_t* nsweep) {
  if (n <= 0) return hipSuccess;
  launched("refine_gate", [=] {
    dev_range(order, 4 * (size_t)n, "refine_gate order");
    for (const void* p : {(const void*)rhs2, (const void*)ynorm2, (const void*)gate, (const void*)nsweep})
      dev_ptr(p, "refine_gate");
  }, s);
  return hipGetLastError();  // like the launch wrappers: a pending error surfaces here
}
hipError_t launch_predict_val(const Launch& L, const int2* items, int n, const double* tx, const double* ty,
                              const double* vx, const double* vy, const double* yV, const double* alpha,
                              double* yhat, double* err) {
  if (n <= 0) return hipSuccess;
  launched("predict_val", [=] {
    dev_range(items, 8 * (size_t)n, "predict_val items");
    for (const void* p : {(const void*)tx, (const void*)ty, (const void*)vx, (const void*)vy, (const void*)yV,
                          (const void*)alpha, (const void*)yhat, (const void*)err})
      dev_ptr(p, "predict_val");
  }, L.stream);
  return hipGetLastError();  // like the launch wrappers: a pending error surfaces here
}
hipError_t launch_krige(hipStream_t s, const SubsetDesc* desc, const ThetaDev* theta, const KrigeItem* items,
                        int n, const double* tx, const double* ty, const double* L64, const double* Inv,
                        const double* alpha, const double* qx, const double* qy, const int32_t* qorig,
                        const int32_t* qflag, double* W, double* mean, double* var) {
  if (n <= 0) return hipSuccess;
  launched("krige", [=] {
    dev_range(items, sizeof(KrigeItem) * (size_t)n, "krige items");
    for (const void* p : {(const void*)desc, (const void*)theta, (const void*)tx, (const void*)ty,
                          (const void*)L64, (const void*)Inv, (const void*)alpha, (const void*)qx,
                          (const void*)qy, (const void*)qorig, (const void*)qflag, (const void*)W,
                          (const void*)mean, (const void*)var})
      dev_ptr(p, "krige");
  }, s);
  return hipGetLastError();  // like the launch wrappers: a pending error surfaces here
}
hipError_t launch_gls(hipStream_t s, const SubsetDesc* desc, const int32_t* order, int n, int, int64_t,
                      const double* Xp, const double* Wp, const double* alpha, double* beta, int32_t* status) {
  if (n <= 0) return hipSuccess;
  launched("gls", [=] {
    dev_range(order, 4 * (size_t)n, "gls order");
    for (const void* p : {(const void*)desc, (const void*)Xp, (const void*)Wp, (const void*)alpha,
                          (const void*)beta, (const void*)status})
      dev_ptr(p, "gls");
  }, s);
  return hipGetLastError();  // like the launch wrappers: a pending error surfaces here
}
hipError_t launch_quad(hipStream_t s, const SubsetDesc* desc, const int32_t* order, int n, const double* yT,
                       const double* alpha, double* quad) {
  if (n <= 0) return hipSuccess;
  launched("quad", [=] {
    dev_range(order, 4 * (size_t)n, "quad order");
    dev_ptr(desc, "quad"); dev_ptr(yT, "quad"); dev_ptr(alpha, "quad"); dev_ptr(quad, "quad");
  }, s);
  return hipGetLastError();  // like the launch wrappers: a pending error surfaces here
}
hipError_t launch_reduce(hipStream_t s, const SubsetDesc* desc, int S, int n_theta, const double* err,
                         int32_t* status, const int32_t* active, const double* rhs2, const double* ynorm2, double,
                         double* sspe, double* total, int32_t* nbad) {
  launched("reduce", [=] {
    dev_range(desc, sizeof(SubsetDesc) * (size_t)S * n_theta, "reduce desc");
    dev_range(status, 4 * (size_t)S * n_theta, "reduce status");
    dev_range(active, 4 * (size_t)S, "reduce active");
    dev_range(sspe, 8 * (size_t)S * n_theta, "reduce sspe");
    dev_range(total, 8 * (size_t)n_theta, "reduce total");
    dev_range(nbad, 4 * (size_t)n_theta, "reduce nbad");
    dev_ptr(err, "reduce err"); dev_ptr(rhs2, "reduce rhs2"); dev_ptr(ynorm2, "reduce ynorm2");
  }, s);
  return hipGetLastError();  // like the launch wrappers: a pending error surfaces here
}
hipError_t launch_math_check(hipStream_t s, int64_t n, const double* t, const double* x, double* e, double* r) {
  if (n <= 0) return hipSuccess;
  launched("math_check", [=] {
    dev_range(t, 8 * (size_t)n, "math t"); dev_range(x, 8 * (size_t)n, "math x");
    dev_range(e, 8 * (size_t)n, "math e"); dev_range(r, 8 * (size_t)n, "math r");
  }, s);
  return hipGetLastError();  // like the launch wrappers: a pending error surfaces here
}

// the device division and the fixed-array prediction need device code
pcv_status part_divide(int64_t, const double*, const double*, int32_t, double, double*) {
  return fail(PCV_ERR_DEVICE, "device division is not part of the CPU harness");
}
pcv_status part_subsets(int64_t, const double*, int32_t, const double*, double, const uint8_t*, int32_t*, int64_t*,
                        int64_t*, int32_t*, int64_t*, int32_t*) {
  return fail(PCV_ERR_DEVICE, "device division is not part of the CPU harness");
}
pcv_status predict_noalloc_impl(pcv_problem* p, int64_t q, const double* ql, double* mean, double* var,
                                int32_t obs_noise, int32_t* owner, bool dev_out) {
  return predict_impl(p, q, ql, mean, var, obs_noise, owner, dev_out);
}

}  // namespace pcv
