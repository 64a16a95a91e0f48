// Kriging prediction without device allocation: pcv_predict's work buffers
// (grouped query coordinates, their flags and original positions, the work
// items, the means and variances, and the per-item panels of the variance's
// forward substitution) placed in one fixed device array instead of memory
// allocated per call.  Same kernel, same items, same results bit for bit.
//
// The array lives in this library's code object, one copy per device, from
// the first call on that device until the process ends.  Its device address
// is taken once per device with hipGetSymbolAddress (with that device
// current) and only that address is used afterwards.  Calls on one device
// share the array, so they are serialised inside the process by a
// per-device mutex held until the call's stream has drained.  Nothing in
// the array needs clearing between calls: every query's mean (and
// variance) is written by the kernel, and each variance panel row is
// written before the kernel reads it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <string>

#include "pcv_host.h"

namespace pcv {

namespace {

constexpr size_t SCRATCH_BYTES = (size_t)PCV_NOALLOC_SCRATCH_MIB << 20;
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
void* g_scratch[MAX_DEVICES] = {};
std::mutex g_mu[MAX_DEVICES];

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

// The fixed layout for q queries and n_items items: items, qx, qy, qorig,
// qflag, mean, var, then the variance panels in what is left.
struct NoAllocLayout {
  size_t items, qx, qy, qorig, qflag, mean, var, w, w_doubles;
};

static bool noalloc_layout(int64_t q, size_t n_items, NoAllocLayout& L) {
  size_t o = 0;
  L.items = o;
  o = align256(o + sizeof(KrigeItem) * n_items);
  L.qx = o;
  o = align256(o + sizeof(double) * q);
  L.qy = o;
  o = align256(o + sizeof(double) * q);
  L.qorig = o;
  o = align256(o + sizeof(int32_t) * q);
  L.qflag = o;
  o = align256(o + sizeof(int32_t) * q);
  L.mean = o;
  o = align256(o + sizeof(double) * q);
  L.var = o;
  o = align256(o + sizeof(double) * q);
  L.w = o;
  if (o >= SCRATCH_BYTES) return false;
  L.w_doubles = (SCRATCH_BYTES - o) / sizeof(double);
  return true;
}

pcv_status predict_noalloc_impl(pcv_problem* p, int64_t q, const double* ql, double* mean, double* var,
                                int32_t obs_noise, int32_t* owner_out, bool dev_out) {
  if (q > PCV_NOALLOC_MAX_QUERIES)
    return fail(PCV_ERR_INVALID, "pcv_predict_noalloc takes at most " + std::to_string(PCV_NOALLOC_MAX_QUERIES) +
                                     " queries per call (got " + std::to_string(q) + ")");
  if (p->device < 0 || p->device >= MAX_DEVICES) return fail(PCV_ERR_INVALID, "device ordinal out of range");
  if (hipSetDevice(p->device) != hipSuccess) return fail(PCV_ERR_DEVICE, "hipSetDevice failed");
  if (q == 0) return PCV_OK;
  std::lock_guard<std::mutex> lock(g_mu[p->device]);
  if (!g_scratch[p->device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(PCV_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch[p->device] = ptr;
  }
  unsigned char* base = static_cast<unsigned char*>(g_scratch[p->device]);

  // routing and the item plan on the host, in buffers the problem keeps
  std::vector<int32_t>& owner = p->na_owner;
  owner.resize(q);
  route(p, q, ql, owner.data());
  if (owner_out && !dev_out) std::copy(owner.begin(), owner.end(), owner_out);
  KrigePlan& P = p->na_plan;
  const int32_t flag = (var ? KRIGE_VAR : 0) | (obs_noise ? KRIGE_OBS_NOISE : 0);
  plan_krige(p, q, ql, owner.data(), nullptr, flag, P);
  const size_t ni = P.items.size();
  NoAllocLayout Lo;
  if (!noalloc_layout(q, ni, Lo)) return fail(PCV_ERR_INVALID, "query count exceeds the scratch array");
  // launch groups: consecutive items whose variance panels fit the panel area
  // together; each item's panel offset is rebased to the start of that area
  std::vector<std::pair<int32_t, int32_t>>& groups = p->na_groups;
  groups.clear();
  {
    int32_t g0 = 0;
    int64_t used = 0;
    for (size_t k = 0; k < ni; ++k) {
      KrigeItem& it = P.items[k];
      const int64_t need = (it.flags & KRIGE_VAR) ? (int64_t)p->desc[it.sidx].npad * KRIGE_Q : 0;
      if (need > (int64_t)Lo.w_doubles)
        return fail(PCV_ERR_INVALID, "a subset's variance panel exceeds the scratch array");
      if (used + need > (int64_t)Lo.w_doubles) {
        groups.emplace_back(g0, (int32_t)k);
        g0 = (int32_t)k;
        used = 0;
      }
      it.woff = used;
      used += need;
    }
    groups.emplace_back(g0, (int32_t)ni);
  }

  hipStream_t st = p->stream;
  KrigeItem* d_items = reinterpret_cast<KrigeItem*>(base + Lo.items);
  double* d_qx = reinterpret_cast<double*>(base + Lo.qx);
  double* d_qy = reinterpret_cast<double*>(base + Lo.qy);
  int32_t* d_qorig = reinterpret_cast<int32_t*>(base + Lo.qorig);
  int32_t* d_qflag = reinterpret_cast<int32_t*>(base + Lo.qflag);
  double* d_mean = reinterpret_cast<double*>(base + Lo.mean);
  double* d_var = reinterpret_cast<double*>(base + Lo.var);
  double* d_W = reinterpret_cast<double*>(base + Lo.w);
  hipError_t e = hipMemcpyAsync(d_qx, P.qx.data(), sizeof(double) * q, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(d_qy, P.qy.data(), sizeof(double) * q, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(d_qorig, P.qorig.data(), sizeof(int32_t) * q, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(d_qflag, P.qflag.data(), sizeof(int32_t) * q, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(d_items, P.items.data(), sizeof(KrigeItem) * ni, hipMemcpyHostToDevice, st);
  // the groups run one after another on the stream and reuse the panel area
  for (size_t g = 0; g < groups.size() && e == hipSuccess; ++g)
    e = launch_krige(st, p->d_desc_fact, p->d_theta_fact, d_items + groups[g].first,
                     groups[g].second - groups[g].first, p->d_tx, p->d_ty, p->d_Lf, p->d_Invf, p->d_alpha_fact,
                     d_qx, d_qy, d_qorig, d_qflag, d_W, d_mean, d_var);
  const hipMemcpyKind out_kind = dev_out ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  if (e == hipSuccess) e = hipMemcpyAsync(mean, d_mean, sizeof(double) * q, out_kind, st);
  if (e == hipSuccess && var) e = hipMemcpyAsync(var, d_var, sizeof(double) * q, out_kind, st);
  if (e == hipSuccess && owner_out && dev_out)
    e = hipMemcpyAsync(owner_out, owner.data(), sizeof(int32_t) * q, hipMemcpyHostToDevice, st);
  // drained before the lock is released: the next call may reuse the array
  const hipError_t es = hipStreamSynchronize(st);
  if (e == hipSuccess) e = es;
  if (e != hipSuccess) return fail(PCV_ERR_DEVICE, std::string("predict_noalloc: ") + hipGetErrorString(e));
  return PCV_OK;
}

}  // namespace pcv
