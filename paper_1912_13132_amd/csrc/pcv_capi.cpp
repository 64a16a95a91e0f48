// C ABI of the parallel CV library: argument validation, device residency of
// a divided problem (Algorithm 1, steps 2-5 of arXiv:1912.13132: divide and
// read once), and the sequence of kernels of one theta-evaluation
// (Algorithm 1, steps 6-9).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/pcv.h"
#include "pcv_device.h"
#include "pcv_host.h"

using pcv::SubsetDesc;
using pcv::TB;

namespace pcv {
thread_local std::string g_err;
pcv_status fail(pcv_status s, const std::string& msg) {
  g_err = msg;
  return s;
}
}  // namespace pcv

using pcv::fail;

#define HIPCHK(x)                                                                          \
  do {                                                                                     \
    hipError_t e_ = (x);                                                                   \
    if (e_ != hipSuccess) {                                                                \
      (void)hipGetLastError(); /* reported here, not again at a later launch */            \
      return fail(e_ == hipErrorOutOfMemory ? PCV_ERR_OOM : PCV_ERR_DEVICE,                \
                  std::string(#x) + ": " + hipGetErrorString(e_));                         \
    }                                                                                      \
  } while (0)

namespace {

bool is_finite(double v) { return std::isfinite(v); }

pcv_status check_theta(const pcv_theta* t) {
  if (!t) return fail(PCV_ERR_INVALID, "theta is NULL");
  if (t->cov != PCV_COV_EXP && t->cov != PCV_COV_MATERN32)
    return fail(PCV_ERR_INVALID, "theta.cov must be PCV_COV_EXP or PCV_COV_MATERN32");
  if (!(t->range > 0.0) || !is_finite(t->range)) return fail(PCV_ERR_INVALID, "theta.range must be > 0");
  if (!(t->lambda >= 0.0) || !is_finite(t->lambda)) return fail(PCV_ERR_INVALID, "theta.lambda must be >= 0");
  if (!(t->sigma2 > 0.0) || !is_finite(t->sigma2)) return fail(PCV_ERR_INVALID, "theta.sigma2 must be > 0");
  return PCV_OK;
}

// Device-array arguments (inputs_on_device): each one must lie inside a
// single device or managed allocation of the current device, checked before
// any copy so that a wrong pointer or length is an argument error.
pcv_status check_device_range(const void* ptr, size_t bytes, const char* what) {
  if (bytes == 0) return PCV_OK;
  if (!ptr) return fail(PCV_ERR_INVALID, std::string(what) + " is NULL");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return fail(PCV_ERR_DEVICE, "hipGetDevice failed");
  hipPointerAttribute_t a;
  std::memset(&a, 0, sizeof(a));
  if (hipPointerGetAttributes(&a, ptr) != hipSuccess) {
    (void)hipGetLastError();
    return fail(PCV_ERR_INVALID, std::string(what) + " is not a device pointer (inputs_on_device is set)");
  }
  if ((a.type != hipMemoryTypeDevice && a.type != hipMemoryTypeManaged) || a.device != dev)
    return fail(PCV_ERR_INVALID, std::string(what) + " is not memory of the current device");
  hipDeviceptr_t base = nullptr;
  size_t size = 0;
  if (hipMemGetAddressRange(&base, &size, (hipDeviceptr_t)ptr) != hipSuccess) {
    (void)hipGetLastError();
    return fail(PCV_ERR_INVALID, std::string(what) + ": no allocation holds it");
  }
  const char* b = static_cast<const char*>(base);
  const char* q = static_cast<const char*>(ptr);
  if (q < b || (size_t)(q - b) > size || bytes > size - (size_t)(q - b))
    return fail(PCV_ERR_INVALID, std::string(what) + " extends past the end of its allocation");
  return PCV_OK;
}

// Copies device arrays to the host, on the caller's stream when there is one
// (queued writes come first), else after a device-wide synchronisation.
struct DeviceReader {
  hipStream_t s = nullptr;
  bool ready = false;
  pcv_status begin(void* stream) {
    s = (hipStream_t)stream;
    if (!s && hipDeviceSynchronize() != hipSuccess)
      return fail(PCV_ERR_DEVICE, "hipDeviceSynchronize failed before reading device inputs");
    ready = true;
    return PCV_OK;
  }
  template <class T>
  pcv_status read(std::vector<T>& dst, const T* src, size_t count, const char* what) {
    pcv_status st = check_device_range(src, count * sizeof(T), what);
    if (st != PCV_OK) return st;
    dst.resize(count);
    if (count == 0) return PCV_OK;
    hipError_t e = hipMemcpyAsync(dst.data(), src, count * sizeof(T), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(PCV_ERR_DEVICE, std::string("reading ") + what + ": " + hipGetErrorString(e));
    }
    return PCV_OK;
  }
};

}  // namespace

extern "C" {

void pcv_default_options(pcv_options* opt) {
  if (!opt) return;
  std::memset(opt, 0, sizeof(*opt));
  opt->prec = PCV_PREC_MIXED;
  opt->max_refine = 2;
  opt->refine_tol = 1e-4;
  opt->graph = 1;
}

const char* pcv_status_string(pcv_status s) {
  switch (s) {
    case PCV_OK: return "PCV_OK";
    case PCV_ERR_INVALID: return "PCV_ERR_INVALID";
    case PCV_ERR_OOM: return "PCV_ERR_OOM";
    case PCV_ERR_NOT_PD: return "PCV_ERR_NOT_PD";
    case PCV_ERR_DEVICE: return "PCV_ERR_DEVICE";
    case PCV_ERR_STATE: return "PCV_ERR_STATE";
    case PCV_ERR_BUSY: return "PCV_ERR_BUSY";
  }
  return "PCV_ERR_UNKNOWN";
}

const char* pcv_last_error(void) { return pcv::g_err.c_str(); }

pcv_status pcv_selftest_math(int64_t n, const double* t, const double* x, double* e, double* r) {
  pcv::g_err.clear();
  if (n < 0 || (n > 0 && (!t || !x || !e || !r))) return fail(PCV_ERR_INVALID, "bad arguments");
  for (int64_t i = 0; i < n; ++i)
    if (!(t[i] >= 0.0) || !(x[i] >= 0.0) || !is_finite(t[i]) || !is_finite(x[i]))
      return fail(PCV_ERR_INVALID, "inputs must be finite and >= 0");
  if (n == 0) return PCV_OK;
  const size_t bytes = sizeof(double) * (size_t)n;
  double* d = nullptr;
  hipError_t err = hipMalloc((void**)&d, 4 * bytes);
  if (err != hipSuccess) {
    (void)hipGetLastError();
    return fail(PCV_ERR_OOM, hipGetErrorString(err));
  }
  if (err == hipSuccess) err = hipMemcpy(d, t, bytes, hipMemcpyHostToDevice);
  if (err == hipSuccess) err = hipMemcpy(d + n, x, bytes, hipMemcpyHostToDevice);
  if (err == hipSuccess) err = pcv::launch_math_check(nullptr, n, d, d + n, d + 2 * n, d + 3 * n);
  if (err == hipSuccess) err = hipMemcpy(e, d + 2 * n, bytes, hipMemcpyDeviceToHost);
  if (err == hipSuccess) err = hipMemcpy(r, d + 3 * n, bytes, hipMemcpyDeviceToHost);
  (void)hipFree(d);
  if (err != hipSuccess) {
    (void)hipGetLastError();
    return fail(PCV_ERR_DEVICE, hipGetErrorString(err));
  }
  return PCV_OK;
}

pcv_status pcv_problem_create(pcv_problem** out, int64_t n, const double* locs, const double* y,
                              int32_t S, const int64_t* train_ptr, const int32_t* train_idx,
                              const int64_t* val_ptr, const int32_t* val_idx, const double* core_rect,
                              const pcv_options* opt) {
  pcv::g_err.clear();
  if (!out) return fail(PCV_ERR_INVALID, "out is NULL");
  *out = nullptr;
  if (n < 1) return fail(PCV_ERR_INVALID, "n must be >= 1");
  if (n > INT32_MAX) return fail(PCV_ERR_INVALID, "n must fit in int32 indices");
  if (!locs || !y) return fail(PCV_ERR_INVALID, "locs and y must be non-NULL");
  if (S < 1) return fail(PCV_ERR_INVALID, "S must be >= 1");
  if (!train_ptr || !val_ptr) return fail(PCV_ERR_INVALID, "train_ptr and val_ptr must be non-NULL");
  pcv_options o;
  pcv_default_options(&o);
  if (opt) o = *opt;
  // device inputs: host copies, then the same validation as host inputs
  std::vector<double> h_locs, h_y, h_rect;
  std::vector<int64_t> h_tp, h_vp;
  std::vector<int32_t> h_ti, h_vi;
  if (o.inputs_on_device) {
    DeviceReader rd;
    pcv_status st = rd.begin(o.hip_stream);
    if (st == PCV_OK) st = rd.read(h_tp, train_ptr, (size_t)S + 1, "train_ptr");
    if (st == PCV_OK) st = rd.read(h_vp, val_ptr, (size_t)S + 1, "val_ptr");
    if (st != PCV_OK) return st;
    for (int32_t i = 0; i < S; ++i)
      if (h_tp[i + 1] < h_tp[i] || h_vp[i + 1] < h_vp[i])
        return fail(PCV_ERR_INVALID, "ptr array decreases at subset " + std::to_string(i));
    if (h_tp[0] != 0 || h_vp[0] != 0) return fail(PCV_ERR_INVALID, "ptr arrays must start at 0");
    if (st == PCV_OK) st = rd.read(h_locs, locs, 2 * (size_t)n, "locs");
    if (st == PCV_OK) st = rd.read(h_y, y, (size_t)n, "y");
    if (st == PCV_OK) st = rd.read(h_ti, train_idx, (size_t)h_tp[S], "train_idx");
    if (st == PCV_OK) st = rd.read(h_vi, val_idx, (size_t)h_vp[S], "val_idx");
    if (st == PCV_OK && core_rect) st = rd.read(h_rect, core_rect, 4 * (size_t)S, "core_rect");
    if (st != PCV_OK) return st;
    locs = h_locs.data();
    y = h_y.data();
    train_ptr = h_tp.data();
    val_ptr = h_vp.data();
    train_idx = h_ti.empty() ? nullptr : h_ti.data();
    val_idx = h_vi.empty() ? nullptr : h_vi.data();
    core_rect = core_rect ? h_rect.data() : nullptr;
  }
  if (train_ptr[0] != 0 || val_ptr[0] != 0) return fail(PCV_ERR_INVALID, "ptr arrays must start at 0");
  for (int32_t i = 0; i < S; ++i) {
    if (train_ptr[i + 1] < train_ptr[i]) return fail(PCV_ERR_INVALID, "train_ptr decreases at subset " + std::to_string(i));
    if (val_ptr[i + 1] < val_ptr[i]) return fail(PCV_ERR_INVALID, "val_ptr decreases at subset " + std::to_string(i));
    if (train_ptr[i + 1] - train_ptr[i] > PCV_MAX_SUBSET)
      return fail(PCV_ERR_INVALID, "subset " + std::to_string(i) + " has more than PCV_MAX_SUBSET training points");
  }
  if ((train_ptr[S] > 0 && !train_idx) || (val_ptr[S] > 0 && !val_idx))
    return fail(PCV_ERR_INVALID, "index arrays must be non-NULL when non-empty");
  for (int64_t j = 0; j < train_ptr[S]; ++j)
    if (train_idx[j] < 0 || train_idx[j] >= n) return fail(PCV_ERR_INVALID, "train_idx[" + std::to_string(j) + "] out of range");
  for (int64_t j = 0; j < val_ptr[S]; ++j)
    if (val_idx[j] < 0 || val_idx[j] >= n) return fail(PCV_ERR_INVALID, "val_idx[" + std::to_string(j) + "] out of range");
  for (int64_t j = 0; j < n; ++j)
    if (!is_finite(locs[2 * j]) || !is_finite(locs[2 * j + 1]) || !is_finite(y[j]))
      return fail(PCV_ERR_INVALID, "non-finite location or value at point " + std::to_string(j));
  if (core_rect)
    for (int64_t j = 0; j < 4LL * S; ++j)
      if (!is_finite(core_rect[j])) return fail(PCV_ERR_INVALID, "non-finite core_rect");
  if (o.prec != PCV_PREC_FP64 && o.prec != PCV_PREC_MIXED) return fail(PCV_ERR_INVALID, "opt.prec invalid");
  if (o.max_refine < 0 || o.max_refine > 8) return fail(PCV_ERR_INVALID, "opt.max_refine must be in [0, 8]");
  if (!(o.refine_tol >= 0.0)) return fail(PCV_ERR_INVALID, "opt.refine_tol must be >= 0");
  if (o.max_wg_per_subset < 0 || o.max_wg_per_subset > 8)
    return fail(PCV_ERR_INVALID, "opt.max_wg_per_subset must be in [0, 8]");

  pcv_problem* p = new pcv_problem();
  p->opt = o;
  pcv_status st = pcv::problem_build(p, n, locs, y, S, train_ptr, train_idx, val_ptr, val_idx, core_rect);
  if (st != PCV_OK) {
    std::string keep = pcv::g_err;
    pcv::problem_free(p);
    pcv::g_err = keep;
    return st;
  }
  *out = p;
  return PCV_OK;
}

pcv_status pcv_problem_destroy(pcv_problem* p) {
  if (!p) return fail(PCV_ERR_INVALID, "problem is NULL");
  pcv::problem_free(p);
  return PCV_OK;
}

pcv_status pcv_problem_info(const pcv_problem* p, int32_t* S, int64_t* nnz_train, int32_t* max_train,
                            size_t* device_bytes) {
  if (!p) return fail(PCV_ERR_INVALID, "problem is NULL");
  if (S) *S = p->S;
  if (nnz_train) *nnz_train = p->nnzT;
  if (max_train) *max_train = p->max_train;
  if (device_bytes) *device_bytes = p->dev_bytes;
  return PCV_OK;
}

pcv_status pcv_eval(pcv_problem* p, const pcv_theta* theta, double* loss, pcv_eval_report* report) {
  pcv::g_err.clear();
  if (!p) return fail(PCV_ERR_INVALID, "problem is NULL");
  if (!loss) return fail(PCV_ERR_INVALID, "loss is NULL");
  pcv_status s = check_theta(theta);
  if (s != PCV_OK) return s;
  return pcv::eval_impl(p, *theta, loss, report);
}

pcv_status pcv_autotune(pcv_problem* p, const pcv_theta* theta, const char* cache_path, int32_t reps,
                        pcv_tune_report* report) {
  pcv::g_err.clear();
  if (!p) return fail(PCV_ERR_INVALID, "problem is NULL");
  pcv_status s = check_theta(theta);
  if (s != PCV_OK) return s;
  if (reps < 1 || reps > 20) return fail(PCV_ERR_INVALID, "reps must be in [1, 20]");
  return pcv::autotune_impl(p, *theta, cache_path, reps, report);
}

pcv_status pcv_eval_batch(pcv_problem* p, int32_t n_theta, const pcv_theta* thetas, double* losses) {
  pcv::g_err.clear();
  if (!p) return fail(PCV_ERR_INVALID, "problem is NULL");
  if (n_theta < 0 || (n_theta > 0 && (!thetas || !losses))) return fail(PCV_ERR_INVALID, "bad batch arguments");
  for (int32_t k = 0; k < n_theta; ++k) {
    pcv_status s = check_theta(&thetas[k]);
    if (s != PCV_OK) return fail(s, "theta[" + std::to_string(k) + "]: " + pcv::g_err);
  }
  return pcv::eval_batch_impl(p, n_theta, thetas, losses, nullptr);
}

pcv_status pcv_eval_batch_ex(pcv_problem* p, int32_t n_theta, const pcv_theta* thetas, double* losses,
                             pcv_eval_report* report) {
  pcv::g_err.clear();
  if (!p) return fail(PCV_ERR_INVALID, "problem is NULL");
  if (n_theta < 0 || (n_theta > 0 && (!thetas || !losses))) return fail(PCV_ERR_INVALID, "bad batch arguments");
  for (int32_t k = 0; k < n_theta; ++k) {
    pcv_status s = check_theta(&thetas[k]);
    if (s != PCV_OK) return fail(s, "theta[" + std::to_string(k) + "]: " + pcv::g_err);
  }
  return pcv::eval_batch_impl(p, n_theta, thetas, losses, report);
}

pcv_status pcv_eval_grid(pcv_problem* p, int32_t n_theta, const pcv_theta* thetas, double* losses,
                         double* per_subset_sspe, int32_t* best) {
  pcv::g_err.clear();
  if (!p) return fail(PCV_ERR_INVALID, "problem is NULL");
  if (n_theta < 0 || (n_theta > 0 && (!thetas || !losses))) return fail(PCV_ERR_INVALID, "bad grid arguments");
  for (int32_t k = 0; k < n_theta; ++k) {
    pcv_status s = check_theta(&thetas[k]);
    if (s != PCV_OK) return fail(s, "theta[" + std::to_string(k) + "]: " + pcv::g_err);
  }
  const int32_t S = p->S;
  std::vector<double> own;
  double* z = per_subset_sspe;
  if (!z && best) {
    own.resize((size_t)n_theta * S);
    z = own.data();
  }
  // the multi-theta launches (one launch per kernel over up to 64 theta
  // values), bit for bit the single evaluations
  pcv_status s = pcv::eval_batch_impl(p, n_theta, thetas, losses, nullptr, z);
  if (s != PCV_OK) return s;
  if (best)
    for (int32_t i = 0; i < S; ++i) {
      int32_t b = -1;
      if (p->active[i] && n_theta > 0) {
        b = 0;
        for (int32_t k = 1; k < n_theta; ++k)
          if (z[(size_t)k * S + i] < z[(size_t)b * S + i]) b = k;
      }
      best[i] = b;
    }
  return PCV_OK;
}

pcv_status pcv_factor(pcv_problem* p, const pcv_theta* theta) {
  pcv::g_err.clear();
  if (!p) return fail(PCV_ERR_INVALID, "problem is NULL");
  pcv_status s = check_theta(theta);
  if (s != PCV_OK) return s;
  return pcv::factor_impl(p, theta, false);
}

pcv_status pcv_gls(pcv_problem* p, int32_t n_cov, const double* X, double* beta, int32_t* status) {
  pcv::g_err.clear();
  if (!p) return fail(PCV_ERR_INVALID, "problem is NULL");
  if (n_cov < 1 || n_cov > pcv::GLS_MAXP) return fail(PCV_ERR_INVALID, "n_cov must be in [1, 8]");
  if (!X || !beta) return fail(PCV_ERR_INVALID, "X or beta is NULL");
  for (int64_t j = 0; j < p->n * n_cov; ++j)
    if (!is_finite(X[j])) return fail(PCV_ERR_INVALID, "non-finite covariate");
  if (!p->factored) return fail(PCV_ERR_STATE, "pcv_gls called before pcv_factor");
  return pcv::gls_impl(p, n_cov, X, beta, status);
}

pcv_status pcv_factor_local(pcv_problem* p, const pcv_theta* thetas) {
  pcv::g_err.clear();
  if (!p) return fail(PCV_ERR_INVALID, "problem is NULL");
  if (!thetas) return fail(PCV_ERR_INVALID, "thetas is NULL");
  for (int32_t i = 0; i < p->S; ++i) {
    pcv_status s = check_theta(thetas + i);
    if (s != PCV_OK) return fail(s, "thetas[" + std::to_string(i) + "]: " + pcv::g_err);
  }
  return pcv::factor_impl(p, thetas, true);
}

pcv_status pcv_predict(pcv_problem* p, int64_t q, const double* qlocs, double* mean, double* var,
                       int32_t obs_noise, int32_t* owner) {
  pcv::g_err.clear();
  if (!p) return fail(PCV_ERR_INVALID, "problem is NULL");
  if (q < 0 || (q > 0 && (!qlocs || !mean))) return fail(PCV_ERR_INVALID, "bad query arguments");
  std::vector<double> h_q;
  const bool dev = p->opt.inputs_on_device != 0;
  if (dev && q > 0) {
    DeviceReader rd;
    pcv_status st = check_device_range(mean, sizeof(double) * q, "mean");
    if (st == PCV_OK && var) st = check_device_range(var, sizeof(double) * q, "var");
    if (st == PCV_OK && owner) st = check_device_range(owner, sizeof(int32_t) * q, "owner");
    if (st == PCV_OK) st = rd.begin(p->own_stream ? nullptr : (void*)p->stream);
    if (st == PCV_OK) st = rd.read(h_q, qlocs, 2 * (size_t)q, "qlocs");
    if (st != PCV_OK) return st;
    qlocs = h_q.data();
  }
  for (int64_t j = 0; j < 2 * q; ++j)
    if (!is_finite(qlocs[j])) return fail(PCV_ERR_INVALID, "non-finite query location");
  if (!p->factored) return fail(PCV_ERR_STATE, "pcv_predict called before pcv_factor");
  return pcv::predict_impl(p, q, qlocs, mean, var, obs_noise, owner, dev);
}

pcv_status pcv_predict_noalloc(pcv_problem* p, int64_t q, const double* qlocs, double* mean, double* var,
                               int32_t obs_noise, int32_t* owner) {
  pcv::g_err.clear();
  if (!p) return fail(PCV_ERR_INVALID, "problem is NULL");
  if (q < 0 || (q > 0 && (!qlocs || !mean))) return fail(PCV_ERR_INVALID, "bad query arguments");
  if (q > PCV_NOALLOC_MAX_QUERIES)
    return fail(PCV_ERR_INVALID, "pcv_predict_noalloc takes at most " + std::to_string(PCV_NOALLOC_MAX_QUERIES) +
                                     " queries per call (got " + std::to_string(q) + ")");
  const bool dev = p->opt.inputs_on_device != 0;
  if (dev && q > 0) {
    DeviceReader rd;
    pcv_status st = check_device_range(mean, sizeof(double) * q, "mean");
    if (st == PCV_OK && var) st = check_device_range(var, sizeof(double) * q, "var");
    if (st == PCV_OK && owner) st = check_device_range(owner, sizeof(int32_t) * q, "owner");
    if (st == PCV_OK) st = rd.begin(p->own_stream ? nullptr : (void*)p->stream);
    if (st == PCV_OK) st = rd.read(p->na_q, qlocs, 2 * (size_t)q, "qlocs");
    if (st != PCV_OK) return st;
    qlocs = p->na_q.data();
  }
  for (int64_t j = 0; j < 2 * q; ++j)
    if (!is_finite(qlocs[j])) return fail(PCV_ERR_INVALID, "non-finite query location");
  if (!p->factored) return fail(PCV_ERR_STATE, "pcv_predict_noalloc called before pcv_factor");
  return pcv::predict_noalloc_impl(p, q, qlocs, mean, var, obs_noise, owner, dev);
}

namespace {
pcv_status check_points(int64_t n, const double* locs) {
  if (n < 1 || !locs) return fail(PCV_ERR_INVALID, "n must be >= 1 and locs non-NULL");
  if (n > INT32_MAX) return fail(PCV_ERR_INVALID, "at most 2^31 - 1 points");
  for (int64_t j = 0; j < 2 * n; ++j)
    if (!is_finite(locs[j])) return fail(PCV_ERR_INVALID, "non-finite location");
  return PCV_OK;
}
pcv_status check_rects(int32_t S, const double* R) {
  if (S < 1 || !R) return fail(PCV_ERR_INVALID, "S must be >= 1 and core_rect non-NULL");
  for (int64_t j = 0; j < 4 * (int64_t)S; ++j)
    if (!is_finite(R[j])) return fail(PCV_ERR_INVALID, "non-finite core rectangle");
  for (int32_t i = 0; i < S; ++i)
    if (!(R[4 * i] <= R[4 * i + 2]) || !(R[4 * i + 1] <= R[4 * i + 3]))
      return fail(PCV_ERR_INVALID, "core rectangle " + std::to_string(i) + " has lo > hi");
  return PCV_OK;
}
}  // namespace

pcv_status pcv_part_divide(int64_t n, const double* locs, const double* domain, int32_t m, double delta,
                           double* core_rect) {
  pcv::g_err.clear();
  pcv_status s = check_points(n, locs);
  if (s != PCV_OK) return s;
  if (!domain || !core_rect || m < 1) return fail(PCV_ERR_INVALID, "bad domain, m or output");
  if (!is_finite(delta) || delta < 0) return fail(PCV_ERR_INVALID, "delta must be finite and >= 0");
  if (!(domain[0] <= domain[2]) || !(domain[1] <= domain[3])) return fail(PCV_ERR_INVALID, "domain has lo > hi");
  return pcv::part_divide(n, locs, domain, m, delta, core_rect);
}

pcv_status pcv_part_count(int64_t n, const double* locs, int32_t S, const double* core_rect, double delta,
                          int64_t* memberships) {
  pcv::g_err.clear();
  pcv_status s = check_points(n, locs);
  if (s == PCV_OK) s = check_rects(S, core_rect);
  if (s != PCV_OK) return s;
  if (!memberships) return fail(PCV_ERR_INVALID, "memberships is NULL");
  if (!is_finite(delta) || delta < 0) return fail(PCV_ERR_INVALID, "delta must be finite and >= 0");
  return pcv::part_subsets(n, locs, S, core_rect, delta, nullptr, nullptr, memberships, nullptr, nullptr,
                           nullptr, nullptr);
}

pcv_status pcv_part_subsets(int64_t n, const double* locs, int32_t S, const double* core_rect, double delta,
                            const uint8_t* is_val, int32_t* owner, int64_t* train_ptr, int32_t* train_idx,
                            int64_t* val_ptr, int32_t* val_idx) {
  pcv::g_err.clear();
  pcv_status s = check_points(n, locs);
  if (s == PCV_OK) s = check_rects(S, core_rect);
  if (s != PCV_OK) return s;
  if (!is_finite(delta) || delta < 0) return fail(PCV_ERR_INVALID, "delta must be finite and >= 0");
  if ((train_idx && !train_ptr) || (val_idx && !val_ptr)) return fail(PCV_ERR_INVALID, "index list without ptr");
  return pcv::part_subsets(n, locs, S, core_rect, delta, is_val, owner, nullptr, train_ptr, train_idx, val_ptr,
                           val_idx);
}

pcv_status pcv_server_set_batch_window(pcv_server* s, double seconds) {
  pcv::g_err.clear();
  if (!s) return fail(PCV_ERR_INVALID, "server is NULL");
  if (!(seconds >= 0.0 && seconds <= 10.0)) return fail(PCV_ERR_INVALID, "window must be in [0, 10] seconds");
  return pcv::server_set_window(s, seconds);
}

pcv_status pcv_server_create(pcv_server** out, pcv_problem* p, size_t mem_budget, int32_t max_inflight) {
  pcv::g_err.clear();
  if (!out) return fail(PCV_ERR_INVALID, "out is NULL");
  *out = nullptr;
  if (!p) return fail(PCV_ERR_INVALID, "problem is NULL");
  if (max_inflight < 1) return fail(PCV_ERR_INVALID, "max_inflight must be >= 1");
  return pcv::server_create(out, p, mem_budget, max_inflight, 3);
}

pcv_status pcv_server_submit_predict(pcv_server* s, int64_t q, const double* qlocs, double* mean,
                                     double* var, int32_t obs_noise, pcv_ticket* ticket) {
  pcv::g_err.clear();
  if (!s || !ticket) return fail(PCV_ERR_INVALID, "server or ticket is NULL");
  if (q < 0 || q > INT32_MAX || (q > 0 && (!qlocs || !mean))) return fail(PCV_ERR_INVALID, "bad query arguments");
  for (int64_t j = 0; j < 2 * q; ++j)
    if (!is_finite(qlocs[j])) return fail(PCV_ERR_INVALID, "non-finite query location");
  if (!pcv::server_problem(s)->factored) return fail(PCV_ERR_STATE, "kriging request before pcv_factor");
  return pcv::server_submit_predict(s, q, qlocs, mean, var, obs_noise, ticket);
}

pcv_status pcv_server_submit_eval(pcv_server* s, const pcv_theta* theta, double* loss, pcv_ticket* ticket) {
  pcv::g_err.clear();
  if (!s || !ticket || !loss) return fail(PCV_ERR_INVALID, "server, loss or ticket is NULL");
  pcv_status st = check_theta(theta);
  if (st != PCV_OK) return st;
  return pcv::server_submit_eval(s, *theta, loss, ticket);
}

pcv_status pcv_server_wait(pcv_server* s, pcv_ticket ticket, double timeout_s) {
  pcv::g_err.clear();
  if (!s) return fail(PCV_ERR_INVALID, "server is NULL");
  if (std::isnan(timeout_s)) return fail(PCV_ERR_INVALID, "timeout is NaN");
  return pcv::server_wait(s, ticket, timeout_s);
}

pcv_status pcv_server_stats(pcv_server* s, double* p50_s, double* p99_s, double* qps, double* evals_per_s) {
  pcv::g_err.clear();
  if (!s) return fail(PCV_ERR_INVALID, "server is NULL");
  pcv_server_report r;
  pcv_status st = pcv::server_report(s, &r);
  if (st != PCV_OK) return st;
  if (p50_s) *p50_s = r.p50_s;
  if (p99_s) *p99_s = r.p99_s;
  if (qps) *qps = r.qps;
  if (evals_per_s) *evals_per_s = r.evals_per_s;
  return PCV_OK;
}

pcv_status pcv_server_report_get(pcv_server* s, pcv_server_report* out) {
  pcv::g_err.clear();
  if (!s || !out) return fail(PCV_ERR_INVALID, "server or report is NULL");
  return pcv::server_report(s, out);
}

pcv_status pcv_server_destroy(pcv_server* s) {
  pcv::g_err.clear();
  if (!s) return fail(PCV_ERR_INVALID, "server is NULL");
  return pcv::server_destroy(s);
}

}  // extern "C"
