// Serving loop over a resident problem: kriging requests (eq. (3) mean and
// the simple-kriging variance, from the FP64 factors of pcv_factor) and
// theta-evaluation requests (eq. (7)), with continuous batching.
//
// Prediction requests are routed in the submitting thread.  A batcher
// thread packs the queued queries, first come first served, into the next
// free workspace slot until the slot's query or scratch capacity is reached
// (a request larger than that spans several batches), groups them by
// subset across requests so each subset's factor is read once per batch,
// and launches the batch on the slot's stream.  A completion thread waits
// for the batches in launch order and scatters results to the callers.
// Slots are pinned host + device buffers allocated once; with several slots
// the host work of one batch overlaps the device work of the previous ones.
// Evaluation requests run in their own thread on the problem's stream, so
// kriging batches and evaluations share the device.
//
// Every query is computed by one lane of the kriging kernel from its own
// coordinates and the subset's resident factors, so its result does not
// depend on which other queries share its batch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/pcv.h"
#include "pcv_device.h"
#include "pcv_host.h"

using pcv::KrigeItem;

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

enum ReqKind { REQ_PREDICT = 0, REQ_EVAL = 1 };

struct Req {
  pcv_ticket id = 0;
  ReqKind kind = REQ_PREDICT;
  // prediction
  int64_t q = 0;
  const double* ql = nullptr;
  double* mean = nullptr;
  double* var = nullptr;
  int32_t flag = 0;
  std::vector<int32_t> owner;
  int64_t next = 0;  // first query not yet placed in a batch
  int64_t done = 0;  // queries of finished batches
  bool failed = false;
  // evaluation
  pcv_theta th{};
  double* loss = nullptr;
  // completion
  bool finished = false;
  pcv_status st = PCV_OK;
  std::string err;
  double t_submit = 0.0, t_done = 0.0;
};

struct Piece {
  Req* r;
  int64_t r0, cnt, b0;  // queries [r0, r0+cnt) of r are batch queries [b0, b0+cnt)
};

// A batch's inputs travel in one copy and its results in another: the
// query coordinates, original positions, flags and items are packed back to
// back in one buffer (in_layout), the means and variances in another.
struct InLayout {
  size_t qy, qorig, qflag, items, bytes;
};
InLayout in_layout(int64_t nq, int64_t ni) {
  InLayout L;
  L.qy = 8 * (size_t)nq;
  L.qorig = 16 * (size_t)nq;
  L.qflag = 20 * (size_t)nq;
  L.items = (24 * (size_t)nq + 15) & ~(size_t)15;
  L.bytes = L.items + sizeof(KrigeItem) * (size_t)ni;
  return L;
}

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  char *d_in = nullptr, *h_in = nullptr;      // packed batch inputs (in_layout)
  double *d_out = nullptr, *h_out = nullptr;  // means [0, nq), variances [nq, 2 nq)
  double* d_W = nullptr;                      // variance scratch
  const double *h_mean = nullptr, *h_var = nullptr;  // the last batch's results in h_out
  std::vector<Piece> pieces;
  int64_t nq = 0;
  bool any_var = false;
  hipError_t err = hipSuccess;
};

}  // namespace

struct pcv_server {
  pcv_problem* p = nullptr;
  int32_t max_inflight = 64;
  int64_t q_cap = 0;       // queries per batch
  int64_t item_cap = 0;    // items per batch
  int64_t w_cap = 0;       // variance scratch doubles per batch
  size_t ws_bytes = 0;     // device bytes of all slots
  std::vector<Slot> slots;
  // Evaluations run on a stream of the server's own (the problem's stream is
  // swapped for it while served).
  hipStream_t eval_stream = nullptr;
  hipStream_t saved_stream = nullptr;

  std::mutex mu;
  std::condition_variable cv_batch;  // batcher: work queued or slot freed
  std::condition_variable cv_done;   // waiters: a request finished
  std::condition_variable cv_admit;  // submitters: in-flight count dropped
  std::condition_variable cv_eval;   // evaluator: evaluation queued
  std::condition_variable cv_comp;   // completion thread: batch launched
  std::deque<Req*> pred_q;           // requests with queries not yet batched
  std::deque<Req*> eval_q;
  std::deque<int> free_slots;
  std::deque<int> launched;          // slots in launch order
  std::unordered_map<pcv_ticket, Req*> reqs;
  pcv_ticket next_id = 1;
  int32_t inflight = 0;
  bool stop = false;
  // Batching window: while evaluations are queued or running, a kriging
  // batch is launched only once its oldest query has waited window_s, or
  // the queue holds a full slot, so that kriging leaves the device to the
  // evaluations between batches; without evaluations a batch is launched
  // as soon as a slot is free.
  double window_s = 0.03;
  int64_t queued_q = 0;   // queries queued and not yet in a batch
  bool eval_busy = false; // the evaluator is running evaluations

  // statistics
  std::vector<double> lat_pred, lat_eval;
  int64_t n_queries = 0, n_batches = 0, batch_queries = 0, admission_waits = 0;
  double t_first = -1.0, t_last = 0.0;

  std::thread th_batch, th_comp, th_eval;
};

namespace pcv {

namespace {

void finish_locked(pcv_server* s, Req* r, pcv_status st, const std::string& err) {
  r->finished = true;
  r->st = st;
  r->err = err;
  r->t_done = now_s();
  s->t_last = std::max(s->t_last, r->t_done);
  if (st == PCV_OK) {
    if (r->kind == REQ_PREDICT) {
      s->lat_pred.push_back(r->t_done - r->t_submit);
      s->n_queries += r->q;
    } else {
      s->lat_eval.push_back(r->t_done - r->t_submit);
    }
  }
  --s->inflight;
  s->cv_admit.notify_all();
  s->cv_done.notify_all();
}

// Fill one slot from the queue head.  Called with the lock held; takes
// queries first come first served while the slot's capacities allow.
void take_batch_locked(pcv_server* s, Slot& sl) {
  const pcv_problem* p = s->p;
  sl.pieces.clear();
  sl.nq = 0;
  sl.any_var = false;
  // per-subset query counts of this batch, to count items and scratch
  static thread_local std::vector<int32_t> cnt;
  cnt.assign(p->S, 0);
  int64_t items = 0, wd = 0;
  bool full = false;
  while (!s->pred_q.empty() && !full) {
    Req* r = s->pred_q.front();
    const int64_t r0 = r->next;
    int64_t j = r0;
    for (; j < r->q && sl.nq + (j - r0) < s->q_cap; ++j) {
      const int32_t i = r->owner[j];
      if (cnt[i] % KRIGE_Q == 0) {
        // a new item for subset i; reserve scratch as if it needs variance
        const int64_t w = (int64_t)p->desc[i].npad * KRIGE_Q;
        if (items + 1 > s->item_cap || wd + w > s->w_cap) {
          full = true;
          break;
        }
        ++items;
        wd += w;
      }
      ++cnt[i];
    }
    if (j > r0) {
      sl.pieces.push_back(Piece{r, r0, j - r0, sl.nq});
      sl.nq += j - r0;
      s->queued_q -= j - r0;
      sl.any_var |= (r->flag & KRIGE_VAR) != 0;
      r->next = j;
    }
    if (r->next == r->q) s->pred_q.pop_front();
    if (sl.nq >= s->q_cap) full = true;
  }
}

void batcher(pcv_server* s) {
  pcv_problem* p = s->p;
  (void)hipSetDevice(p->device);
  KrigePlan plan;
  std::vector<double> ql;
  std::vector<int32_t> owner, flags;
  for (;;) {
    int si;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      // drain the queue before stopping; while evaluations are active, wait
      // for the window or a full slot
      for (;;) {
        if (s->stop && s->pred_q.empty()) break;
        if (!s->pred_q.empty() && !s->free_slots.empty()) {
          const bool evals = s->eval_busy || !s->eval_q.empty();
          const double due = s->pred_q.front()->t_submit + s->window_s;
          if (s->stop || !evals || s->queued_q >= s->q_cap || now_s() >= due) break;
          s->cv_batch.wait_for(lk, std::chrono::duration<double>(std::max(0.0, due - now_s())));
          continue;
        }
        s->cv_batch.wait(lk);
      }
      if (s->pred_q.empty()) break;
      si = s->free_slots.front();
      s->free_slots.pop_front();
      take_batch_locked(s, s->slots[si]);
    }
    Slot& sl = s->slots[si];
    // gather the batch's queries in piece order and plan the launch
    const int64_t nq = sl.nq;
    ql.resize(2 * nq);
    owner.resize(nq);
    flags.resize(nq);
    for (const Piece& pc : sl.pieces) {
      std::copy(pc.r->ql + 2 * pc.r0, pc.r->ql + 2 * (pc.r0 + pc.cnt), ql.begin() + 2 * pc.b0);
      std::copy(pc.r->owner.begin() + pc.r0, pc.r->owner.begin() + pc.r0 + pc.cnt, owner.begin() + pc.b0);
      std::fill(flags.begin() + pc.b0, flags.begin() + pc.b0 + pc.cnt, pc.r->flag);
    }
    plan_krige(p, nq, ql.data(), owner.data(), flags.data(), 0, plan);
    const size_t ni = plan.items.size();
    const InLayout L = in_layout(nq, (int64_t)ni);
    std::memcpy(sl.h_in, plan.qx.data(), 8 * (size_t)nq);
    std::memcpy(sl.h_in + L.qy, plan.qy.data(), 8 * (size_t)nq);
    std::memcpy(sl.h_in + L.qorig, plan.qorig.data(), 4 * (size_t)nq);
    std::memcpy(sl.h_in + L.qflag, plan.qflag.data(), 4 * (size_t)nq);
    std::memcpy(sl.h_in + L.items, plan.items.data(), sizeof(KrigeItem) * ni);
    sl.h_mean = sl.h_out;
    sl.h_var = sl.h_out + nq;
    hipError_t e = hipSuccess;
    hipStream_t st = sl.stream;
    if (e == hipSuccess) e = hipMemcpyAsync(sl.d_in, sl.h_in, L.bytes, hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
      e = launch_krige(st, p->d_desc_fact, p->d_theta_fact, reinterpret_cast<const KrigeItem*>(sl.d_in + L.items),
                       (int)ni, p->d_tx, p->d_ty, p->d_Lf, p->d_Invf, p->d_alpha_fact,
                       reinterpret_cast<const double*>(sl.d_in), reinterpret_cast<const double*>(sl.d_in + L.qy),
                       reinterpret_cast<const int32_t*>(sl.d_in + L.qorig),
                       reinterpret_cast<const int32_t*>(sl.d_in + L.qflag), sl.d_W, sl.d_out, sl.d_out + nq);
    if (e == hipSuccess)
      e = hipMemcpyAsync(sl.h_out, sl.d_out, (sl.any_var ? 16 : 8) * (size_t)nq, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipEventRecord(sl.done, st);
    sl.err = e;
    {
      std::lock_guard<std::mutex> lk(s->mu);
      ++s->n_batches;
      s->batch_queries += nq;
      s->launched.push_back(si);
    }
    s->cv_comp.notify_one();
  }
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->launched.push_back(-1);  // end marker for the completion thread
  }
  s->cv_comp.notify_one();
}

void completer(pcv_server* s) {
  (void)hipSetDevice(s->p->device);
  for (;;) {
    int si;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_comp.wait(lk, [&] { return !s->launched.empty(); });
      si = s->launched.front();
      s->launched.pop_front();
    }
    if (si < 0) break;
    Slot& sl = s->slots[si];
    hipError_t e = sl.err;
    if (e == hipSuccess) e = hipEventSynchronize(sl.done);
    // a request is only read or written here while it has pieces in flight,
    // and it cannot finish (and be collected) before its last piece is back
    if (e == hipSuccess)
      for (const Piece& pc : sl.pieces) {
        if (pc.r->failed) continue;
        std::copy(sl.h_mean + pc.b0, sl.h_mean + pc.b0 + pc.cnt, pc.r->mean + pc.r0);
        if (pc.r->var) std::copy(sl.h_var + pc.b0, sl.h_var + pc.b0 + pc.cnt, pc.r->var + pc.r0);
      }
    std::lock_guard<std::mutex> lk(s->mu);
    for (const Piece& pc : sl.pieces) {
      Req* r = pc.r;
      r->done += pc.cnt;
      if (e != hipSuccess && !r->failed) {
        // drop the request's queries that are still queued
        r->failed = true;
        r->err = std::string("kriging batch: ") + hipGetErrorString(e);
        (void)hipGetLastError();
        if (r->next < r->q) {
          s->queued_q -= r->q - r->next;
          r->next = r->q = std::max(r->next, r->done);
          s->pred_q.erase(std::remove(s->pred_q.begin(), s->pred_q.end(), r), s->pred_q.end());
        }
      }
      if (!r->finished && r->done == r->next && r->next == r->q)
        finish_locked(s, r, r->failed ? PCV_ERR_DEVICE : PCV_OK, r->err);
    }
    sl.pieces.clear();
    s->free_slots.push_back(si);
    s->cv_batch.notify_one();
  }
}

// Evaluations queued together run as one batch (several theta values per
// launch when the workspace allows; results identical to one at a time).
void evaluator(pcv_server* s) {
  (void)hipSetDevice(s->p->device);
  std::vector<Req*> batch;
  std::vector<pcv_theta> th;
  std::vector<double> loss;
  for (;;) {
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_eval.wait(lk, [&] { return s->stop || !s->eval_q.empty(); });
      if (s->eval_q.empty()) break;  // stop requested and nothing left
      batch.clear();
      while (!s->eval_q.empty() && batch.size() < 64) {
        batch.push_back(s->eval_q.front());
        s->eval_q.pop_front();
      }
      s->eval_busy = true;
    }
    th.resize(batch.size());
    loss.assign(batch.size(), 0.0);
    for (size_t k = 0; k < batch.size(); ++k) th[k] = batch[k]->th;
    g_err.clear();
    pcv_status st = eval_batch_impl(s->p, (int32_t)batch.size(), th.data(), loss.data(), nullptr);
    std::vector<pcv_status> sts(batch.size(), st);
    std::vector<std::string> errs(batch.size(), st == PCV_OK ? "" : g_err);
    if (st != PCV_OK && batch.size() > 1) {
      // find which ones fail: evaluate them one by one
      for (size_t k = 0; k < batch.size(); ++k) {
        g_err.clear();
        sts[k] = eval_impl(s->p, th[k], &loss[k], nullptr);
        errs[k] = sts[k] == PCV_OK ? "" : g_err;
      }
    }
    for (size_t k = 0; k < batch.size(); ++k)
      if (sts[k] == PCV_OK) *batch[k]->loss = loss[k];
    {
      std::lock_guard<std::mutex> lk(s->mu);
      for (size_t k = 0; k < batch.size(); ++k) finish_locked(s, batch[k], sts[k], errs[k]);
      s->eval_busy = false;
    }
    s->cv_batch.notify_one();  // kriging need not wait for the window any more
  }
}

double pct(std::vector<double> v, double f) {
  if (v.empty()) return 0.0;
  std::sort(v.begin(), v.end());
  // nearest-rank percentile
  size_t k = (size_t)std::ceil(f * (double)v.size());
  k = std::min(std::max<size_t>(k, 1), v.size());
  return v[k - 1];
}

void free_slots_mem(pcv_server* s) {
  for (Slot& sl : s->slots) {
    for (void* d : {(void*)sl.d_in, (void*)sl.d_out, (void*)sl.d_W})
      if (d) (void)hipFree(d);
    for (void* h : {(void*)sl.h_in, (void*)sl.h_out})
      if (h) (void)hipHostFree(h);
    if (sl.done) (void)hipEventDestroy(sl.done);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
  }
  s->slots.clear();
  if (s->eval_stream) {
    (void)hipStreamSynchronize(s->eval_stream);
    if (s->saved_stream) s->p->stream = s->saved_stream;
    (void)hipStreamDestroy(s->eval_stream);
    s->eval_stream = nullptr;
  }
}

}  // namespace

pcv_status server_create(pcv_server** out, pcv_problem* p, size_t mem_budget, int32_t max_inflight,
                         int32_t n_slots) {
  hipError_t e = hipSetDevice(p->device);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(PCV_ERR_DEVICE, hipGetErrorString(e));
  }
  // evaluations of a served problem stay on its one stream
  pcv_status st0 = set_served(p, true);
  if (st0 != PCV_OK) return st0;
  pcv_server* s = new pcv_server();
  s->p = p;
  s->max_inflight = max_inflight;
  if (mem_budget == 0) mem_budget = (size_t)8 << 30;
  // Per slot: 40 bytes per query (coordinates, mean, variance, index, flags)
  // and, per item of up to KRIGE_Q queries, a KrigeItem and an
  // npad x KRIGE_Q variance panel.
  // (signed: a budget below the query buffers leaves no room for items)
  const int64_t per_slot = (int64_t)std::min<size_t>(mem_budget / (size_t)n_slots, (size_t)1 << 60);
  const int64_t w_item = (int64_t)std::max(p->max_npad, (int32_t)pcv::TB) * KRIGE_Q;
  s->q_cap = std::max<int64_t>(64, std::min<int64_t>(1 << 20, per_slot / 4 / 40));
  s->w_cap = std::max<int64_t>(0, per_slot - s->q_cap * 40) / 8;
  s->item_cap = s->w_cap / w_item;
  if (s->item_cap < 1) {
    delete s;
    (void)set_served(p, false);
    return fail(PCV_ERR_INVALID, "mem_budget too small for one kriging item per slot (need " +
                                     std::to_string((w_item * 8 + 64 * 40 * 4) * n_slots) + " bytes)");
  }
  e = hipStreamCreateWithFlags(&s->eval_stream, hipStreamNonBlocking);
  if (e != hipSuccess) {
    delete s;
    (void)set_served(p, false);
    (void)hipGetLastError();
    return fail(PCV_ERR_DEVICE, std::string("server stream: ") + hipGetErrorString(e));
  }
  s->slots.resize(n_slots);
  for (Slot& sl : s->slots) {
    const int64_t Q = s->q_cap, I = s->item_cap;
    e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
    const size_t in_cap = in_layout(Q, I).bytes;
    if (e == hipSuccess) e = hipMalloc((void**)&sl.d_in, in_cap);
    if (e == hipSuccess) e = hipMalloc((void**)&sl.d_out, 16 * Q);
    if (e == hipSuccess) e = hipMalloc((void**)&sl.d_W, 8 * s->w_cap);
    if (e == hipSuccess) e = hipHostMalloc((void**)&sl.h_in, in_cap, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void**)&sl.h_out, 16 * Q, hipHostMallocDefault);
    if (e != hipSuccess) break;
    s->ws_bytes += (size_t)Q * 40 + sizeof(KrigeItem) * I + 8 * (size_t)s->w_cap;
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();  // a failed allocation must not surface at a later launch
    free_slots_mem(s);
    delete s;
    (void)set_served(p, false);
    return fail(e == hipErrorOutOfMemory ? PCV_ERR_OOM : PCV_ERR_DEVICE,
                std::string("server workspace: ") + hipGetErrorString(e));
  }
  for (int i = 0; i < n_slots; ++i) s->free_slots.push_back(i);
  s->saved_stream = p->stream;
  p->stream = s->eval_stream;
  s->th_batch = std::thread(batcher, s);
  s->th_comp = std::thread(completer, s);
  s->th_eval = std::thread(evaluator, s);
  *out = s;
  return PCV_OK;
}

namespace {

// Block until an in-flight place is free, then register the request.
pcv_ticket admit(pcv_server* s, Req* r, std::unique_lock<std::mutex>& lk) {
  if (s->inflight >= s->max_inflight) {
    ++s->admission_waits;
    s->cv_admit.wait(lk, [&] { return s->inflight < s->max_inflight; });
  }
  r->id = s->next_id++;
  r->t_submit = now_s();
  if (s->t_first < 0) s->t_first = r->t_submit;
  s->reqs[r->id] = r;
  ++s->inflight;
  return r->id;
}

}  // namespace

pcv_status server_submit_predict(pcv_server* s, int64_t q, const double* ql, double* mean, double* var,
                                 int32_t obs_noise, pcv_ticket* ticket) {
  Req* r = new Req();
  r->kind = REQ_PREDICT;
  r->q = q;
  r->ql = ql;
  r->mean = mean;
  r->var = var;
  r->flag = (var ? KRIGE_VAR : 0) | (obs_noise ? KRIGE_OBS_NOISE : 0);
  r->owner.resize(q);
  route(s->p, q, ql, r->owner.data());  // in the caller's thread
  std::unique_lock<std::mutex> lk(s->mu);
  *ticket = admit(s, r, lk);
  if (q == 0) {
    finish_locked(s, r, PCV_OK, "");
    return PCV_OK;
  }
  s->pred_q.push_back(r);
  s->queued_q += q;
  s->cv_batch.notify_one();
  return PCV_OK;
}

pcv_status server_set_window(pcv_server* s, double seconds) {
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->window_s = seconds;
  }
  s->cv_batch.notify_one();
  return PCV_OK;
}

pcv_status server_submit_eval(pcv_server* s, const pcv_theta& th, double* loss, pcv_ticket* ticket) {
  Req* r = new Req();
  r->kind = REQ_EVAL;
  r->th = th;
  r->loss = loss;
  std::unique_lock<std::mutex> lk(s->mu);
  *ticket = admit(s, r, lk);
  s->eval_q.push_back(r);
  s->cv_eval.notify_one();
  return PCV_OK;
}

pcv_status server_wait(pcv_server* s, pcv_ticket t, double timeout_s) {
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->reqs.find(t);
  if (it == s->reqs.end()) return fail(PCV_ERR_INVALID, "unknown or already collected ticket");
  Req* r = it->second;
  auto ready = [&] { return r->finished; };
  if (timeout_s < 0) {
    s->cv_done.wait(lk, ready);
  } else if (!s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), ready)) {
    return fail(PCV_ERR_BUSY, "request not finished within the timeout");
  }
  const pcv_status st = r->st;
  const std::string err = r->err;
  s->reqs.erase(it);
  delete r;
  if (st != PCV_OK) return fail(st, err);
  return PCV_OK;
}

pcv_status server_report(pcv_server* s, pcv_server_report* o) {
  std::lock_guard<std::mutex> lk(s->mu);
  o->n_predict = (int64_t)s->lat_pred.size();
  o->n_eval = (int64_t)s->lat_eval.size();
  o->n_queries = s->n_queries;
  o->n_batches = s->n_batches;
  o->mean_batch_queries = s->n_batches ? (double)s->batch_queries / (double)s->n_batches : 0.0;
  o->p50_s = pct(s->lat_pred, 0.50);
  o->p99_s = pct(s->lat_pred, 0.99);
  o->max_s = pct(s->lat_pred, 1.0);
  o->eval_p50_s = pct(s->lat_eval, 0.50);
  o->eval_p99_s = pct(s->lat_eval, 0.99);
  o->elapsed_s = s->t_first < 0 ? 0.0 : std::max(0.0, s->t_last - s->t_first);
  o->qps = o->elapsed_s > 0 ? (double)s->n_queries / o->elapsed_s : 0.0;
  o->evals_per_s = o->elapsed_s > 0 ? (double)o->n_eval / o->elapsed_s : 0.0;
  o->admission_waits = s->admission_waits;
  o->workspace_bytes = (int64_t)s->ws_bytes;
  o->batch_query_cap = s->q_cap;
  o->batch_item_cap = s->item_cap;
  return PCV_OK;
}

const pcv_problem* server_problem(const pcv_server* s) { return s->p; }

pcv_status server_destroy(pcv_server* s) {
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_batch.notify_all();
  s->cv_eval.notify_all();
  // the batcher drains its queue before it stops; the completer follows it
  s->th_batch.join();
  s->th_comp.join();
  s->th_eval.join();
  for (auto& kv : s->reqs) delete kv.second;
  s->reqs.clear();
  free_slots_mem(s);
  pcv_problem* p = s->p;
  delete s;
  return set_served(p, false);
}

}  // namespace pcv
