// Problem residency and the evaluation / factorisation / prediction
// sequences behind the C ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "pcv_host.h"

using pcv::fail;
using pcv::SubsetDesc;
using pcv::TB;

#define HIPCHK(x)                                                                          \
  do {                                                                                     \
    hipError_t e_ = (x);                                                                   \
    if (e_ != hipSuccess) {                                                                \
      (void)hipGetLastError(); /* reported here, not again at a later launch */            \
      return fail(e_ == hipErrorOutOfMemory ? PCV_ERR_OOM : PCV_ERR_DEVICE,                \
                  std::string(#x) + ": " + hipGetErrorString(e_));                         \
    }                                                                                      \
  } while (0)

namespace pcv {
namespace {

template <typename T>
pcv_status dalloc(pcv_problem* p, T** ptr, size_t count) {
  *ptr = nullptr;
  if (count == 0) count = 1;
  const size_t bytes = count * sizeof(T);
  if (p->opt.mem_cap_bytes && p->dev_bytes + bytes > p->opt.mem_cap_bytes)
    return fail(PCV_ERR_OOM, "device memory cap exceeded (" + std::to_string(p->dev_bytes + bytes) +
                                 " > " + std::to_string(p->opt.mem_cap_bytes) + " bytes)");
  hipError_t e = hipMalloc((void**)ptr, bytes);
  if (e != hipSuccess) {
    *ptr = nullptr;
    (void)hipGetLastError();
    return fail(e == hipErrorOutOfMemory ? PCV_ERR_OOM : PCV_ERR_DEVICE,
                std::string("hipMalloc(") + std::to_string(bytes) + "): " + hipGetErrorString(e));
  }
  p->dev_bytes += bytes;
  p->allocs.push_back((void*)*ptr);
  return PCV_OK;
}

template <typename T>
pcv_status upload(pcv_problem* p, T** dst, const std::vector<T>& src) {
  pcv_status s = dalloc(p, dst, src.size());
  if (s != PCV_OK) return s;
  if (!src.empty()) HIPCHK(hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
  return PCV_OK;
}

void dfree(pcv_problem* p, void* ptr, size_t bytes) {
  if (!ptr) return;
  (void)hipFree(ptr);
  p->allocs.erase(std::remove(p->allocs.begin(), p->allocs.end(), ptr), p->allocs.end());
  p->dev_bytes -= bytes;
}
// Free what dalloc(p, &ptr, count) allocated (its byte count) and clear ptr.
template <typename T>
void dfree_n(pcv_problem* p, T*& ptr, size_t count) {
  dfree(p, (void*)ptr, std::max<size_t>(count, 1) * sizeof(T));
  ptr = nullptr;
}

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Fill the pinned theta block; the evaluation sequence uploads it.
void set_theta_host(pcv_problem* p, const pcv_theta& th) {
  ThetaDev* h = p->h_theta;
  h->cov = th.cov;
  h->pad = 0;
  h->range = th.range;
  h->inv_range = 1.0 / th.range;
  h->lambda = th.lambda;
  h->sigma2 = th.sigma2;
}

pcv_status ensure_L(pcv_problem* p, bool fp64) {
  if (fp64 && !p->d_L64) return dalloc(p, &p->d_L64, (size_t)p->nL);
  if (!fp64 && !p->d_L32) return dalloc(p, &p->d_L32, (size_t)p->nL);
  return PCV_OK;
}

// Largest n^3 first (longest-processing-time order), ties by index.
std::vector<int32_t> lpt_order(const std::vector<SubsetDesc>& d, const std::vector<int32_t>& ids) {
  std::vector<int32_t> o = ids;
  std::stable_sort(o.begin(), o.end(), [&](int32_t a, int32_t b) { return d[a].npad > d[b].npad; });
  return o;
}

// The schedule groups of an evaluation: whole rounds of one work-group per
// compute unit over the largest subsets, then the remainder (when the
// two-group schedule is on and applies), else one group.  A subset is
// factored with the shape its group's largest subset selects, whatever
// launches the group is split into, so its factor carries the same bits in
// pcv_eval, in a served evaluation and in the multi-theta launches.
int n_sched(const pcv_problem* p) {
  return p->tune_two_groups && p->groups.size() > 1 ? (int)p->groups.size() : 1;
}
const pcv_group& sched(const pcv_problem* p, int k) { return n_sched(p) > 1 ? p->groups[k] : p->g_all; }
int32_t sched_npad(const pcv_problem* p, int k) {
  const pcv_group& G = sched(p, k);
  return G.cnt > 0 ? p->desc[p->order_eval[G.o0]].npad : 0;
}

// Work-groups per subset in the first factorisation launch.  With one
// work-group per subset the launch lasts at least as long as its largest
// factorisation; a subset whose cost (npad^3) exceeds the launch's average
// cost per compute unit is shared by round(cost / average) work-groups (at
// least 2, at most max_wg_per_subset), largest first, while the shared
// blocks fit one per compute unit.  Sharing pays only with several 256-row
// chunks per panel, hence the size floor.
constexpr int32_t COOP_MIN_NPAD = 2048;

}  // namespace

void plan_coop(pcv_problem* p) {
  const pcv_group& G0 = sched(p, 0);
  p->coop_group_cnt = G0.cnt;
  p->coop_blocks = p->coop_slots = 0;
  p->coop_order.clear();
  p->coop_info.clear();
  const int maxwg = p->opt.max_wg_per_subset ? p->opt.max_wg_per_subset : 8;
  if (maxwg < 2 || p->n_cu < 2 || G0.cnt <= 0) return;
  double tot = 0.0;
  for (int32_t k = 0; k < G0.cnt; ++k) tot += std::pow((double)p->desc[p->order_eval[G0.o0 + k]].npad, 3);
  const double avg = tot / p->n_cu;
  std::vector<int32_t> order, info;
  int32_t used = 0, slots = 0, k = 0;
  for (; k < G0.cnt; ++k) {
    const int32_t i = p->order_eval[G0.o0 + k];
    const double c = std::pow((double)p->desc[i].npad, 3);
    if (p->desc[i].npad < COOP_MIN_NPAD || c <= avg) break;
    const int32_t nwg = std::min<int32_t>(maxwg, std::max<int32_t>(2, (int32_t)std::lround(c / avg)));
    if (used + nwg > p->n_cu) break;
    for (int32_t r = 0; r < nwg; ++r) {
      order.push_back(i);
      info.push_back(r | nwg << 8 | slots << 16);
    }
    used += nwg;
    ++slots;
  }
  if (slots == 0) return;
  for (; k < G0.cnt; ++k) order.push_back(p->order_eval[G0.o0 + k]);
  p->coop_blocks = used;
  p->coop_slots = slots;
  p->coop_order = std::move(order);
  p->coop_info = std::move(info);
}

namespace {

// Bucket grid over the core rectangles: G x G buckets spanning the domain,
// each listing the cores that touch it.
void build_router(pcv_problem* p) {
  const int S = p->S;
  pcv_router& R = p->router;
  const double* C = p->core_rect.data();
  R.xmax = R.ymax = -INFINITY;
  R.xmin = R.ymin = INFINITY;
  for (int i = 0; i < S; ++i) {
    R.xmin = std::min(R.xmin, C[4 * i + 0]);
    R.ymin = std::min(R.ymin, C[4 * i + 1]);
    R.xmax = std::max(R.xmax, C[4 * i + 2]);
    R.ymax = std::max(R.ymax, C[4 * i + 3]);
  }
  R.G = std::max(1, std::min(512, (int)std::sqrt((double)S) * 2));
  R.bw = (R.xmax - R.xmin) / R.G;
  R.bh = (R.ymax - R.ymin) / R.G;
  const int G = R.G;
  auto bx = [&](double x) { return std::min(G - 1, std::max(0, (int)std::floor((x - R.xmin) / R.bw))); };
  auto by = [&](double y) { return std::min(G - 1, std::max(0, (int)std::floor((y - R.ymin) / R.bh))); };
  std::vector<std::vector<int32_t>> buckets((size_t)G * G);
  if (R.bw > 0 && R.bh > 0)
    for (int i = 0; i < S; ++i) {
      const int x0 = bx(C[4 * i]), x1 = bx(C[4 * i + 2]), y0 = by(C[4 * i + 1]), y1 = by(C[4 * i + 3]);
      for (int yy = y0; yy <= y1; ++yy)
        for (int xx = x0; xx <= x1; ++xx) buckets[(size_t)yy * G + xx].push_back(i);
    }
  R.ptr.assign((size_t)G * G + 1, 0);
  for (size_t b = 0; b < buckets.size(); ++b) R.ptr[b + 1] = R.ptr[b] + (int32_t)buckets[b].size();
  R.list.clear();
  for (auto& v : buckets) R.list.insert(R.list.end(), v.begin(), v.end());
}

}  // namespace

// Route queries to cores: half-open [lo, hi) per axis, edges on the domain
// maximum closed, lowest index first; a point in no core goes to the
// nearest core rectangle (lowest index on ties).  Without rectangles: the
// nearest training centroid.
void route(const pcv_problem* p, int64_t q, const double* ql, int32_t* owner) {
  const int S = p->S;
  if (!p->core_rect.empty()) {
    const double* C = p->core_rect.data();
    const pcv_router& R = p->router;
    const int G = R.G;
    for (int64_t j = 0; j < q; ++j) {
      const double x = ql[2 * j], y = ql[2 * j + 1];
      int hit = -1;
      if (x >= R.xmin && x <= R.xmax && y >= R.ymin && y <= R.ymax && R.bw > 0 && R.bh > 0) {
        const int bxi = std::min(G - 1, std::max(0, (int)std::floor((x - R.xmin) / R.bw)));
        const int byi = std::min(G - 1, std::max(0, (int)std::floor((y - R.ymin) / R.bh)));
        const size_t b = (size_t)byi * G + bxi;
        for (int32_t k = R.ptr[b]; k < R.ptr[b + 1]; ++k) {
          const int32_t i = R.list[k];
          const double* r = C + 4 * i;
          const bool inx = x >= r[0] && (x < r[2] || (x == r[2] && r[2] == R.xmax));
          const bool iny = y >= r[1] && (y < r[3] || (y == r[3] && r[3] == R.ymax));
          if (inx && iny && (hit < 0 || i < hit)) hit = i;
        }
      }
      if (hit < 0) {
        double best = INFINITY;
        for (int i = 0; i < S; ++i) {
          const double* r = C + 4 * i;
          const double dx = std::max(std::max(r[0] - x, 0.0), x - r[2]);
          const double dy = std::max(std::max(r[1] - y, 0.0), y - r[3]);
          const double d2 = dx * dx + dy * dy;
          if (d2 < best) {
            best = d2;
            hit = i;
          }
        }
      }
      owner[j] = hit;
    }
  } else {
    for (int64_t j = 0; j < q; ++j) {
      double best = INFINITY;
      int hit = 0;
      for (int i = 0; i < S; ++i) {
        if (p->desc[i].n == 0) continue;
        const double dx = ql[2 * j] - p->centroid[2 * i], dy = ql[2 * j + 1] - p->centroid[2 * i + 1];
        const double d2 = dx * dx + dy * dy;
        if (d2 < best) {
          best = d2;
          hit = i;
        }
      }
      owner[j] = hit;
    }
  }
}

void plan_krige(const pcv_problem* p, int64_t q, const double* ql, const int32_t* owner,
                const int32_t* flags, int32_t flag_all, KrigePlan& P) {
  const int S = p->S;
  P.qx.resize(q);
  P.qy.resize(q);
  P.qorig.resize(q);
  P.qflag.resize(q);
  P.items.clear();
  P.w_doubles = 0;
  // counting sort by owner keeps the input order inside a subset
  P.cnt.assign(S + 1, 0);
  for (int64_t j = 0; j < q; ++j) ++P.cnt[owner[j] + 1];
  for (int i = 0; i < S; ++i) P.cnt[i + 1] += P.cnt[i];
  P.pos.assign(P.cnt.begin(), P.cnt.end() - 1);
  for (int64_t j = 0; j < q; ++j) {
    const int32_t i = owner[j];
    const int64_t k = P.pos[i]++;
    P.qx[k] = ql[2 * j] - p->centroid[2 * i];
    P.qy[k] = ql[2 * j + 1] - p->centroid[2 * i + 1];
    P.qorig[k] = (int32_t)j;
    P.qflag[k] = flags ? flags[j] : flag_all;
  }
  for (int i = 0; i < S; ++i)
    for (int64_t k = P.cnt[i]; k < P.cnt[i + 1]; k += KRIGE_Q) {
      KrigeItem it;
      it.sidx = i;
      it.q0 = (int32_t)k;
      it.nq = (int32_t)std::min<int64_t>(KRIGE_Q, P.cnt[i + 1] - k);
      it.flags = 0;
      for (int64_t m = k; m < k + it.nq; ++m) it.flags |= P.qflag[m] & KRIGE_VAR;
      it.woff = 0;
      if (it.flags & KRIGE_VAR) {
        it.woff = P.w_doubles;
        P.w_doubles += (int64_t)p->desc[i].npad * KRIGE_Q;
      }
      P.items.push_back(it);
    }
}

namespace {
// Device copies of the sharing plan (its blocks, their ranks and counters).
pcv_status upload_coop(pcv_problem* p) {
  if (p->coop_slots <= 0) return PCV_OK;
  pcv_status s = upload(p, &p->d_coop_order, p->coop_order);
  if (s == PCV_OK) s = upload(p, &p->d_coop_info, p->coop_info);
  if (s == PCV_OK) s = dalloc(p, &p->d_coop_sync, (size_t)4 * p->coop_slots);
  return s;
}
void free_coop(pcv_problem* p) {
  dfree(p, p->d_coop_order, sizeof(int32_t) * std::max<size_t>(1, p->coop_order.size()));
  dfree(p, p->d_coop_info, sizeof(int32_t) * std::max<size_t>(1, p->coop_info.size()));
  dfree(p, p->d_coop_sync, sizeof(int32_t) * std::max<size_t>(1, (size_t)4 * p->coop_slots));
  p->d_coop_order = p->d_coop_info = p->d_coop_sync = nullptr;
}
}  // namespace

pcv_status problem_build(pcv_problem* p, int64_t n, const double* locs, const double* y, int32_t S,
                         const int64_t* tptr, const int32_t* tidx, const int64_t* vptr,
                         const int32_t* vidx, const double* core_rect) {
  HIPCHK(hipGetDevice(&p->device));
  if (p->opt.hip_stream) {
    p->stream = (hipStream_t)p->opt.hip_stream;
    p->own_stream = false;
  } else {
    HIPCHK(hipStreamCreateWithFlags(&p->stream, hipStreamNonBlocking));
    p->own_stream = true;
  }
  p->n = n;
  p->S = S;
  p->desc.resize(S);
  p->active.assign(S, 0);
  p->centroid.assign(2 * (size_t)S, 0.0);
  p->ynorm2.assign(S, 0.0);
  if (core_rect) {
    p->core_rect.assign(core_rect, core_rect + 4 * (size_t)S);
    build_router(p);
  }
  p->train_ptr.assign(tptr, tptr + S + 1);
  p->train_idx.assign(tidx, tidx + tptr[S]);

  int64_t offT = 0, offV = 0, offP = 0, offL = 0, offInv = 0, offPC = 0;
  std::vector<int32_t> act_ids, all_ids;
  for (int32_t i = 0; i < S; ++i) {
    SubsetDesc& d = p->desc[i];
    d.n = (int32_t)(tptr[i + 1] - tptr[i]);
    d.m = (int32_t)(vptr[i + 1] - vptr[i]);
    // at least one padding row: the first one carries y_T through the
    // factorisation (the forward substitution, see launch_potrf_*)
    d.npad = d.n > 0 ? (d.n / TB + 1) * TB : 0;
    d.th = 0;
    d.offT = offT;
    d.offV = offV;
    d.offP = offP;
    d.offL = offL;
    d.offInv = offInv;
    d.offPC = offPC;
    d.offX = offP;
    d.offE = offV;
    offT += d.n;
    offV += d.m;
    offP += d.npad;
    offL += packed_size(d.npad);
    offInv += (int64_t)d.npad * TB;
    {
      const int64_t nbk = d.npad / TB;
      offPC += (int64_t)TB * nbk * (nbk - 1) / 2;
    }
    p->max_train = std::max(p->max_train, d.n);
    p->max_npad = std::max(p->max_npad, d.npad);
    if (d.m > 0) {
      p->active[i] = 1;
      act_ids.push_back(i);
      p->n_val_total += d.m;
    }
    if (d.n > 0) all_ids.push_back(i);
  }
  p->nnzT = offT;
  p->nnzV = offV;
  p->nP = offP;
  p->nL = offL;
  p->nInv = offInv;
  p->nPC = offPC;
  p->n_active = (int32_t)act_ids.size();
  p->order_eval = lpt_order(p->desc, act_ids);
  p->order_all = lpt_order(p->desc, all_ids);
  // schedule groups: whole rounds of the largest subsets, then the rest
  int n_cu = 0;
  HIPCHK(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, p->device));
  p->n_cu = n_cu;
  std::vector<int32_t> bounds{0};
  if (n_cu > 0 && p->n_active > n_cu && p->n_active % n_cu != 0) {
    bounds.push_back(p->n_active / n_cu * n_cu);
  }
  bounds.push_back(p->n_active);
  for (size_t g = 0; g + 1 < bounds.size(); ++g) {
    pcv_group G;
    G.o0 = bounds[g];
    G.cnt = bounds[g + 1] - bounds[g];
    G.r0 = (int32_t)p->row_items_eval.size();
    G.v0 = (int32_t)p->val_items.size();
    for (int32_t k = G.o0; k < G.o0 + G.cnt; ++k) {
      const int32_t i = p->order_eval[k];
      for (int rb = 0; rb < p->desc[i].npad / TB; ++rb) p->row_items_eval.push_back(make_int2(i, rb));
      for (int vb = 0; vb < (p->desc[i].m + 63) / 64; ++vb) p->val_items.push_back(make_int2(i, vb));
    }
    G.nr = (int32_t)p->row_items_eval.size() - G.r0;
    G.nv = (int32_t)p->val_items.size() - G.v0;
    p->groups.push_back(G);
  }
  p->g_all.cnt = p->n_active;
  p->g_all.nr = (int32_t)p->row_items_eval.size();
  p->g_all.nv = (int32_t)p->val_items.size();
  plan_coop(p);
  // residual tiles: within each group, largest row block first
  p->tile_items = p->row_items_eval;
  for (const pcv_group& G : p->groups)
    std::stable_sort(p->tile_items.begin() + G.r0, p->tile_items.begin() + G.r0 + G.nr,
                     [](const int2& a, const int2& b) { return a.y > b.y; });

  // per-subset panels, centred on the subset's training centroid (FP64)
  std::vector<double> tx(offT), ty(offT), yT(offT), vx(offV), vy(offV), yV(offV);
  std::vector<double> px64(offP, INFINITY), py64(offP, INFINITY);
  std::vector<float> px32(offP, INFINITY), py32(offP, INFINITY);
  std::vector<double> pv64(offP, 0.0);  // y_T in the padded layout
  std::vector<float> pv32(offP, 0.0f);
  for (int32_t i = 0; i < S; ++i) {
    const SubsetDesc& d = p->desc[i];
    double cx = 0.0, cy = 0.0;
    if (d.n > 0) {
      for (int64_t j = tptr[i]; j < tptr[i + 1]; ++j) {
        cx += locs[2 * (int64_t)tidx[j]];
        cy += locs[2 * (int64_t)tidx[j] + 1];
      }
      cx /= d.n;
      cy /= d.n;
    } else if (d.m > 0) {
      for (int64_t j = vptr[i]; j < vptr[i + 1]; ++j) {
        cx += locs[2 * (int64_t)vidx[j]];
        cy += locs[2 * (int64_t)vidx[j] + 1];
      }
      cx /= d.m;
      cy /= d.m;
    }
    p->centroid[2 * i] = cx;
    p->centroid[2 * i + 1] = cy;
    double y2 = 0.0;
    for (int64_t j = tptr[i], a = 0; j < tptr[i + 1]; ++j, ++a) {
      const int64_t g = tidx[j];
      tx[d.offT + a] = locs[2 * g] - cx;
      ty[d.offT + a] = locs[2 * g + 1] - cy;
      px64[d.offP + a] = tx[d.offT + a];
      py64[d.offP + a] = ty[d.offT + a];
      px32[d.offP + a] = (float)tx[d.offT + a];
      py32[d.offP + a] = (float)ty[d.offT + a];
      yT[d.offT + a] = y[g];
      pv64[d.offP + a] = y[g];
      pv32[d.offP + a] = (float)y[g];
      y2 += y[g] * y[g];
    }
    p->ynorm2[i] = y2;
    for (int64_t j = vptr[i], a = 0; j < vptr[i + 1]; ++j, ++a) {
      const int64_t g = vidx[j];
      vx[d.offV + a] = locs[2 * g] - cx;
      vy[d.offV + a] = locs[2 * g + 1] - cy;
      yV[d.offV + a] = y[g];
    }
  }

  pcv_status s;
#define TRY(x)              \
  do {                      \
    s = (x);                \
    if (s != PCV_OK) return s; \
  } while (0)
  TRY(upload(p, &p->d_desc, p->desc));
  TRY(upload(p, &p->d_order_eval, p->order_eval));
  TRY(upload(p, &p->d_order_all, p->order_all));
  TRY(upload_coop(p));
  TRY(upload(p, &p->d_active, p->active));
  TRY(upload(p, &p->d_row_items, p->row_items_eval));
  TRY(upload(p, &p->d_tile_items, p->tile_items));
  TRY(upload(p, &p->d_val_items, p->val_items));
  TRY(upload(p, &p->d_tx, tx));
  TRY(upload(p, &p->d_ty, ty));
  TRY(upload(p, &p->d_yT, yT));
  TRY(upload(p, &p->d_px32, px32));
  TRY(upload(p, &p->d_py32, py32));
  TRY(upload(p, &p->d_pv64, pv64));
  TRY(upload(p, &p->d_pv32, pv32));
  TRY(upload(p, &p->d_px64, px64));
  TRY(upload(p, &p->d_py64, py64));
  TRY(upload(p, &p->d_vx, vx));
  TRY(upload(p, &p->d_vy, vy));
  TRY(upload(p, &p->d_yV, yV));
  TRY(upload(p, &p->d_ynorm2, p->ynorm2));
  TRY(dalloc(p, &p->d_z, (size_t)p->nP));
  TRY(dalloc(p, &p->d_x, (size_t)p->nP));
  TRY(dalloc(p, &p->d_alpha, (size_t)p->nP));
  TRY(dalloc(p, &p->d_r, (size_t)p->nP));
  TRY(dalloc(p, &p->d_rrow, (size_t)p->nP));
  TRY(dalloc(p, &p->d_pcol, (size_t)std::max<int64_t>(p->nPC, 1)));
  TRY(dalloc(p, &p->d_rhs2, (size_t)S));
  TRY(dalloc(p, &p->d_yhat, (size_t)p->nnzV));
  TRY(dalloc(p, &p->d_err, (size_t)p->nnzV));
  TRY(dalloc(p, &p->d_logdet, (size_t)S));
  TRY(dalloc(p, &p->d_sspe, (size_t)S));
  TRY(dalloc(p, &p->d_quad, (size_t)S));
  TRY(dalloc(p, &p->d_status, (size_t)S));
  TRY(dalloc(p, &p->d_bad, (size_t)S));
  TRY(dalloc(p, &p->d_gate, (size_t)S));
  TRY(dalloc(p, &p->d_nsweep, (size_t)S));
  TRY(dalloc(p, &p->d_theta, 1));
  TRY(dalloc(p, &p->d_total, 1));
  TRY(dalloc(p, &p->d_nbad, 1));
  TRY(dalloc(p, &p->d_Inv, (size_t)p->nInv));
#undef TRY
  HIPCHK(hipMemset(p->d_status, 0, sizeof(int32_t) * S));
  HIPCHK(hipMemset(p->d_logdet, 0, sizeof(double) * S));
  HIPCHK(hipHostMalloc((void**)&p->h_theta, sizeof(ThetaDev), hipHostMallocDefault));
  HIPCHK(hipHostMalloc((void**)&p->h_total, sizeof(double), hipHostMallocDefault));
  HIPCHK(hipHostMalloc((void**)&p->h_nbad, sizeof(int32_t), hipHostMallocDefault));
  if (p->opt.profile) {
    for (auto& e : p->ev) HIPCHK(hipEventCreate(&e));
    p->events = true;
  }
  return PCV_OK;
}

namespace {

void drop_post_streams(pcv_problem* p) {
  for (hipEvent_t e : p->ev_fact)
    if (e) (void)hipEventDestroy(e);
  p->ev_fact.clear();
  for (int q = 0; q < 2; ++q) {
    if (p->ev_post[q]) (void)hipEventDestroy(p->ev_post[q]);
    if (p->post_stream[q]) {
      (void)hipStreamSynchronize(p->post_stream[q]);
      (void)hipStreamDestroy(p->post_stream[q]);
    }
    p->ev_post[q] = nullptr;
    p->post_stream[q] = nullptr;
  }
}

// The two post streams, their join events and one event per schedule group,
// made together: created into locals and kept only when every creation
// succeeded, so the problem holds either all of them or none.
pcv_status ensure_post_streams(pcv_problem* p) {
  if (p->post_stream[0] && p->ev_fact.size() == p->groups.size()) return PCV_OK;
  drop_post_streams(p);
  hipStream_t st[2] = {};
  hipEvent_t ep[2] = {};
  std::vector<hipEvent_t> ef(p->groups.size(), nullptr);
  hipError_t e = hipSuccess;
  for (int q = 0; q < 2 && e == hipSuccess; ++q) {
    e = hipStreamCreateWithFlags(&st[q], hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ep[q], hipEventDisableTiming);
  }
  for (size_t k = 0; k < ef.size() && e == hipSuccess; ++k) e = hipEventCreateWithFlags(&ef[k], hipEventDisableTiming);
  if (e != hipSuccess) {
    for (hipEvent_t x : ef)
      if (x) (void)hipEventDestroy(x);
    for (int q = 0; q < 2; ++q) {
      if (ep[q]) (void)hipEventDestroy(ep[q]);
      if (st[q]) (void)hipStreamDestroy(st[q]);
    }
    (void)hipGetLastError();
    return fail(PCV_ERR_DEVICE, std::string("post streams: ") + hipGetErrorString(e));
  }
  for (int q = 0; q < 2; ++q) {
    p->post_stream[q] = st[q];
    p->ev_post[q] = ep[q];
  }
  p->ev_fact = std::move(ef);
  return PCV_OK;
}

}  // namespace

// Drop the captured evaluations (they are captured again when next needed).
void drop_graphs(pcv_problem* p) {
  for (auto& g : p->graph_exec)
    if (g) {
      (void)hipGraphExecDestroy(g);
      g = nullptr;
    }
  for (auto& pl : p->batch.plans)
    if (pl.graph) {
      (void)hipGraphExecDestroy(pl.graph);
      pl.graph = nullptr;
    }
}

pcv_status set_served(pcv_problem* p, bool on) {
  HIPCHK(hipSetDevice(p->device));
  HIPCHK(hipStreamSynchronize(p->stream));
  drop_graphs(p);
  drop_post_streams(p);
  p->served = on;
  return PCV_OK;
}

pcv_status apply_tuning(pcv_problem* p, int32_t small_npad, int32_t max_wg, bool two_groups) {
  if (max_wg < 0 || max_wg > 8 || small_npad < 0) return fail(PCV_ERR_INVALID, "bad tuning parameters");
  HIPCHK(hipSetDevice(p->device));
  HIPCHK(hipStreamSynchronize(p->stream));  // nothing in flight uses the old plan
  drop_graphs(p);
  drop_post_streams(p);
  p->tune_small_npad = small_npad;
  p->tune_two_groups = two_groups;
  p->opt.max_wg_per_subset = max_wg;
  free_coop(p);
  plan_coop(p);
  pcv_status s = upload_coop(p);
  if (s != PCV_OK) {
    // keep the problem usable: no sharing
    free_coop(p);
    p->coop_blocks = p->coop_slots = 0;
    p->coop_order.clear();
    p->coop_info.clear();
  }
  return s;
}

void problem_free(pcv_problem* p) {
  if (!p) return;
  if (p->stream) (void)hipStreamSynchronize(p->stream);
  for (auto& g : p->graph_exec)
    if (g) (void)hipGraphExecDestroy(g);
  for (auto& pl : p->batch.plans)
    if (pl.graph) (void)hipGraphExecDestroy(pl.graph);
  if (p->batch.h_theta) (void)hipHostFree(p->batch.h_theta);
  if (p->batch.h_total) (void)hipHostFree(p->batch.h_total);
  if (p->batch.h_nbad) (void)hipHostFree(p->batch.h_nbad);
  for (void* a : p->allocs) (void)hipFree(a);
  p->allocs.clear();
  if (p->h_theta) (void)hipHostFree(p->h_theta);
  if (p->h_total) (void)hipHostFree(p->h_total);
  if (p->h_nbad) (void)hipHostFree(p->h_nbad);
  if (p->events)
    for (auto& e : p->ev) (void)hipEventDestroy(e);
  drop_post_streams(p);
  if (p->own_stream && p->stream) (void)hipStreamDestroy(p->stream);
  delete p;
}

namespace {

// Factor + solve alpha = M^{-1} y_T in FP64 for the subsets in `d_order`
// (device list of `count` subset ids) into the given buffers.
pcv_status factor_solve64(pcv_problem* p, const SubsetDesc* d_desc, const ThetaDev* d_theta,
                          const int32_t* d_order, int count, double* Lb, double* Invb, double* zb,
                          double* alphab, double* logdetb, int32_t* statusb) {
  Launch Lc{p->stream, d_desc, d_theta};
  // z = L^{-1} y_T from the factorisation's y_T row
  HIPCHK(launch_potrf_f64(Lc, d_order, count, p->d_px64, p->d_py64, p->d_pv64, zb, Lb, Invb, logdetb, statusb));
  HIPCHK(launch_trsv_bwd_f64(Lc, d_order, count, p->max_npad, Lb, Invb, zb, alphab, nullptr));
  return PCV_OK;
}

}  // namespace

namespace {

// Phases of one theta-evaluation: upload of the theta block from pinned
// memory, factorisation, solves, refinement sweeps, kriging of the
// validation points, reduction, download of the loss and of the count of
// subsets that need the FP64 re-run.  Profiling records an event after each
// of the first six.
constexpr int N_PHASES = 7;

// The first launch may share its largest subsets (planned, not served, and
// in FP32 that launch takes the 8-wave shape the sharing needs).
bool coop_active(const pcv_problem* p) {
  return p->coop_slots > 0 && !p->served && p->n_active > 0 &&
         (p->opt.prec != PCV_PREC_MIXED || sched_npad(p, 0) > p->tune_small_npad);
}

// At most one evaluation with a shared factorisation launch runs on a device
// at a time in this process.  The work-groups of a shared subset wait for
// each other, which is safe while every work-group of the launch can become
// resident; two such launches side by side could hold each other's compute
// units until their bounded waits run out.  An evaluation that finds its
// device's flag taken factors with one work-group per subset instead (the
// same bits).  The flag is released after the evaluation's stream has
// drained.
constexpr int COOP_MAX_DEVICES = 64;
std::atomic<int> g_coop_busy[COOP_MAX_DEVICES];

struct CoopGuard {
  int dev = -1;
  hipStream_t stream = nullptr;
  bool held = false;
  bool acquire(int d, hipStream_t st) {
    if (d < 0 || d >= COOP_MAX_DEVICES) return false;
    int z = 0;
    held = g_coop_busy[d].compare_exchange_strong(z, 1, std::memory_order_acq_rel);
    dev = d;
    stream = st;
    return held;
  }
  ~CoopGuard() {
    if (!held) return;
    (void)hipStreamSynchronize(stream);
    g_coop_busy[dev].store(0, std::memory_order_release);
  }
};

// Subsets per factorisation launch: one launch, or for a served problem
// launches of one work-group per compute unit.  A served problem's
// evaluation runs launch by launch with the host waiting for each (the
// server's kriging streams may share its hardware queue, whose work runs in
// order), so a kriging batch waits behind one launch at most, and a
// factorisation launch lasts about one work-group's time.
int32_t factor_chunk(const pcv_problem* p, int32_t cnt) {
  return p->served && p->n_cu > 0 ? std::min(cnt, p->n_cu) : std::max(cnt, 1);
}

pcv_status enqueue_phase(pcv_problem* p, hipStream_t st, int phase, bool mixed, int sweeps,
                         const pcv_group& G) {
  Launch Lc{st, p->d_desc, p->d_theta};
  const int32_t* order = p->d_order_eval + G.o0;
  const int32_t cnt = G.cnt;
  // a served problem's evaluation waits for each launch before the next, so
  // that a kriging batch sharing its hardware queue never waits behind more
  // than one launch
#define PACE()                                       \
  do {                                               \
    if (p->served) HIPCHK(hipStreamSynchronize(st)); \
  } while (0)
  switch (phase) {
    case 0:
      HIPCHK(hipMemcpyAsync(p->d_theta, p->h_theta, sizeof(ThetaDev), hipMemcpyHostToDevice, st));
      break;
    case 1:
      if (p->coop_now && G.o0 == 0 && cnt == p->coop_group_cnt) {
        // the first launch with its largest subsets shared by several work-groups
        const CoopPlan cp{p->d_coop_info, p->coop_blocks, p->d_coop_sync, p->coop_slots, p->d_order_eval, cnt};
        const int nb = (int)p->coop_order.size();
        if (mixed)
          HIPCHK(launch_potrf_f32(Lc, p->d_coop_order, nb, p->desc[p->order_eval[0]].npad, p->d_px32,
                                  p->d_py32, p->d_pv32, p->d_z, p->d_L32, p->d_Inv, p->d_logdet, p->d_status,
                                  &cp));
        else
          HIPCHK(launch_potrf_f64(Lc, p->d_coop_order, nb, p->d_px64, p->d_py64, p->d_pv64, p->d_z, p->d_L64,
                                  p->d_Inv, p->d_logdet, p->d_status, &cp));
        break;
      }
      // the part of each schedule group inside G, in launches of
      // factor_chunk subsets, each with its schedule group's shape
      for (int k = 0; k < n_sched(p); ++k) {
        const pcv_group& SG = sched(p, k);
        const int32_t a = std::max(G.o0, SG.o0), e = std::min(G.o0 + cnt, SG.o0 + SG.cnt);
        for (int32_t c0 = a; c0 < e; c0 += factor_chunk(p, e - a)) {
          const int32_t c = std::min(factor_chunk(p, e - a), e - c0);
          if (mixed)
            HIPCHK(launch_potrf_f32(Lc, p->d_order_eval + c0, c, sched_npad(p, k), p->d_px32, p->d_py32, p->d_pv32,
                                    p->d_z, p->d_L32, p->d_Inv, p->d_logdet, p->d_status, nullptr,
                                    p->tune_small_npad));
          else
            HIPCHK(launch_potrf_f64(Lc, p->d_order_eval + c0, c, p->d_px64, p->d_py64, p->d_pv64, p->d_z, p->d_L64,
                                    p->d_Inv, p->d_logdet, p->d_status));
          PACE();
        }
      }
      break;
    case 2:
      // z = L^{-1} y_T came out of the factorisation (the y_T row)
      if (mixed) {
        HIPCHK(launch_trsv_bwd_f32(Lc, order, cnt, p->max_npad, p->d_L32, p->d_Inv, p->d_z,
                                   p->d_alpha, nullptr));
        PACE();
      } else {
        HIPCHK(launch_trsv_bwd_f64(Lc, order, cnt, p->max_npad, p->d_L64, p->d_Inv, p->d_z,
                                   p->d_alpha, nullptr));
        PACE();
      }
      break;
    case 3:
      // every subset takes the first sweep; a later one only where the
      // residual the previous sweep measured is still above refine_tol
      for (int it = 0; it < sweeps; ++it) {
        const int32_t* gate = it > 0 ? p->d_gate : nullptr;
        if (it > 0) {
          HIPCHK(launch_refine_gate(st, cnt, order, p->S, it, p->d_rhs2, p->d_ynorm2, p->opt.refine_tol,
                                    p->d_gate, p->d_nsweep));
          PACE();
        }
        HIPCHK(launch_residual(Lc, p->d_tile_items + G.r0, G.nr, p->d_row_items + G.r0, G.nr, p->d_tx, p->d_ty,
                               p->d_yT, p->d_alpha, p->d_rrow, p->d_pcol, p->d_r, gate));
        PACE();
        HIPCHK(launch_trsv_fwd_f32(Lc, order, cnt, p->max_npad, p->d_L32, p->d_Inv, nullptr,
                                   p->d_r, p->d_z, p->d_rhs2, gate));
        PACE();
        HIPCHK(launch_trsv_bwd_f32(Lc, order, cnt, p->max_npad, p->d_L32, p->d_Inv, p->d_z,
                                   p->d_x, p->d_alpha, gate));
        PACE();
      }
      break;
    case 4:
      HIPCHK(launch_predict_val(Lc, p->d_val_items + G.v0, G.nv, p->d_tx, p->d_ty, p->d_vx,
                                p->d_vy, p->d_yV, p->d_alpha, p->d_yhat, p->d_err));
      PACE();
      HIPCHK(launch_quad(st, p->d_desc, order, cnt, p->d_yT, p->d_alpha, p->d_quad));
      PACE();
      break;
    case 5:
      HIPCHK(launch_reduce(st, p->d_desc, p->S, 1, p->d_err, p->d_status, p->d_active,
                           sweeps > 0 ? p->d_rhs2 : nullptr, p->d_ynorm2, p->opt.refine_tol, p->d_sspe,
                           p->d_total, p->d_nbad));
      break;
    case 6:
      HIPCHK(hipMemcpyAsync(p->h_total, p->d_total, sizeof(double), hipMemcpyDeviceToHost, st));
      HIPCHK(hipMemcpyAsync(p->h_nbad, p->d_nbad, sizeof(int32_t), hipMemcpyDeviceToHost, st));
      break;
  }
  return PCV_OK;
}
#undef PACE

// The whole evaluation on st.  With several schedule groups the
// factorisations run group after group on st and each group's later phases
// on post stream k % 2 once its factorisation is done; the post streams are
// joined back into st before the reduction.
int n_groups(const pcv_problem* p) { return p->served ? 1 : n_sched(p); }

pcv_status enqueue_all(pcv_problem* p, hipStream_t st, const hipStream_t* ps, bool mixed, int sweeps) {
  pcv_status s = PCV_OK;
  const int K = n_groups(p);
  if (K <= 1) {
    for (int ph = 0; ph < N_PHASES && s == PCV_OK; ++ph) s = enqueue_phase(p, st, ph, mixed, sweeps, p->g_all);
    return s;
  }
  if (p->ev_fact.size() != (size_t)K || !ps[0] || !ps[1])
    return fail(PCV_ERR_STATE, "two-stream schedule without its streams and events");
  if ((s = enqueue_phase(p, st, 0, mixed, sweeps, p->g_all)) != PCV_OK) return s;
  for (int k = 0; k < K; ++k) {
    if ((s = enqueue_phase(p, st, 1, mixed, sweeps, p->groups[k])) != PCV_OK) return s;
    HIPCHK(hipEventRecord(p->ev_fact[k], st));
  }
  for (int k = 0; k < K; ++k) {
    hipStream_t q = ps[k & 1];
    HIPCHK(hipStreamWaitEvent(q, p->ev_fact[k], 0));
    for (int ph = 2; ph <= 4 && s == PCV_OK; ++ph) s = enqueue_phase(p, q, ph, mixed, sweeps, p->groups[k]);
    if (s != PCV_OK) return s;
  }
  for (int q = 0; q < 2; ++q) {
    HIPCHK(hipEventRecord(p->ev_post[q], ps[q]));
    HIPCHK(hipStreamWaitEvent(st, p->ev_post[q], 0));
  }
  for (int ph = 5; ph < N_PHASES && s == PCV_OK; ++ph) s = enqueue_phase(p, st, ph, mixed, sweeps, p->g_all);
  return s;
}

// Capture the whole evaluation on private streams, so that the caller's
// stream may be the null stream, and instantiate it as one graph.
pcv_status capture_eval(pcv_problem* p, bool mixed, int sweeps, hipGraphExec_t* out) {
  hipStream_t cs = nullptr, cps[2] = {};
  HIPCHK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  hipError_t e = hipSuccess;
  if (n_groups(p) > 1) {
    e = hipStreamCreateWithFlags(&cps[0], hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&cps[1], hipStreamNonBlocking);
  }
  if (e != hipSuccess) {
    for (hipStream_t x : {cs, cps[0], cps[1]})
      if (x) (void)hipStreamDestroy(x);
    (void)hipGetLastError();
    return fail(PCV_ERR_DEVICE, std::string("hipStreamCreate: ") + hipGetErrorString(e));
  }
  hipGraph_t g = nullptr;
  pcv_status s = PCV_OK;
  e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) s = fail(PCV_ERR_DEVICE, std::string("hipStreamBeginCapture: ") + hipGetErrorString(e));
  if (e == hipSuccess) {
    s = enqueue_all(p, cs, cps, mixed, sweeps);
    e = hipStreamEndCapture(cs, &g);
    if (s == PCV_OK && e != hipSuccess) s = fail(PCV_ERR_DEVICE, std::string("graph capture: ") + hipGetErrorString(e));
  }
  if (s == PCV_OK) {
    e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      *out = nullptr;
      s = fail(PCV_ERR_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    }
  }
  if (g) (void)hipGraphDestroy(g);
  for (hipStream_t x : {cps[1], cps[0]})
    if (x) (void)hipStreamDestroy(x);
  (void)hipStreamDestroy(cs);
  if (s != PCV_OK) (void)hipGetLastError();  // reported here, not again at a later launch
  return s;
}

// The schedule of enqueue_all launched eagerly with timing events: ev[0]
// after the theta upload, ev[1] after the first group's factorisation, ev[7]
// after the last group's (all on the factorisation stream); ev[2], ev[3],
// ev[4] after the first group's solves, refinement and kriging (on its post
// stream); ev[6] after the join and ev[5] after the reduction.
pcv_status enqueue_profiled(pcv_problem* p, bool mixed, int sweeps) {
  hipStream_t st = p->stream;
  const int K = n_groups(p);
  const pcv_group& G0 = K > 1 ? p->groups[0] : p->g_all;
  if (K > 1 && (p->ev_fact.size() != (size_t)K || !p->post_stream[0] || !p->post_stream[1]))
    return fail(PCV_ERR_STATE, "two-stream schedule without its streams and events");
  pcv_status s = enqueue_phase(p, st, 0, mixed, sweeps, p->g_all);
  if (s != PCV_OK) return s;
  HIPCHK(hipEventRecord(p->ev[0], st));
  if ((s = enqueue_phase(p, st, 1, mixed, sweeps, G0)) != PCV_OK) return s;
  HIPCHK(hipEventRecord(p->ev[1], st));
  if (K > 1) HIPCHK(hipEventRecord(p->ev_fact[0], st));
  for (int k = 1; k < K; ++k) {
    if ((s = enqueue_phase(p, st, 1, mixed, sweeps, p->groups[k])) != PCV_OK) return s;
    HIPCHK(hipEventRecord(p->ev_fact[k], st));
  }
  HIPCHK(hipEventRecord(p->ev[7], st));
  hipStream_t q0 = K > 1 ? p->post_stream[0] : st;
  if (K > 1) HIPCHK(hipStreamWaitEvent(q0, p->ev_fact[0], 0));
  for (int ph = 2; ph <= 4; ++ph) {
    if ((s = enqueue_phase(p, q0, ph, mixed, sweeps, G0)) != PCV_OK) return s;
    HIPCHK(hipEventRecord(p->ev[ph], q0));
  }
  for (int k = 1; k < K; ++k) {
    hipStream_t q = p->post_stream[k & 1];
    HIPCHK(hipStreamWaitEvent(q, p->ev_fact[k], 0));
    for (int ph = 2; ph <= 4 && s == PCV_OK; ++ph) s = enqueue_phase(p, q, ph, mixed, sweeps, p->groups[k]);
    if (s != PCV_OK) return s;
  }
  if (K > 1)
    for (int q = 0; q < 2; ++q) {
      HIPCHK(hipEventRecord(p->ev_post[q], p->post_stream[q]));
      HIPCHK(hipStreamWaitEvent(st, p->ev_post[q], 0));
    }
  HIPCHK(hipEventRecord(p->ev[6], st));
  if ((s = enqueue_phase(p, st, 5, mixed, sweeps, p->g_all)) != PCV_OK) return s;
  HIPCHK(hipEventRecord(p->ev[5], st));
  return enqueue_phase(p, st, 6, mixed, sweeps, p->g_all);
}

// Enqueue one theta-evaluation on the problem's stream: as one graph
// (default), eagerly, or eagerly with timing events when profiling.
pcv_status enqueue_eval(pcv_problem* p, bool mixed, int sweeps) {
  if (n_groups(p) > 1) {
    pcv_status s = ensure_post_streams(p);
    if (s != PCV_OK) return s;
  }
  if (p->events) return enqueue_profiled(p, mixed, sweeps);
  if (!p->opt.graph || p->served) return enqueue_all(p, p->stream, p->post_stream, mixed, sweeps);
  // [0]: the evaluation as planned; [1]: with one work-group per subset,
  // for evaluations that find another shared launch in flight
  hipGraphExec_t& g = (p->coop_now || !coop_active(p)) ? p->graph_exec[0] : p->graph_exec[1];
  if (!g) {
    pcv_status s = capture_eval(p, mixed, sweeps, &g);
    if (s != PCV_OK) return s;
  }
  HIPCHK(hipGraphLaunch(g, p->stream));
  return PCV_OK;
}

// Error estimate of a mixed evaluation (opt.est_error): one more refinement
// sweep over the subsets in fp_list's complement that were factored in FP32,
// its correction added to a copy of alpha (d_rrow, free once the residual is
// formed), and the loss recomputed from the copy into est_total.  The
// evaluation's own buffers other than d_r, d_z, d_x, d_rrow, d_pcol and
// d_gate are left as they are.
pcv_status estimate_loss(pcv_problem* p, const std::vector<int32_t>& fb_list, double* out_total) {
  pcv_status s;
  if (!p->d_est_yhat) {
    const size_t nv = (size_t)std::max<int64_t>(p->nnzV, 1);
    if ((s = dalloc(p, &p->d_est_yhat, nv)) != PCV_OK) return s;
    if ((s = dalloc(p, &p->d_est_err, nv)) != PCV_OK) return s;
    if ((s = dalloc(p, &p->d_est_sspe, (size_t)p->S)) != PCV_OK) return s;
    if ((s = dalloc(p, &p->d_est_total, 1)) != PCV_OK) return s;
    if ((s = dalloc(p, &p->d_est_nbad, 1)) != PCV_OK) return s;
  }
  hipStream_t st = p->stream;
  Launch Lc{st, p->d_desc, p->d_theta};
  std::vector<int32_t> gate(p->S, 0);
  for (int32_t i : p->order_eval) gate[i] = 1;
  for (int32_t i : fb_list) gate[i] = 0;
  HIPCHK(hipMemcpyAsync(p->d_gate, gate.data(), sizeof(int32_t) * p->S, hipMemcpyHostToDevice, st));
  const pcv_group& G = p->g_all;
  const int32_t* order = p->d_order_eval;
  const int cnt = p->n_active;
  HIPCHK(launch_residual(Lc, p->d_tile_items + G.r0, G.nr, p->d_row_items + G.r0, G.nr, p->d_tx, p->d_ty, p->d_yT,
                         p->d_alpha, p->d_rrow, p->d_pcol, p->d_r, p->d_gate));
  HIPCHK(hipMemcpyAsync(p->d_rrow, p->d_alpha, sizeof(double) * p->nP, hipMemcpyDeviceToDevice, st));
  HIPCHK(launch_trsv_fwd_f32(Lc, order, cnt, p->max_npad, p->d_L32, p->d_Inv, nullptr, p->d_r, p->d_z, nullptr,
                             p->d_gate));
  HIPCHK(launch_trsv_bwd_f32(Lc, order, cnt, p->max_npad, p->d_L32, p->d_Inv, p->d_z, p->d_x, p->d_rrow,
                             p->d_gate));
  HIPCHK(launch_predict_val(Lc, p->d_val_items, (int)p->val_items.size(), p->d_tx, p->d_ty, p->d_vx, p->d_vy,
                            p->d_yV, p->d_rrow, p->d_est_yhat, p->d_est_err));
  HIPCHK(launch_reduce(st, p->d_desc, p->S, 1, p->d_est_err, p->d_status, p->d_active, nullptr, nullptr, 0.0,
                       p->d_est_sspe, p->d_est_total, p->d_est_nbad));
  HIPCHK(hipMemcpyAsync(out_total, p->d_est_total, sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  return PCV_OK;
}

}  // namespace

pcv_status eval_impl(pcv_problem* p, const pcv_theta& th, double* loss, pcv_eval_report* rep) {
  const double t0 = now_s();
  HIPCHK(hipSetDevice(p->device));
  const bool mixed = p->opt.prec == PCV_PREC_MIXED;
  pcv_status s = ensure_L(p, !mixed);
  if (s != PCV_OK) return s;
  set_theta_host(p, th);
  const int sweeps = mixed ? p->opt.max_refine : 0;
  CoopGuard coop;
  // debug bit 1: behave as if another shared launch held the device
  p->coop_now = coop_active(p) && !(p->opt.debug_flags & 2) && coop.acquire(p->device, p->stream);
  s = enqueue_eval(p, mixed, sweeps);
  if (s != PCV_OK) return s;
  HIPCHK(hipStreamSynchronize(p->stream));
  Launch Lc{p->stream, p->d_desc, p->d_theta};

  int32_t n_fallback = 0;
  std::vector<int32_t> fb_list;
  const bool force_fb = mixed && (p->opt.debug_flags & 1) && p->n_active > 0;
  if (*p->h_nbad > 0 || force_fb) {
    std::vector<int32_t> status(p->S);
    HIPCHK(hipMemcpy(status.data(), p->d_status, sizeof(int32_t) * p->S, hipMemcpyDeviceToHost));
    std::vector<int32_t> bad;
    for (int32_t i : p->order_eval)
      if (status[i] || force_fb) bad.push_back(i);
    if (!mixed) {
      if (status[bad[0]] == PCV_STATUS_SYNC_TIMEOUT)
        return fail(PCV_ERR_DEVICE, "subset " + std::to_string(bad[0]) +
                                        ": a work-group of its shared factorisation waited past its bound");
      return fail(PCV_ERR_NOT_PD, "subset " + std::to_string(bad[0]) + " is not positive definite (pivot " +
                                      std::to_string(status[bad[0]] - 1) + ")");
    }
    // FP64 re-run of the subsets whose FP32 factorisation broke down, their
    // FP64 factors packed into a buffer sized for them alone
    n_fallback = (int32_t)bad.size();
    fb_list = bad;
    std::vector<SubsetDesc> dfb = p->desc;
    int64_t need = 0;
    for (int32_t i : bad) {
      dfb[i].offL = need;
      need += packed_size(dfb[i].npad);
    }
    if (!p->d_desc_fb && (s = dalloc(p, &p->d_desc_fb, (size_t)p->S)) != PCV_OK) return s;
    if (need > p->L64fb_cap) {
      dfree(p, p->d_L64fb, sizeof(double) * (size_t)p->L64fb_cap);
      p->d_L64fb = nullptr;
      p->L64fb_cap = 0;
      if ((s = dalloc(p, &p->d_L64fb, (size_t)need)) != PCV_OK) return s;
      p->L64fb_cap = need;
    }
    HIPCHK(hipMemcpy(p->d_desc_fb, dfb.data(), sizeof(SubsetDesc) * p->S, hipMemcpyHostToDevice));
    int32_t* d_bad = p->d_bad;
    HIPCHK(hipMemcpyAsync(d_bad, bad.data(), sizeof(int32_t) * bad.size(), hipMemcpyHostToDevice, p->stream));
    s = factor_solve64(p, p->d_desc_fb, p->d_theta, d_bad, (int)bad.size(), p->d_L64fb, p->d_Inv, p->d_z,
                       p->d_alpha, p->d_logdet, p->d_status);
    if (s == PCV_OK) {
      HIPCHK(launch_predict_val(Lc, p->d_val_items, (int)p->val_items.size(), p->d_tx, p->d_ty, p->d_vx,
                                p->d_vy, p->d_yV, p->d_alpha, p->d_yhat, p->d_err));
      HIPCHK(launch_quad(p->stream, p->d_desc, p->d_order_eval, p->n_active, p->d_yT, p->d_alpha, p->d_quad));
      HIPCHK(launch_reduce(p->stream, p->d_desc, p->S, 1, p->d_err, p->d_status, p->d_active, nullptr,
                           nullptr, 0.0, p->d_sspe, p->d_total, p->d_nbad));
      HIPCHK(hipMemcpyAsync(p->h_total, p->d_total, sizeof(double), hipMemcpyDeviceToHost, p->stream));
      HIPCHK(hipMemcpyAsync(p->h_nbad, p->d_nbad, sizeof(int32_t), hipMemcpyDeviceToHost, p->stream));
      HIPCHK(hipStreamSynchronize(p->stream));
    }
    if (s != PCV_OK) return s;
    if (*p->h_nbad > 0) {
      HIPCHK(hipMemcpy(status.data(), p->d_status, sizeof(int32_t) * p->S, hipMemcpyDeviceToHost));
      for (int32_t i : bad)
        if (status[i])
          return fail(PCV_ERR_NOT_PD, "subset " + std::to_string(i) + " is not positive definite in FP64");
    }
  }
  *loss = *p->h_total;
  double est = mixed ? -1.0 : 0.0;
  // (only when a report asks for it)
  if (rep && mixed && p->opt.est_error && p->n_active > 0 && (int32_t)fb_list.size() < p->n_active) {
    double total2 = 0.0;
    if ((s = estimate_loss(p, fb_list, &total2)) != PCV_OK) return s;
    est = *loss != 0.0 ? std::fabs(*loss - total2) / std::fabs(*loss) : std::fabs(total2);
  } else if (mixed && p->opt.est_error) {
    est = 0.0;  // every evaluated subset came from the FP64 path
  }
  if (rep) {
    rep->est_rel_err = est;
    rep->sspe = *loss;
    rep->n_val = p->n_val_total;
    rep->mse = p->n_val_total ? *loss / (double)p->n_val_total : 0.0;
    rep->n_subsets_used = p->n_active;
    rep->n_fallback_fp64 = n_fallback;
    // sweeps per subset: all of them with one sweep or none, else as the
    // gates decided; a subset re-run in FP64 counts none
    std::vector<int32_t> ns(p->S, 0);
    if (sweeps > 1) HIPCHK(hipMemcpy(ns.data(), p->d_nsweep, sizeof(int32_t) * p->S, hipMemcpyDeviceToHost));
    std::vector<char> fb(p->S, 0);
    for (int32_t i : fb_list) fb[i] = 1;
    rep->max_refine_iters = 0;
    for (int32_t i : p->order_eval) {
      if (sweeps <= 1) ns[i] = sweeps;
      if (fb[i]) ns[i] = 0;
      rep->max_refine_iters = std::max(rep->max_refine_iters, ns[i]);
    }
    if (rep->per_subset_iters)
      for (int32_t i = 0; i < p->S; ++i) rep->per_subset_iters[i] = p->active[i] ? ns[i] : 0;
    rep->max_rel_residual = 0.0;
    if (sweeps > 0) {
      std::vector<double> r2(p->S);
      HIPCHK(hipMemcpy(r2.data(), p->d_rhs2, sizeof(double) * p->S, hipMemcpyDeviceToHost));
      for (int32_t i : p->order_eval)
        if (p->ynorm2[i] > 0) rep->max_rel_residual = std::max(rep->max_rel_residual, std::sqrt(r2[i] / p->ynorm2[i]));
    }
    if (rep->per_subset_sspe)
      HIPCHK(hipMemcpy(rep->per_subset_sspe, p->d_sspe, sizeof(double) * p->S, hipMemcpyDeviceToHost));
    if (rep->per_subset_logdet) {
      std::vector<double> ld(p->S);
      HIPCHK(hipMemcpy(ld.data(), p->d_logdet, sizeof(double) * p->S, hipMemcpyDeviceToHost));
      for (int32_t i = 0; i < p->S; ++i) rep->per_subset_logdet[i] = p->active[i] ? ld[i] : 0.0;
    }
    {
      // composite likelihood, summed in subset order with compensation
      std::vector<double> ld(p->S), qd(p->S);
      HIPCHK(hipMemcpy(ld.data(), p->d_logdet, sizeof(double) * p->S, hipMemcpyDeviceToHost));
      HIPCHK(hipMemcpy(qd.data(), p->d_quad, sizeof(double) * p->S, hipMemcpyDeviceToHost));
      const double l2pi = std::log(2.0 * M_PI), ls2 = std::log(th.sigma2);
      double sum = 0.0, comp = 0.0;
      for (int32_t i = 0; i < p->S; ++i) {
        double v = 0.0;
        if (p->active[i]) {
          const double n = (double)p->desc[i].n;
          v = n * l2pi + n * ls2 + ld[i] + qd[i] / th.sigma2;
          const double t = sum + v;
          comp += std::fabs(sum) >= std::fabs(v) ? (sum - t) + v : (v - t) + sum;
          sum = t;
        }
        if (rep->per_subset_neg2loglik) rep->per_subset_neg2loglik[i] = v;
      }
      rep->neg2loglik = sum + comp;
    }
    rep->ms_factor = rep->ms_solve = rep->ms_refine = rep->ms_predict = rep->ms_reduce = 0.0;
    rep->ms_factor_all = 0.0;
    rep->n_factor_first = n_groups(p) > 1 ? p->groups[0].cnt : p->n_active;
    rep->n_coop_subsets = p->coop_now ? p->coop_slots : 0;
    if (p->events) {
      float ms;
      HIPCHK(hipEventElapsedTime(&ms, p->ev[0], p->ev[1]));
      rep->ms_factor = ms;
      HIPCHK(hipEventElapsedTime(&ms, p->ev[1], p->ev[2]));
      rep->ms_solve = ms;
      HIPCHK(hipEventElapsedTime(&ms, p->ev[2], p->ev[3]));
      rep->ms_refine = ms;
      HIPCHK(hipEventElapsedTime(&ms, p->ev[3], p->ev[4]));
      rep->ms_predict = ms;
      HIPCHK(hipEventElapsedTime(&ms, p->ev[6], p->ev[5]));
      rep->ms_reduce = ms;
      HIPCHK(hipEventElapsedTime(&ms, p->ev[0], p->ev[7]));
      rep->ms_factor_all = ms;
    }
    rep->seconds = now_s() - t0;
  }
  return PCV_OK;
}

namespace {

// Device bytes of one theta slot of the batch workspace.
size_t batch_slot_bytes(const pcv_problem* p, bool mixed) {
  // per theta slot: factor, inverses, vectors, partials, predictions, the
  // per-subset arrays and descriptors, and the plans' item lists
  return (size_t)p->nL * (mixed ? 4 : 8) + (size_t)p->nInv * 8 + (size_t)p->nP * 8 * 6 +
         (size_t)p->nPC * 8 + (size_t)p->nnzV * 8 * 2 + (size_t)p->S * (8 * 4 + 4 * 3 + sizeof(SubsetDesc)) +
         (size_t)p->S * 4 + (p->row_items_eval.size() * 2 + p->val_items.size()) * sizeof(int2) + 64;
}

// The multi-theta workspace's buffers (those allocated so far), freed.
void free_batch(pcv_problem* p, int B, bool mixed) {
  pcv_batch& b = p->batch;
  const size_t S = (size_t)p->S, Bs = (size_t)B;
  dfree_n(p, b.d_desc, Bs * S);
  if (mixed) {
    float* L = (float*)b.d_L;
    dfree_n(p, L, Bs * p->nL);
  } else {
    double* L = (double*)b.d_L;
    dfree_n(p, L, Bs * p->nL);
  }
  b.d_L = nullptr;
  dfree_n(p, b.d_Inv, Bs * p->nInv);
  for (double** q : {&b.d_z, &b.d_x, &b.d_alpha, &b.d_r, &b.d_rrow}) dfree_n(p, *q, Bs * p->nP);
  dfree_n(p, b.d_pcol, Bs * std::max<int64_t>(p->nPC, 1));
  dfree_n(p, b.d_yhat, Bs * std::max<int64_t>(p->nnzV, 1));
  dfree_n(p, b.d_err, Bs * std::max<int64_t>(p->nnzV, 1));
  for (double** q : {&b.d_rhs2, &b.d_logdet, &b.d_sspe, &b.d_quad}) dfree_n(p, *q, Bs * S);
  for (int32_t** q : {&b.d_status, &b.d_gate, &b.d_nsweep}) dfree_n(p, *q, Bs * S);
  dfree_n(p, b.d_total, Bs);
  dfree_n(p, b.d_nbad, Bs);
  dfree_n(p, b.d_theta, Bs);
  if (b.h_theta) (void)hipHostFree(b.h_theta);
  if (b.h_total) (void)hipHostFree(b.h_total);
  if (b.h_nbad) (void)hipHostFree(b.h_nbad);
  b.h_theta = nullptr;
  b.h_total = nullptr;
  b.h_nbad = nullptr;
  b.B = 0;
}

// Allocate the workspace for B theta slots; on failure nothing of it is
// kept (so that a caller can fall back to one theta at a time).
pcv_status ensure_batch(pcv_problem* p, int B, bool mixed) {
  pcv_batch& b = p->batch;
  if (b.B >= B) return PCV_OK;
  if (b.B > 0) return fail(PCV_ERR_STATE, "batch workspace already sized");
  const int S = p->S;
  pcv_status s;
#define TRYB(x)                  \
  do {                           \
    s = (x);                     \
    if (s != PCV_OK) {           \
      free_batch(p, B, mixed);   \
      return s;                  \
    }                            \
  } while (0)
  std::vector<SubsetDesc> db((size_t)B * S);
  for (int t = 0; t < B; ++t)
    for (int i = 0; i < S; ++i) {
      SubsetDesc d = p->desc[i];
      d.th = t;
      d.offP += (int64_t)t * p->nP;
      d.offL += (int64_t)t * p->nL;
      d.offInv += (int64_t)t * p->nInv;
      d.offPC += (int64_t)t * p->nPC;
      d.offE += (int64_t)t * p->nnzV;
      db[(size_t)t * S + i] = d;
    }
  TRYB(upload(p, &b.d_desc, db));
  if (mixed) {
    float* L = nullptr;
    TRYB(dalloc(p, &L, (size_t)B * p->nL));
    b.d_L = L;
  } else {
    double* L = nullptr;
    TRYB(dalloc(p, &L, (size_t)B * p->nL));
    b.d_L = L;
  }
  TRYB(dalloc(p, &b.d_Inv, (size_t)B * p->nInv));
  for (double** q : {&b.d_z, &b.d_x, &b.d_alpha, &b.d_r, &b.d_rrow}) TRYB(dalloc(p, q, (size_t)B * p->nP));
  TRYB(dalloc(p, &b.d_pcol, (size_t)B * std::max<int64_t>(p->nPC, 1)));
  TRYB(dalloc(p, &b.d_yhat, (size_t)B * std::max<int64_t>(p->nnzV, 1)));
  TRYB(dalloc(p, &b.d_err, (size_t)B * std::max<int64_t>(p->nnzV, 1)));
  for (double** q : {&b.d_rhs2, &b.d_logdet, &b.d_sspe, &b.d_quad}) TRYB(dalloc(p, q, (size_t)B * S));
  TRYB(dalloc(p, &b.d_status, (size_t)B * S));
  TRYB(dalloc(p, &b.d_gate, (size_t)B * S));
  TRYB(dalloc(p, &b.d_nsweep, (size_t)B * S));
  TRYB(dalloc(p, &b.d_total, (size_t)B));
  TRYB(dalloc(p, &b.d_nbad, (size_t)B));
  TRYB(dalloc(p, &b.d_theta, (size_t)B));
#undef TRYB
  hipError_t e = hipHostMalloc((void**)&b.h_theta, sizeof(ThetaDev) * B, hipHostMallocDefault);
  if (e == hipSuccess) e = hipHostMalloc((void**)&b.h_total, sizeof(double) * B, hipHostMallocDefault);
  if (e == hipSuccess) e = hipHostMalloc((void**)&b.h_nbad, sizeof(int32_t) * B, hipHostMallocDefault);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    free_batch(p, B, mixed);
    return fail(e == hipErrorOutOfMemory ? PCV_ERR_OOM : PCV_ERR_DEVICE,
                std::string("batch host buffers: ") + hipGetErrorString(e));
  }
  b.B = B;
  return PCV_OK;
}

// Item lists over (slot, subset) pairs for the first nb slots, largest
// subsets first (slots of one subset adjacent).
pcv_status batch_plan(pcv_problem* p, int nb, pcv_batch_plan** out) {
  pcv_batch& b = p->batch;
  for (auto& pl : b.plans)
    if (pl.nb == nb) {
      *out = &pl;
      return PCV_OK;
    }
  pcv_batch_plan* pl = nullptr;
  for (auto& q : b.plans)
    if (q.nb == 0) {
      pl = &q;
      break;
    }
  if (!pl) {
    pl = &b.plans[1];  // replace the remainder plan
    if (pl->graph) (void)hipGraphExecDestroy(pl->graph);
    dfree(p, pl->d_order, sizeof(int32_t) * pl->n_order);
    dfree(p, pl->d_row_items, sizeof(int2) * pl->n_row);
    dfree(p, pl->d_tile_items, sizeof(int2) * pl->n_tile);
    dfree(p, pl->d_val_items, sizeof(int2) * pl->n_val);
    *pl = pcv_batch_plan{};
  }
  const int S = p->S;
  std::vector<int32_t> order;
  std::vector<int2> rows, vals;
  for (int32_t i : p->order_eval)
    for (int t = 0; t < nb; ++t) {
      const int32_t k = t * S + i;
      order.push_back(k);
      for (int rb = 0; rb < p->desc[i].npad / TB; ++rb) rows.push_back(make_int2(k, rb));
      for (int vb = 0; vb < (p->desc[i].m + 63) / 64; ++vb) vals.push_back(make_int2(k, vb));
    }
  std::vector<int2> tiles = rows;
  std::stable_sort(tiles.begin(), tiles.end(), [](const int2& a, const int2& c) { return a.y > c.y; });
  pcv_status s;
  if ((s = upload(p, &pl->d_order, order)) != PCV_OK || (s = upload(p, &pl->d_row_items, rows)) != PCV_OK ||
      (s = upload(p, &pl->d_tile_items, tiles)) != PCV_OK || (s = upload(p, &pl->d_val_items, vals)) != PCV_OK) {
    // nothing of a plan that did not fit is kept
    dfree_n(p, pl->d_order, order.size());
    dfree_n(p, pl->d_row_items, rows.size());
    dfree_n(p, pl->d_tile_items, tiles.size());
    dfree_n(p, pl->d_val_items, vals.size());
    *pl = pcv_batch_plan{};
    return s;
  }
  pl->n_order = (int)order.size();
  pl->n_row = (int)rows.size();
  pl->n_tile = (int)tiles.size();
  pl->n_val = (int)vals.size();
  pl->nb = nb;
  *out = pl;
  return PCV_OK;
}

// One launch per kernel over the plan's (slot, subset) pairs, as in a
// single evaluation (upload of the theta slots, factorisation, solves,
// refinement, kriging of the validation points, per-slot reductions,
// download of the per-slot losses and fallback counts).
pcv_status enqueue_batch(pcv_problem* p, const pcv_batch_plan& pl, hipStream_t st, bool mixed, int sweeps,
                         bool ev) {
  pcv_batch& b = p->batch;
  Launch Lc{st, b.d_desc, b.d_theta};
  const int nb = pl.nb;
  // a served problem waits for each launch before the next, so that a
  // kriging batch sharing its hardware queue waits behind one launch at most
  auto pace = [&]() { return p->served ? hipStreamSynchronize(st) : hipSuccess; };
  const int32_t chunk = factor_chunk(p, pl.n_order);
  HIPCHK(hipMemcpyAsync(b.d_theta, b.h_theta, sizeof(ThetaDev) * nb, hipMemcpyHostToDevice, st));
  if (ev) HIPCHK(hipEventRecord(p->ev[0], st));
  if (mixed) {
    float* L = (float*)b.d_L;
    // pairs are ordered subset by subset (LPT), nb theta slots each: the
    // pairs of each schedule group take that group's shape, as in pcv_eval
    for (int k = 0; k < n_sched(p); ++k) {
      const pcv_group& SG = sched(p, k);
      const int32_t a = SG.o0 * nb, e = std::min(pl.n_order, (SG.o0 + SG.cnt) * nb);
      const int32_t ck = factor_chunk(p, e - a);
      for (int32_t c0 = a; c0 < e; c0 += ck) {
        HIPCHK(launch_potrf_f32(Lc, pl.d_order + c0, std::min(ck, e - c0), sched_npad(p, k), p->d_px32, p->d_py32,
                                p->d_pv32, b.d_z, L, b.d_Inv, b.d_logdet, b.d_status, nullptr,
                                p->tune_small_npad));
        HIPCHK(pace());
      }
    }
    if (ev) HIPCHK(hipEventRecord(p->ev[1], st));
    HIPCHK(launch_trsv_bwd_f32(Lc, pl.d_order, pl.n_order, p->max_npad, L, b.d_Inv, b.d_z, b.d_alpha, nullptr));
    HIPCHK(pace());
    if (ev) HIPCHK(hipEventRecord(p->ev[2], st));
    for (int it = 0; it < sweeps; ++it) {
      const int32_t* gate = it > 0 ? b.d_gate : nullptr;
      if (it > 0) {
        HIPCHK(launch_refine_gate(st, pl.n_order, pl.d_order, p->S, it, b.d_rhs2, p->d_ynorm2, p->opt.refine_tol,
                                  b.d_gate, b.d_nsweep));
        HIPCHK(pace());
      }
      HIPCHK(launch_residual(Lc, pl.d_tile_items, pl.n_tile, pl.d_row_items, pl.n_row, p->d_tx, p->d_ty, p->d_yT,
                             b.d_alpha, b.d_rrow, b.d_pcol, b.d_r, gate));
      HIPCHK(pace());
      HIPCHK(launch_trsv_fwd_f32(Lc, pl.d_order, pl.n_order, p->max_npad, L, b.d_Inv, nullptr, b.d_r, b.d_z,
                                 b.d_rhs2, gate));
      HIPCHK(pace());
      HIPCHK(launch_trsv_bwd_f32(Lc, pl.d_order, pl.n_order, p->max_npad, L, b.d_Inv, b.d_z, b.d_x, b.d_alpha,
                                 gate));
      HIPCHK(pace());
    }
  } else {
    double* L = (double*)b.d_L;
    for (int32_t c0 = 0; c0 < pl.n_order; c0 += chunk) {
      HIPCHK(launch_potrf_f64(Lc, pl.d_order + c0, std::min(chunk, pl.n_order - c0), p->d_px64, p->d_py64,
                              p->d_pv64, b.d_z, L, b.d_Inv, b.d_logdet, b.d_status));
      HIPCHK(pace());
    }
    if (ev) HIPCHK(hipEventRecord(p->ev[1], st));
    HIPCHK(launch_trsv_bwd_f64(Lc, pl.d_order, pl.n_order, p->max_npad, L, b.d_Inv, b.d_z, b.d_alpha, nullptr));
    HIPCHK(pace());
    if (ev) HIPCHK(hipEventRecord(p->ev[2], st));
  }
  if (ev) HIPCHK(hipEventRecord(p->ev[3], st));
  HIPCHK(launch_predict_val(Lc, pl.d_val_items, pl.n_val, p->d_tx, p->d_ty, p->d_vx, p->d_vy, p->d_yV, b.d_alpha,
                            b.d_yhat, b.d_err));
  HIPCHK(pace());
  if (ev) HIPCHK(hipEventRecord(p->ev[4], st));
  HIPCHK(launch_reduce(st, b.d_desc, p->S, nb, b.d_err, b.d_status, p->d_active, sweeps > 0 ? b.d_rhs2 : nullptr,
                       p->d_ynorm2, p->opt.refine_tol, b.d_sspe, b.d_total, b.d_nbad));
  if (ev) HIPCHK(hipEventRecord(p->ev[5], st));
  HIPCHK(hipMemcpyAsync(b.h_total, b.d_total, sizeof(double) * nb, hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(b.h_nbad, b.d_nbad, sizeof(int32_t) * nb, hipMemcpyDeviceToHost, st));
  return PCV_OK;
}

}  // namespace

pcv_status eval_batch_impl(pcv_problem* p, int32_t K, const pcv_theta* thetas, double* losses,
                           pcv_eval_report* rep, double* zs) {
  const double t0 = now_s();
  HIPCHK(hipSetDevice(p->device));
  if (rep) {
    rep->ms_factor = rep->ms_solve = rep->ms_refine = rep->ms_predict = rep->ms_reduce = 0.0;
    rep->ms_factor_all = 0.0;
    rep->n_factor_first = p->n_active;
    rep->n_coop_subsets = 0;
    rep->n_fallback_fp64 = 0;
    rep->n_val = p->n_val_total;
    rep->n_subsets_used = p->n_active;
    rep->est_rel_err = p->opt.prec == PCV_PREC_MIXED ? -1.0 : 0.0;
  }
  const bool mixed = p->opt.prec == PCV_PREC_MIXED;
  const int sweeps = mixed ? p->opt.max_refine : 0;
  // theta slots that fit the batch budget (the cap, else 16 GiB), at most 64
  const size_t slot = batch_slot_bytes(p, mixed);
  size_t budget = (size_t)16 << 30;
  if (p->opt.mem_cap_bytes) budget = p->opt.mem_cap_bytes > p->dev_bytes ? p->opt.mem_cap_bytes - p->dev_bytes : 0;
  int B = (int)std::min<size_t>({(size_t)64, (size_t)K, budget / std::max<size_t>(slot, 1)});
  if (p->batch.B > 0) B = std::min(std::max(B, 1), p->batch.B);
  // theta values k0.. one at a time
  auto singles = [&](int32_t k0) -> pcv_status {
    for (int32_t k = k0; k < K; ++k) {
      pcv_eval_report r1;
      std::memset(&r1, 0, sizeof(r1));
      r1.per_subset_sspe = zs ? zs + (size_t)k * p->S : nullptr;
      pcv_status s = eval_impl(p, thetas[k], &losses[k], (rep || zs) ? &r1 : nullptr);
      if (s != PCV_OK) return s;
      if (rep) {
        rep->ms_factor += r1.ms_factor;
        rep->ms_solve += r1.ms_solve;
        rep->ms_refine += r1.ms_refine;
        rep->ms_predict += r1.ms_predict;
        rep->ms_reduce += r1.ms_reduce;
        rep->ms_factor_all += r1.ms_factor_all;
        rep->n_factor_first = r1.n_factor_first;
        rep->n_coop_subsets = r1.n_coop_subsets;
        rep->n_fallback_fp64 += r1.n_fallback_fp64;
      }
    }
    if (rep) rep->seconds = now_s() - t0;
    return PCV_OK;
  };
  if (K < 2 || B < 2 || p->n_active == 0) return singles(0);
  // a workspace or plan that does not fit the memory cap (or the device)
  // leaves nothing behind, and the theta values go one at a time
  pcv_status s = ensure_batch(p, B, mixed);
  if (s == PCV_ERR_OOM) return singles(0);
  if (s != PCV_OK) return s;
  pcv_batch& b = p->batch;
  for (int32_t g0 = 0; g0 < K; g0 += B) {
    const int nb = std::min(B, K - g0);
    for (int t = 0; t < nb; ++t) {
      const pcv_theta& th = thetas[g0 + t];
      ThetaDev& h = b.h_theta[t];
      h.cov = th.cov;
      h.pad = 0;
      h.range = th.range;
      h.inv_range = 1.0 / th.range;
      h.lambda = th.lambda;
      h.sigma2 = th.sigma2;
    }
    pcv_batch_plan* pl = nullptr;
    if ((s = batch_plan(p, nb, &pl)) == PCV_ERR_OOM) return singles(g0);
    if (s != PCV_OK) return s;
    const bool ev = p->events && rep;
    if (p->opt.graph && !ev && !p->served) {
      if (!pl->graph) {
        hipStream_t cs = nullptr;
        HIPCHK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
          s = enqueue_batch(p, *pl, cs, mixed, sweeps, false);
          e = hipStreamEndCapture(cs, &g);
        }
        if (s == PCV_OK && e == hipSuccess) e = hipGraphInstantiate(&pl->graph, g, nullptr, nullptr, 0);
        if (g) (void)hipGraphDestroy(g);
        (void)hipStreamDestroy(cs);
        if (s != PCV_OK) return s;
        if (e != hipSuccess) {
          pl->graph = nullptr;
          (void)hipGetLastError();
          return fail(PCV_ERR_DEVICE, std::string("batch graph: ") + hipGetErrorString(e));
        }
      }
      HIPCHK(hipGraphLaunch(pl->graph, p->stream));
    } else {
      if ((s = enqueue_batch(p, *pl, p->stream, mixed, sweeps, ev)) != PCV_OK) return s;
    }
    HIPCHK(hipStreamSynchronize(p->stream));
    if (ev) {
      float ms[5];
      for (int k = 0; k < 5; ++k) HIPCHK(hipEventElapsedTime(&ms[k], p->ev[k], p->ev[k + 1]));
      rep->ms_factor += ms[0];
      rep->ms_factor_all += ms[0];
      rep->ms_solve += ms[1];
      rep->ms_refine += ms[2];
      rep->ms_predict += ms[3];
      rep->ms_reduce += ms[4];
    }
    if (zs)
      HIPCHK(hipMemcpy(zs + (size_t)g0 * p->S, b.d_sspe, sizeof(double) * (size_t)nb * p->S,
                       hipMemcpyDeviceToHost));
    for (int t = 0; t < nb; ++t) {
      if (b.h_nbad[t] > 0 || (mixed && (p->opt.debug_flags & 1))) {
        // a subset broke down or did not converge: this theta goes through
        // the single evaluation, which re-runs those subsets in FP64
        pcv_eval_report r1;
        std::memset(&r1, 0, sizeof(r1));
        r1.per_subset_sspe = zs ? zs + (size_t)(g0 + t) * p->S : nullptr;
        s = eval_impl(p, thetas[g0 + t], &losses[g0 + t], zs ? &r1 : nullptr);
        if (s != PCV_OK) return s;
        if (rep) ++rep->n_fallback_fp64;
      } else {
        losses[g0 + t] = b.h_total[t];
      }
    }
  }
  if (rep) rep->seconds = now_s() - t0;
  return PCV_OK;
}

pcv_status factor_impl(pcv_problem* p, const pcv_theta* th, bool local) {
  HIPCHK(hipSetDevice(p->device));
  p->factored = false;
  pcv_status s = PCV_OK;
  if (!p->d_Lf) {
    if ((s = dalloc(p, &p->d_Lf, (size_t)p->nL)) != PCV_OK) return s;
    if ((s = dalloc(p, &p->d_Invf, (size_t)p->nInv)) != PCV_OK) return s;
    if ((s = dalloc(p, &p->d_alpha_fact, (size_t)p->nP)) != PCV_OK) return s;
    if ((s = dalloc(p, &p->d_zf, (size_t)p->nP)) != PCV_OK) return s;
    if ((s = dalloc(p, &p->d_logdetf, (size_t)p->S)) != PCV_OK) return s;
    if ((s = dalloc(p, &p->d_statusf, (size_t)p->S)) != PCV_OK) return s;
    if ((s = dalloc(p, &p->d_theta_fact, (size_t)p->S)) != PCV_OK) return s;
  }
  // one theta for every subset (slot 0), or subset i's own theta in slot i
  if (local && !p->d_desc_local) {
    std::vector<SubsetDesc> dl = p->desc;
    for (int32_t i = 0; i < p->S; ++i) dl[i].th = i;
    if ((s = upload(p, &p->d_desc_local, dl)) != PCV_OK) return s;
  }
  const int nth = local ? p->S : 1;
  std::vector<ThetaDev> h(nth);
  for (int k = 0; k < nth; ++k) {
    h[k].cov = th[k].cov;
    h[k].pad = 0;
    h[k].range = th[k].range;
    h[k].inv_range = 1.0 / th[k].range;
    h[k].lambda = th[k].lambda;
    h[k].sigma2 = th[k].sigma2;
  }
  HIPCHK(hipMemcpyAsync(p->d_theta_fact, h.data(), sizeof(ThetaDev) * nth, hipMemcpyHostToDevice, p->stream));
  p->d_desc_fact = local ? p->d_desc_local : p->d_desc;
  const int count = (int)p->order_all.size();
  s = factor_solve64(p, p->d_desc_fact, p->d_theta_fact, p->d_order_all, count, p->d_Lf, p->d_Invf, p->d_zf,
                     p->d_alpha_fact, p->d_logdetf, p->d_statusf);
  if (s != PCV_OK) return s;
  std::vector<int32_t> status(p->S);
  HIPCHK(hipMemcpyAsync(status.data(), p->d_statusf, sizeof(int32_t) * p->S, hipMemcpyDeviceToHost, p->stream));
  HIPCHK(hipStreamSynchronize(p->stream));
  for (int32_t i : p->order_all)
    if (status[i]) return fail(PCV_ERR_NOT_PD, "subset " + std::to_string(i) + " is not positive definite in FP64");
  p->fact_theta = th[0];
  p->factored = true;
  return PCV_OK;
}

pcv_status gls_impl(pcv_problem* p, int32_t ncov, const double* X, double* beta, int32_t* status_out) {
  HIPCHK(hipSetDevice(p->device));
  const int64_t nP = p->nP;
  // covariates of every training membership, gathered into the padded layout
  std::vector<double> Xp((size_t)ncov * nP, 0.0);
  for (int32_t i = 0; i < p->S; ++i) {
    const SubsetDesc& d = p->desc[i];
    for (int64_t j = p->train_ptr[i], a = 0; j < p->train_ptr[i + 1]; ++j, ++a)
      for (int c = 0; c < ncov; ++c) Xp[(size_t)c * nP + d.offP + a] = X[(int64_t)p->train_idx[j] * ncov + c];
  }
  double *d_X = nullptr, *d_W = nullptr, *d_beta = nullptr;
  int32_t* d_st = nullptr;
  const int count = (int)p->order_all.size();
  Launch Lc{p->stream, p->d_desc_fact, p->d_theta_fact};
  hipError_t e = hipMalloc((void**)&d_X, sizeof(double) * Xp.size());
  if (e == hipSuccess) e = hipMalloc((void**)&d_W, sizeof(double) * Xp.size());
  if (e == hipSuccess) e = hipMalloc((void**)&d_beta, sizeof(double) * (size_t)p->S * ncov);
  if (e == hipSuccess) e = hipMalloc((void**)&d_st, sizeof(int32_t) * p->S);
  if (e == hipSuccess) e = hipMemcpyAsync(d_X, Xp.data(), sizeof(double) * Xp.size(), hipMemcpyHostToDevice, p->stream);
  if (e == hipSuccess) e = hipMemsetAsync(d_W, 0, sizeof(double) * Xp.size(), p->stream);
  // W = M^{-1} X column by column through the resident FP64 factors
  for (int c = 0; c < ncov && e == hipSuccess; ++c) {
    e = launch_trsv_fwd_f64(Lc, p->d_order_all, count, p->max_npad, p->d_Lf, p->d_Invf, nullptr,
                            d_X + (size_t)c * nP, p->d_zf, nullptr);
    if (e == hipSuccess)
      e = launch_trsv_bwd_f64(Lc, p->d_order_all, count, p->max_npad, p->d_Lf, p->d_Invf, p->d_zf,
                              d_W + (size_t)c * nP, nullptr);
  }
  if (e == hipSuccess)
    e = launch_gls(p->stream, p->d_desc_fact, p->d_order_all, count, ncov, nP, d_X, d_W, p->d_alpha_fact, d_beta,
                   d_st);
  std::vector<double> hb((size_t)p->S * ncov);
  std::vector<int32_t> hs(p->S);
  if (e == hipSuccess)
    e = hipMemcpyAsync(hb.data(), d_beta, sizeof(double) * hb.size(), hipMemcpyDeviceToHost, p->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(hs.data(), d_st, sizeof(int32_t) * p->S, hipMemcpyDeviceToHost, p->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
  for (void* b : {(void*)d_X, (void*)d_W, (void*)d_beta, (void*)d_st}) (void)hipFree(b);
  if (e != hipSuccess) {
    (void)hipGetLastError();  // a failed allocation must not surface at a later launch
    return fail(e == hipErrorOutOfMemory ? PCV_ERR_OOM : PCV_ERR_DEVICE, std::string("gls: ") + hipGetErrorString(e));
  }
  // subsets without training points have no estimate
  std::vector<char> has(p->S, 0);
  for (int32_t i : p->order_all) has[i] = 1;
  for (int32_t i = 0; i < p->S; ++i) {
    for (int c = 0; c < ncov; ++c) beta[(int64_t)i * ncov + c] = has[i] ? hb[(size_t)i * ncov + c] : __builtin_nan("");
    if (status_out) status_out[i] = has[i] ? hs[i] : -1;
  }
  return PCV_OK;
}

pcv_status predict_impl(pcv_problem* p, int64_t q, const double* ql, double* mean, double* var,
                        int32_t obs_noise, int32_t* owner_out, bool dev_out) {
  HIPCHK(hipSetDevice(p->device));
  if (q == 0) return PCV_OK;
  std::vector<int32_t> owner(q);
  route(p, q, ql, owner.data());
  if (owner_out && !dev_out) std::copy(owner.begin(), owner.end(), owner_out);
  KrigePlan P;
  const int32_t flag = (var ? KRIGE_VAR : 0) | (obs_noise ? KRIGE_OBS_NOISE : 0);
  plan_krige(p, q, ql, owner.data(), nullptr, flag, P);
  // transient device buffers for this request
  double *d_qx = nullptr, *d_qy = nullptr, *d_mean = nullptr, *d_var = nullptr, *d_W = nullptr;
  int32_t *d_qorig = nullptr, *d_qflag = nullptr;
  KrigeItem* d_items = nullptr;
  const size_t ni = P.items.size();
  hipError_t e = hipSuccess;
  if (e == hipSuccess) e = hipMalloc((void**)&d_qx, sizeof(double) * q);
  if (e == hipSuccess) e = hipMalloc((void**)&d_qy, sizeof(double) * q);
  if (e == hipSuccess) e = hipMalloc((void**)&d_mean, sizeof(double) * q);
  if (e == hipSuccess) e = hipMalloc((void**)&d_var, sizeof(double) * q);
  if (e == hipSuccess) e = hipMalloc((void**)&d_qorig, sizeof(int32_t) * q);
  if (e == hipSuccess) e = hipMalloc((void**)&d_qflag, sizeof(int32_t) * q);
  if (e == hipSuccess) e = hipMalloc((void**)&d_items, sizeof(KrigeItem) * ni);
  if (e == hipSuccess && P.w_doubles) e = hipMalloc((void**)&d_W, sizeof(double) * P.w_doubles);
  if (e == hipSuccess) e = hipMemcpyAsync(d_qx, P.qx.data(), sizeof(double) * q, hipMemcpyHostToDevice, p->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(d_qy, P.qy.data(), sizeof(double) * q, hipMemcpyHostToDevice, p->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d_qorig, P.qorig.data(), sizeof(int32_t) * q, hipMemcpyHostToDevice, p->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d_qflag, P.qflag.data(), sizeof(int32_t) * q, hipMemcpyHostToDevice, p->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d_items, P.items.data(), sizeof(KrigeItem) * ni, hipMemcpyHostToDevice, p->stream);
  if (e == hipSuccess)
    e = launch_krige(p->stream, p->d_desc_fact, p->d_theta_fact, d_items, (int)ni, p->d_tx, p->d_ty, p->d_Lf,
                     p->d_Invf, p->d_alpha_fact, d_qx, d_qy, d_qorig, d_qflag, d_W, d_mean, d_var);
  const hipMemcpyKind out_kind = dev_out ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  if (e == hipSuccess) e = hipMemcpyAsync(mean, d_mean, sizeof(double) * q, out_kind, p->stream);
  if (e == hipSuccess && var) e = hipMemcpyAsync(var, d_var, sizeof(double) * q, out_kind, p->stream);
  if (e == hipSuccess && owner_out && dev_out)
    e = hipMemcpyAsync(owner_out, owner.data(), sizeof(int32_t) * q, hipMemcpyHostToDevice, p->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
  for (void* b : {(void*)d_qx, (void*)d_qy, (void*)d_mean, (void*)d_var, (void*)d_W, (void*)d_qorig,
                  (void*)d_qflag, (void*)d_items})
    (void)hipFree(b);
  if (e != hipSuccess) {
    (void)hipGetLastError();  // a failed allocation must not surface at a later launch
    return fail(e == hipErrorOutOfMemory ? PCV_ERR_OOM : PCV_ERR_DEVICE,
                std::string("predict: ") + hipGetErrorString(e));
  }
  return PCV_OK;
}

}  // namespace pcv
