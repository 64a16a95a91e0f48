// Division of the domain into cores and subsets on the device (Sec. 2.3
// shells, Sec. 2.4 recursive division, Algorithm 1 steps 2-3).  Input
// preparation: no part of the CV arithmetic.  The results equal the host
// partitioner's (same FP64 comparisons, same tie rules, same order):
//
//  * divide: the recursive balanced division, level by level.  Every
//    rectangle with k > 1 cores sorts the coordinates of its candidate points
//    along its split axis (two stable radix sorts over all segments: by
//    coordinate, then by segment), and one wave per
//    rectangle repeats the 64 bisection steps on the cut c that balance
//    k_r #{a < c + delta} against k_l #{a >= c - delta}; counts are found by
//    a 64-way cooperative search in the sorted segment.  Candidates of the
//    children are selected in order from the parent's (a stable select).
//  * count / subsets: each point tests the cores listed in its bucket of a
//    grid over the domain (cores widened by delta, clipped to the domain);
//    subset lists are (subset, point) pairs generated in point order and
//    stably sorted by subset, so each list is in increasing point order.
//
// Half-open rectangles [lo, hi) per axis, edges on the domain maximum closed.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "../../include/pcv.h"
#include "pcv_host.h"

namespace pcv {

namespace {

struct DevBuf {
  void* p = nullptr;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
};

#define PCHK(x)                                                                                    \
  do {                                                                                             \
    hipError_t e_ = (x);                                                                           \
    if (e_ != hipSuccess) {                                                                        \
      (void)hipGetLastError(); /* reported here, not again at a later launch */                    \
      return fail(e_ == hipErrorOutOfMemory ? PCV_ERR_OOM : PCV_ERR_DEVICE,                        \
                  std::string("partition: ") + #x + ": " + hipGetErrorString(e_));                  \
    }                                                                                              \
  } while (0)

template <typename T>
hipError_t dmalloc(DevBuf& b, T** p, size_t count) {
  hipError_t e = hipMalloc(&b.p, std::max<size_t>(count, 1) * sizeof(T));
  *p = (T*)b.p;
  return e;
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------
struct RectDev {
  double lo, hi;   // range along the split axis
  int64_t off, len;  // candidate segment
  int32_t kl, kr, axis, pad;
};

// rect id of every candidate element (segments are contiguous, sorted by offset)
__global__ void k_seg_keys(const RectDev* __restrict__ rects, int nr, const int32_t* __restrict__ cand, int64_t total,
                           const double* __restrict__ x, const double* __restrict__ y, int32_t* __restrict__ seg,
                           double* __restrict__ key) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  int a = 0, b = nr - 1;  // last rect with off <= e
  while (a < b) {
    const int m = (a + b + 1) >> 1;
    if (rects[m].off <= e) a = m;
    else b = m - 1;
  }
  seg[e] = a;
  const int32_t p = cand[e];
  key[e] = rects[a].axis == 0 ? x[p] : y[p];
}

// number of entries of the sorted a[0..tot) that are < v (one wave)
__device__ int64_t wave_count_below(const double* __restrict__ a, int64_t tot, double v) {
  const int lane = threadIdx.x & 63;
  int64_t lo = 0, hi = tot;  // a[i] < v for i < lo, a[i] >= v for i >= hi
  while (hi - lo > 64) {
    const int64_t step = (hi - lo + 63) / 64;
    const int64_t idx = lo + (int64_t)(lane + 1) * step - 1;
    const bool pr = idx < hi && a[idx] < v;
    const int k = __popcll(__ballot(pr));
    const int64_t nlo = std::min<int64_t>(lo + (int64_t)k * step, hi);
    const int64_t nhi = std::min<int64_t>(hi, lo + (int64_t)(k + 1) * step - 1);
    lo = nlo;
    hi = std::max(nhi, nlo);
  }
  const int64_t idx = lo + lane;
  const bool pr = idx < hi && a[idx] < v;
  return lo + __popcll(__ballot(pr));
}

// the cut of every rectangle (one wave each) and its children's sizes
__global__ __launch_bounds__(64) void k_bisect(const RectDev* __restrict__ rects, const double* __restrict__ sorted,
                                               double delta, double* __restrict__ cut, int64_t* __restrict__ nl,
                                               int64_t* __restrict__ nr) {
  const RectDev R = rects[blockIdx.x];
  const double* a = sorted + R.off;
  const int64_t tot = R.len;
  double b_lo = R.lo, b_hi = R.hi;
  for (int it = 0; it < 64; ++it) {
    const double mid = 0.5 * (b_lo + b_hi);
    const int64_t cl = wave_count_below(a, tot, mid + delta);
    const int64_t cr = tot - wave_count_below(a, tot, mid - delta);
    if ((int64_t)R.kr * cl - (int64_t)R.kl * cr < 0) b_lo = mid;
    else b_hi = mid;
  }
  double c = b_hi;
  if (delta <= 0.0) {
    const int64_t j = wave_count_below(a, tot, c);
    if (0 < j && j < tot) c = 0.5 * (a[j - 1] + a[j]);
  }
  c = std::min(std::max(c, R.lo), R.hi);
  const int64_t l = wave_count_below(a, tot, c + delta);
  const int64_t r = tot - wave_count_below(a, tot, c - delta);
  if ((threadIdx.x & 63) == 0) {
    cut[blockIdx.x] = c;
    nl[blockIdx.x] = l;
    nr[blockIdx.x] = r;
  }
}

// flags of the candidates that go to the left / right child (0 for leaves)
__global__ void k_child_flags(const RectDev* __restrict__ rects, const double* __restrict__ cut, double delta,
                              const int32_t* __restrict__ seg, const double* __restrict__ key, int64_t total,
                              uint8_t* __restrict__ fl, uint8_t* __restrict__ fr) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const int s = seg[e];
  const RectDev R = rects[s];
  const double c = cut[s], v = key[e];
  fl[e] = (R.kl > 1 && v < c + delta) ? 1 : 0;
  fr[e] = (R.kr > 1 && v >= c - delta) ? 1 : 0;
}

__device__ __forceinline__ bool in_rect(double x, double y, const double* r, double xmax, double ymax) {
  return x >= r[0] && (x < r[2] || (x == r[2] && r[2] >= xmax)) && y >= r[1] &&
         (y < r[3] || (y == r[3] && r[3] >= ymax));
}

struct GridDev {
  double x0, y0, dx, dy;
  int32_t g, pad;
};

__device__ __forceinline__ int bucket_of(const GridDev& G, double x, double y) {
  const int bx = min(G.g - 1, max(0, (int)floor((x - G.x0) / G.dx)));
  const int by = min(G.g - 1, max(0, (int)floor((y - G.y0) / G.dy)));
  return by * G.g + bx;
}

// Per point: owner (lowest-index core holding it) and the number of training
// memberships (own core unless held out, plus the shells holding it unless
// held out); with `pairs`, also the (subset, point) pairs at `pos`.
__global__ void k_members(int64_t n, const double* __restrict__ x, const double* __restrict__ y,
                          const double* __restrict__ core, const double* __restrict__ big, GridDev G,
                          const int32_t* __restrict__ bptr, const int32_t* __restrict__ blist, double xmax,
                          double ymax, const uint8_t* __restrict__ is_val, int32_t* __restrict__ owner,
                          int32_t* __restrict__ cnt, const int64_t* __restrict__ pos, int32_t* __restrict__ key,
                          int32_t* __restrict__ val) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const double px = x[p], py = y[p];
  const int b = bucket_of(G, px, py);
  int own = -1;
  for (int32_t k = bptr[b]; k < bptr[b + 1]; ++k) {
    const int32_t i = blist[k];
    if (in_rect(px, py, core + 4 * i, xmax, ymax) && (own < 0 || i < own)) own = i;
  }
  const bool v = is_val && is_val[p];
  int c = 0;
  int64_t w = pos ? pos[p] : 0;
  // subsets in increasing index: the own core is one of the listed cores
  for (int32_t k = bptr[b]; k < bptr[b + 1]; ++k) {
    const int32_t i = blist[k];
    const bool mem = (i == own) || (in_rect(px, py, big + 4 * i, xmax, ymax) && !in_rect(px, py, core + 4 * i, xmax, ymax));
    if (mem && !v) {
      if (key) {
        key[w] = i;
        val[w] = (int32_t)p;
        ++w;
      }
      ++c;
    }
  }
  if (owner) owner[p] = own;
  if (cnt) cnt[p] = c;
}

// first index of value i in the sorted keys, for i = 0..S
__global__ void k_ptr_from_keys(const int32_t* __restrict__ keys, int64_t total, int S, int64_t* __restrict__ ptr) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i > S) return;
  int64_t a = 0, b = total;
  while (a < b) {
    const int64_t m = (a + b) >> 1;
    if (keys[m] < i) a = m + 1;
    else b = m;
  }
  ptr[i] = a;
}

// ---------------------------------------------------------------------------
// host helpers
// ---------------------------------------------------------------------------
// Bucket grid over the domain listing, per bucket, the cores whose widened
// rectangle touches it (cores in increasing index order).
void build_grid(const double* big, int S, double xmin, double ymin, double xmax, double ymax, int64_t n, GridDev& G,
                std::vector<int32_t>& bptr, std::vector<int32_t>& blist) {
  const int g = std::max(1, std::min(1024, (int)std::sqrt((double)S) * 2));
  G.g = g;
  G.x0 = xmin;
  G.y0 = ymin;
  G.dx = (xmax - xmin) / g;
  G.dy = (ymax - ymin) / g;
  if (!(G.dx > 0)) G.dx = 1.0;
  if (!(G.dy > 0)) G.dy = 1.0;
  std::vector<std::vector<int32_t>> bk((size_t)g * g);
  auto bx = [&](double v) { return std::min(g - 1, std::max(0, (int)std::floor((v - G.x0) / G.dx))); };
  auto by = [&](double v) { return std::min(g - 1, std::max(0, (int)std::floor((v - G.y0) / G.dy))); };
  for (int i = 0; i < S; ++i) {
    const double* r = big + 4 * i;
    for (int yy = by(r[1]); yy <= by(r[3]); ++yy)
      for (int xx = bx(r[0]); xx <= bx(r[2]); ++xx) bk[(size_t)yy * g + xx].push_back(i);
  }
  bptr.assign((size_t)g * g + 1, 0);
  for (size_t b = 0; b < bk.size(); ++b) bptr[b + 1] = bptr[b] + (int32_t)bk[b].size();
  blist.clear();
  for (auto& v : bk) blist.insert(blist.end(), v.begin(), v.end());
  (void)n;
}

struct Geometry {
  std::vector<double> big;
  double xmin, ymin, xmax, ymax;
};

Geometry widen(const double* R, int S, double delta) {
  Geometry g;
  g.xmin = g.ymin = INFINITY;
  g.xmax = g.ymax = -INFINITY;
  for (int i = 0; i < S; ++i) {
    g.xmin = std::min(g.xmin, R[4 * i]);
    g.ymin = std::min(g.ymin, R[4 * i + 1]);
    g.xmax = std::max(g.xmax, R[4 * i + 2]);
    g.ymax = std::max(g.ymax, R[4 * i + 3]);
  }
  g.big.resize(4 * (size_t)S);
  for (int i = 0; i < S; ++i) {
    if (delta > 0) {
      g.big[4 * i] = std::max(R[4 * i] - delta, g.xmin);
      g.big[4 * i + 1] = std::max(R[4 * i + 1] - delta, g.ymin);
      g.big[4 * i + 2] = std::min(R[4 * i + 2] + delta, g.xmax);
      g.big[4 * i + 3] = std::min(R[4 * i + 3] + delta, g.ymax);
    } else {  // no shells: the widened rectangle is the core
      for (int k = 0; k < 4; ++k) g.big[4 * i + k] = R[4 * i + k];
    }
  }
  return g;
}

// Coordinates on the device, split by axis.
pcv_status upload_xy(int64_t n, const double* locs, DevBuf& bx, DevBuf& by, double** dx, double** dy) {
  std::vector<double> hx(n), hy(n);
  for (int64_t i = 0; i < n; ++i) {
    hx[i] = locs[2 * i];
    hy[i] = locs[2 * i + 1];
  }
  PCHK(dmalloc(bx, dx, n));
  PCHK(dmalloc(by, dy, n));
  PCHK(hipMemcpy(*dx, hx.data(), 8 * n, hipMemcpyHostToDevice));
  PCHK(hipMemcpy(*dy, hy.data(), 8 * n, hipMemcpyHostToDevice));
  return PCV_OK;
}

}  // namespace

pcv_status part_divide(int64_t n, const double* locs, const double* domain, int32_t m, double delta,
                       double* core_rect) {
  DevBuf bxb, byb;
  double *dx = nullptr, *dy = nullptr;
  pcv_status s = upload_xy(n, locs, bxb, byb, &dx, &dy);
  if (s != PCV_OK) return s;
  struct HostRect {
    double r[4];
    int32_t k, axis, base;
  };
  // level state: rectangles with k > 1 and their candidate segments
  std::vector<HostRect> level;
  std::vector<int64_t> off;
  if (m == 1) {
    for (int k = 0; k < 4; ++k) core_rect[k] = domain[k];
    return PCV_OK;
  }
  level.push_back(HostRect{{domain[0], domain[1], domain[2], domain[3]}, m, 0, 0});
  off = {0, n};
  DevBuf candb;
  int32_t* cand = nullptr;
  PCHK(dmalloc(candb, &cand, n));
  {
    std::vector<int32_t> all(n);
    for (int64_t i = 0; i < n; ++i) all[i] = (int32_t)i;
    PCHK(hipMemcpy(cand, all.data(), 4 * n, hipMemcpyHostToDevice));
  }
  int64_t total = n;
  while (!level.empty()) {
    const int nr = (int)level.size();
    std::vector<RectDev> hr(nr);
    for (int i = 0; i < nr; ++i) {
      const HostRect& R = level[i];
      hr[i].lo = R.r[R.axis];
      hr[i].hi = R.r[R.axis + 2];
      hr[i].off = off[i];
      hr[i].len = off[i + 1] - off[i];
      hr[i].kl = R.k / 2;
      hr[i].kr = R.k - R.k / 2;
      hr[i].axis = R.axis;
      hr[i].pad = 0;
    }
    DevBuf rb, segb, keyb, sortb, cutb, nlb, nrb, flb, frb, tmpb, outb, cntb;
    RectDev* drect;
    int32_t* seg;
    double *key, *sorted, *cut;
    int64_t *dnl, *dnr;
    uint8_t *fl, *fr;
    PCHK(dmalloc(rb, &drect, nr));
    PCHK(hipMemcpy(drect, hr.data(), sizeof(RectDev) * nr, hipMemcpyHostToDevice));
    PCHK(dmalloc(segb, &seg, total));
    PCHK(dmalloc(keyb, &key, total));
    PCHK(dmalloc(sortb, &sorted, total));
    PCHK(dmalloc(cutb, &cut, nr));
    PCHK(dmalloc(nlb, &dnl, nr));
    PCHK(dmalloc(nrb, &dnr, nr));
    PCHK(dmalloc(flb, &fl, total));
    PCHK(dmalloc(frb, &fr, total));
    const int TPB = 256;
    const unsigned blocks = (unsigned)((total + TPB - 1) / TPB);
    if (total > 0) hipLaunchKernelGGL(k_seg_keys, dim3(blocks), dim3(TPB), 0, 0, drect, nr, cand, total, dx, dy, seg, key);
    PCHK(hipGetLastError());
    // keys sorted within their segments: a global sort by coordinate, then a
    // stable global sort by segment (radix sorts are stable)
    DevBuf k2b, s2b, s3b, tmpb2;
    double* key2;
    int32_t *seg2, *seg3;
    PCHK(dmalloc(k2b, &key2, total));
    PCHK(dmalloc(s2b, &seg2, total));
    PCHK(dmalloc(s3b, &seg3, total));
    size_t tb = 0, tbb = 0;
    PCHK(hipcub::DeviceRadixSort::SortPairs(nullptr, tb, key, key2, seg, seg2, (int)total));
    PCHK(hipcub::DeviceRadixSort::SortPairs(nullptr, tbb, seg2, seg3, key2, sorted, (int)total));
    char* tmp;
    PCHK(dmalloc(tmpb, &tmp, std::max(tb, tbb)));
    tb = std::max(tb, tbb);
    if (total > 0) {
      PCHK(hipcub::DeviceRadixSort::SortPairs((void*)tmp, tb, key, key2, seg, seg2, (int)total));
      PCHK(hipcub::DeviceRadixSort::SortPairs((void*)tmp, tb, seg2, seg3, key2, sorted, (int)total));
    }
    hipLaunchKernelGGL(k_bisect, dim3(nr), dim3(64), 0, 0, drect, sorted, delta, cut, dnl, dnr);
    PCHK(hipGetLastError());
    if (total > 0)
      hipLaunchKernelGGL(k_child_flags, dim3(blocks), dim3(TPB), 0, 0, drect, cut, delta, seg, key, total, fl, fr);
    PCHK(hipGetLastError());
    std::vector<double> hc(nr);
    std::vector<int64_t> hl(nr), hrr(nr);
    PCHK(hipMemcpy(hc.data(), cut, 8 * nr, hipMemcpyDeviceToHost));
    PCHK(hipMemcpy(hl.data(), dnl, 8 * nr, hipMemcpyDeviceToHost));
    PCHK(hipMemcpy(hrr.data(), dnr, 8 * nr, hipMemcpyDeviceToHost));
    // children: leaves are written out, the others form the next level
    // (left children first, then right children, each in parent order)
    std::vector<HostRect> next;
    std::vector<int64_t> noff = {0};
    for (int side = 0; side < 2; ++side)
      for (int i = 0; i < nr; ++i) {
        const HostRect& R = level[i];
        const int kl = R.k / 2, kr = R.k - R.k / 2;
        HostRect c = R;
        c.axis = 1 - R.axis;
        if (side == 0) {
          c.r[R.axis + 2] = hc[i];
          c.k = kl;
          c.base = R.base;
        } else {
          c.r[R.axis] = hc[i];
          c.k = kr;
          c.base = R.base + kl;
        }
        if (c.k == 1) {
          for (int k = 0; k < 4; ++k) core_rect[4 * c.base + k] = c.r[k];
        } else {
          next.push_back(c);
          noff.push_back(noff.back() + (side == 0 ? hl[i] : hrr[i]));
        }
      }
    if (next.empty()) break;
    // candidates of the next level: stable selection, left pass then right
    // pass (the left children's segments come first)
    int64_t nleft = 0;
    {
      size_t nl_children = 0;
      for (int i = 0; i < nr; ++i)
        if (level[i].k / 2 > 1) ++nl_children;
      nleft = noff[nl_children];
    }
    const int64_t ntot = noff.back();
    int32_t* ncand = nullptr;
    PCHK(dmalloc(outb, &ncand, ntot));
    int64_t* dcount;
    PCHK(dmalloc(cntb, &dcount, 1));
    size_t tb2 = 0;
    PCHK(hipcub::DeviceSelect::Flagged(nullptr, tb2, cand, fl, ncand, dcount, (int)total));
    DevBuf tmp2b;
    char* tmp2;
    PCHK(dmalloc(tmp2b, &tmp2, tb2));
    if (nleft > 0) PCHK(hipcub::DeviceSelect::Flagged((void*)tmp2, tb2, cand, fl, ncand, dcount, (int)total));
    if (ntot > nleft)
      PCHK(hipcub::DeviceSelect::Flagged((void*)tmp2, tb2, cand, fr, ncand + nleft, dcount, (int)total));
    // replace the candidate array
    std::swap(candb.p, outb.p);
    cand = (int32_t*)candb.p;
    level.swap(next);
    off.swap(noff);
    total = ntot;
  }
  return PCV_OK;
}

pcv_status part_subsets(int64_t n, const double* locs, int32_t S, const double* core_rect, double delta,
                        const uint8_t* is_val, int32_t* owner, int64_t* memberships, int64_t* train_ptr,
                        int32_t* train_idx, int64_t* val_ptr, int32_t* val_idx) {
  DevBuf bxb, byb;
  double *dx = nullptr, *dy = nullptr;
  pcv_status s = upload_xy(n, locs, bxb, byb, &dx, &dy);
  if (s != PCV_OK) return s;
  Geometry geo = widen(core_rect, S, delta);
  GridDev G;
  std::vector<int32_t> bptr, blist;
  build_grid(geo.big.data(), S, geo.xmin, geo.ymin, geo.xmax, geo.ymax, n, G, bptr, blist);
  DevBuf coreb, bigb, bpb, blb, valb, ownb, cntb, posb;
  double *dcore, *dbig;
  int32_t *dbp, *dbl, *down, *dcnt;
  uint8_t* dval = nullptr;
  int64_t* dpos;
  PCHK(dmalloc(coreb, &dcore, 4 * (size_t)S));
  PCHK(dmalloc(bigb, &dbig, 4 * (size_t)S));
  PCHK(dmalloc(bpb, &dbp, bptr.size()));
  PCHK(dmalloc(blb, &dbl, blist.size()));
  PCHK(hipMemcpy(dcore, core_rect, 32 * (size_t)S, hipMemcpyHostToDevice));
  PCHK(hipMemcpy(dbig, geo.big.data(), 32 * (size_t)S, hipMemcpyHostToDevice));
  PCHK(hipMemcpy(dbp, bptr.data(), 4 * bptr.size(), hipMemcpyHostToDevice));
  if (!blist.empty()) PCHK(hipMemcpy(dbl, blist.data(), 4 * blist.size(), hipMemcpyHostToDevice));
  if (is_val) {
    PCHK(dmalloc(valb, &dval, n));
    PCHK(hipMemcpy(dval, is_val, n, hipMemcpyHostToDevice));
  }
  PCHK(dmalloc(ownb, &down, n));
  PCHK(dmalloc(cntb, &dcnt, n));
  PCHK(dmalloc(posb, &dpos, n + 1));
  const int TPB = 256;
  const unsigned blocks = (unsigned)((n + TPB - 1) / TPB);
  hipLaunchKernelGGL(k_members, dim3(blocks), dim3(TPB), 0, 0, n, dx, dy, dcore, dbig, G, dbp, dbl, geo.xmax,
                     geo.ymax, dval, down, dcnt, (const int64_t*)nullptr, (int32_t*)nullptr, (int32_t*)nullptr);
  PCHK(hipGetLastError());
  std::vector<int32_t> own(n);
  PCHK(hipMemcpy(own.data(), down, 4 * n, hipMemcpyDeviceToHost));
  for (int64_t p = 0; p < n; ++p)
    if (own[p] < 0) return fail(PCV_ERR_INVALID, "cores do not cover point " + std::to_string(p));
  if (owner) std::copy(own.begin(), own.end(), owner);
  // positions of every point's pairs
  {
    std::vector<int32_t> hc(n);
    PCHK(hipMemcpy(hc.data(), dcnt, 4 * n, hipMemcpyDeviceToHost));
    std::vector<int64_t> hp(n + 1, 0);
    for (int64_t p = 0; p < n; ++p) hp[p + 1] = hp[p] + hc[p];
    PCHK(hipMemcpy(dpos, hp.data(), 8 * (n + 1), hipMemcpyHostToDevice));
    const int64_t total = hp[n];
    // without a held-out set: every point once in its core plus its shells
    if (memberships) *memberships = total;
    if (train_ptr) {
      DevBuf kb, vb, ksb, vsb, tmpb, ptrb;
      int32_t *k, *v, *ks, *vs;
      int64_t* dptr;
      PCHK(dmalloc(kb, &k, total));
      PCHK(dmalloc(vb, &v, total));
      PCHK(dmalloc(ksb, &ks, total));
      PCHK(dmalloc(vsb, &vs, total));
      PCHK(dmalloc(ptrb, &dptr, (size_t)S + 1));
      hipLaunchKernelGGL(k_members, dim3(blocks), dim3(TPB), 0, 0, n, dx, dy, dcore, dbig, G, dbp, dbl, geo.xmax,
                         geo.ymax, dval, (int32_t*)nullptr, (int32_t*)nullptr, dpos, k, v);
      PCHK(hipGetLastError());
      size_t tb2 = 0;
      PCHK(hipcub::DeviceRadixSort::SortPairs(nullptr, tb2, k, ks, v, vs, (int)total));
      char* tmp;
      PCHK(dmalloc(tmpb, &tmp, tb2));
      PCHK(hipcub::DeviceRadixSort::SortPairs((void*)tmp, tb2, k, ks, v, vs, (int)total));
      hipLaunchKernelGGL(k_ptr_from_keys, dim3((S + 1 + 255) / 256), dim3(256), 0, 0, ks, total, S, dptr);
      PCHK(hipGetLastError());
      PCHK(hipMemcpy(train_ptr, dptr, 8 * ((size_t)S + 1), hipMemcpyDeviceToHost));
      if (train_idx) PCHK(hipMemcpy(train_idx, vs, 4 * total, hipMemcpyDeviceToHost));
    }
  }
  // validation lists: held-out points by owner, in point order
  if (val_ptr) {
    std::vector<int64_t> cnt((size_t)S + 1, 0);
    for (int64_t p = 0; p < n; ++p)
      if (is_val && is_val[p]) ++cnt[own[p] + 1];
    for (int32_t i = 0; i < S; ++i) cnt[i + 1] += cnt[i];
    std::copy(cnt.begin(), cnt.end(), val_ptr);
    if (val_idx) {
      std::vector<int64_t> at(cnt.begin(), cnt.end() - 1);
      for (int64_t p = 0; p < n; ++p)
        if (is_val && is_val[p]) val_idx[at[own[p]]++] = (int32_t)p;
    }
  }
  return PCV_OK;
}

}  // namespace pcv
