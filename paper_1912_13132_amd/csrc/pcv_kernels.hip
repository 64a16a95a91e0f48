// Device kernels of one theta-evaluation of the parallel CV loss
// (Gerber & Nychka, arXiv:1912.13132).
//
//   (the factorisation k_potrf<T> lives in pcv_potrf.hip)
//   k_trsv_fwd<T>   forward substitution L z = b (FP64 accumulation)
//   k_trsv_bwd<T>   backward substitution L^T x = z, optionally alpha += x
//   k_residual      r = y_T - (Sigma + lambda I) alpha in FP64, the matrix
//                   regenerated from FP64 coordinates (refinement residual)
//   k_predict_val   kriging predictor eq. (3) at the validation points and
//                   squared errors of eq. (4), FP64
//   k_reduce        per-subset SSPE z_i and the sum of eq. (7) / Algorithm 1
//                   (fixed-order compensated FP64 sums)
#include "pcv_device.h"

namespace pcv {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename T>
struct Mfma;
// 16x16x4 MFMA.  Operands: lane i + 16 k supplies A[i][k] and B[k][i].
// Result element v of lane l sits at column l % 16 and row crow(l / 16, v):
// 4 (l/16) + v for FP32, 4 v + l/16 for FP64 (checked on gfx950).
template <>
struct Mfma<float> {
  typedef f32x4 acc_t;
  static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int crow(int lk, int v) { return 4 * lk + v; }
};
template <>
struct Mfma<double> {
  typedef f64x4 acc_t;
  static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int crow(int lk, int v) { return 4 * v + lk; }
};

// Correlation c(d) of Sec. 3 (exponential) or the Matern-3/2 member of the
// same family, t = d / theta.
__device__ __forceinline__ float corr(int cov, float d, float inv_range) {
  const float t = d * inv_range;
  const float e = expf(-t);
  return cov == 1 ? (1.0f + t) * e : e;
}
__device__ __forceinline__ double corr(int cov, double d, double inv_range) {
  const double t = d * inv_range;
  const double e = exp(-t);
  return cov == 1 ? (1.0 + t) * e : e;
}
__device__ __forceinline__ float dist(float x, float y) { return sqrtf(x * x + y * y); }
__device__ __forceinline__ double dist(double x, double y) { return sqrt(x * x + y * y); }

// 16-byte vector of T for global -> LDS staging.
template <typename T>
struct Vec16;
template <>
struct Vec16<float> {
  typedef float4 type;
  static constexpr int W = 4;
};
template <>
struct Vec16<double> {
  typedef double2 type;
  static constexpr int W = 2;
};

// K extent of one staged chunk: 128 bytes of every row.
template <typename T>
struct Tile {
  static constexpr int KC = 128 / sizeof(T);
  static constexpr int LD = KC + 1;  // padded LDS row
};

// ---------------------------------------------------------------------------
// Forward substitution L z = b, one workgroup per subset, FP64 accumulation.
// Block J: t = b_J - L[J, 0:J] z[0:J]  (each wave 16 rows, lanes over k),
//          z_J = Inv_J t.
// b is the training vector (rhs_train, length n, 0 beyond) or a padded
// vector (rhs_pad, length npad).
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_trsv_fwd(const SubsetDesc* __restrict__ desc,
                                                  const int32_t* __restrict__ order,
                                                  const T* __restrict__ Lbuf,
                                                  const double* __restrict__ Invbuf,
                                                  const double* __restrict__ rhs_train,
                                                  const double* __restrict__ rhs_pad,
                                                  double* __restrict__ zbuf,
                                                  double* __restrict__ rhs2out) {
  __shared__ double t[TB];
  __shared__ double b2s[4];
  const int sidx = order[blockIdx.x];
  const SubsetDesc D = desc[sidx];
  const int n = D.n, npad = D.npad, nb = npad / TB;
  const T* __restrict__ L = Lbuf + D.offL;
  const double* __restrict__ Inv = Invbuf + D.offInv;
  double* __restrict__ z = zbuf + D.offP;
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  double b2 = 0.0;
  for (int J = 0; J < nb; ++J) {
    const int c0 = J * TB;
    double acc[16];
#pragma unroll
    for (int rr = 0; rr < 16; ++rr) acc[rr] = 0.0;
    for (int k = l; k < c0; k += 64) {
      const double zk = z[k];
#pragma unroll
      for (int rr = 0; rr < 16; ++rr) acc[rr] += (double)L[packed_rowoff(c0 + 16 * w + rr) + k] * zk;
    }
#pragma unroll
    for (int rr = 0; rr < 16; ++rr) {
      double s = acc[rr];
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
      if (l == rr) {
        const int row = c0 + 16 * w + rr;
        double b;
        if (rhs_pad)
          b = rhs_pad[D.offP + row];
        else
          b = row < n ? rhs_train[D.offT + row] : 0.0;
        t[16 * w + rr] = b - s;
        b2 += b * b;
      }
    }
    __syncthreads();
    if (tid < TB) {
      const double* Ir = Inv + (int64_t)J * TB * TB + tid * TB;
      double s = 0.0;
      for (int j = 0; j <= tid; ++j) s += Ir[j] * t[j];
      z[c0 + tid] = s;
    }
    __syncthreads();
  }
  if (rhs2out) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) b2 += __shfl_xor(b2, off, 64);
    if (l == 0) b2s[w] = b2;
    __syncthreads();
    if (tid == 0) rhs2out[sidx] = (b2s[0] + b2s[1]) + (b2s[2] + b2s[3]);
  }
}

// ---------------------------------------------------------------------------
// Backward substitution L^T x = z, one workgroup per subset.
// Block J (descending): t = z_J - L[J+1:, J]^T x[J+1:]  (lanes over the TB
// columns, waves over rows), x_J = Inv_J^T t.  If alpha_accum is given,
// alpha += x as each block is finished.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_trsv_bwd(const SubsetDesc* __restrict__ desc,
                                                  const int32_t* __restrict__ order,
                                                  const T* __restrict__ Lbuf,
                                                  const double* __restrict__ Invbuf,
                                                  const double* __restrict__ zbuf,
                                                  double* __restrict__ xbuf,
                                                  double* __restrict__ alpha_accum) {
  __shared__ double part[4][TB];
  __shared__ double t[TB];
  const int sidx = order[blockIdx.x];
  const SubsetDesc D = desc[sidx];
  const int npad = D.npad, nb = npad / TB;
  const T* __restrict__ L = Lbuf + D.offL;
  const double* __restrict__ Inv = Invbuf + D.offInv;
  const double* __restrict__ z = zbuf + D.offP;
  double* __restrict__ x = xbuf + D.offP;
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  for (int J = nb - 1; J >= 0; --J) {
    const int c0 = J * TB;
    double acc = 0.0;
    int r = c0 + TB + w;
    for (; r + 12 < npad; r += 16) {
      const double x0 = x[r], x1 = x[r + 4], x2 = x[r + 8], x3 = x[r + 12];
      const double l0 = (double)L[packed_rowoff(r) + c0 + l];
      const double l1 = (double)L[packed_rowoff(r + 4) + c0 + l];
      const double l2 = (double)L[packed_rowoff(r + 8) + c0 + l];
      const double l3 = (double)L[packed_rowoff(r + 12) + c0 + l];
      acc += l0 * x0;
      acc += l1 * x1;
      acc += l2 * x2;
      acc += l3 * x3;
    }
    for (; r < npad; r += 4) acc += (double)L[packed_rowoff(r) + c0 + l] * x[r];
    part[w][l] = acc;
    __syncthreads();
    if (tid < TB) t[tid] = z[c0 + tid] - (part[0][tid] + part[1][tid] + part[2][tid] + part[3][tid]);
    __syncthreads();
    if (tid < TB) {
      const double* I0 = Inv + (int64_t)J * TB * TB;
      double s = 0.0;
      for (int j = tid; j < TB; ++j) s += I0[j * TB + tid] * t[j];
      x[c0 + tid] = s;
      if (alpha_accum) alpha_accum[D.offP + c0 + tid] += s;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Refinement residual r = y_T - (Sigma + lambda I) alpha in FP64, the matrix
// regenerated from FP64 coordinates.  Item = (subset, block of 64 rows);
// thread (row, phase) sums columns c = phase mod 4.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_residual(const SubsetDesc* __restrict__ desc,
                                                  const int2* __restrict__ items,
                                                  const ThetaDev* __restrict__ theta,
                                                  const double* __restrict__ tx,
                                                  const double* __restrict__ ty,
                                                  const double* __restrict__ yT,
                                                  const double* __restrict__ alphabuf,
                                                  double* __restrict__ rbuf) {
  __shared__ double red[4][64];
  const int2 it = items[blockIdx.x];
  const SubsetDesc D = desc[it.x];
  const int n = D.n;
  const int tid = threadIdx.x, q = tid >> 6, l = tid & 63;
  const int row = it.y * 64 + l;
  const int cov = theta->cov;
  const double ir = theta->inv_range, lam = theta->lambda;
  const double* __restrict__ X = tx + D.offT;
  const double* __restrict__ Y = ty + D.offT;
  const double* __restrict__ a = alphabuf + D.offP;
  double s = 0.0;
  if (row < n) {
    const double xr = X[row], yr = Y[row];
    for (int c = q; c < n; c += 4) s += corr(cov, dist(xr - X[c], yr - Y[c]), ir) * a[c];
  }
  red[q][l] = s;
  __syncthreads();
  if (q == 0 && row < D.npad) {
    double r = 0.0;
    if (row < n) r = yT[D.offT + row] - ((red[0][l] + red[1][l]) + (red[2][l] + red[3][l])) - lam * a[row];
    rbuf[D.offP + row] = r;
  }
}

// ---------------------------------------------------------------------------
// Kriging at the validation points (eq. (3)) and squared errors (eq. (4)).
// Item = (subset, block of 64 validation points).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_predict_val(const SubsetDesc* __restrict__ desc,
                                                     const int2* __restrict__ items,
                                                     const ThetaDev* __restrict__ theta,
                                                     const double* __restrict__ tx,
                                                     const double* __restrict__ ty,
                                                     const double* __restrict__ vx,
                                                     const double* __restrict__ vy,
                                                     const double* __restrict__ yV,
                                                     const double* __restrict__ alphabuf,
                                                     double* __restrict__ yhat,
                                                     double* __restrict__ err) {
  __shared__ double red[4][64];
  const int2 it = items[blockIdx.x];
  const SubsetDesc D = desc[it.x];
  const int n = D.n, m = D.m;
  const int tid = threadIdx.x, q = tid >> 6, l = tid & 63;
  const int v = it.y * 64 + l;
  const int cov = theta->cov;
  const double ir = theta->inv_range;
  const double* __restrict__ X = tx + D.offT;
  const double* __restrict__ Y = ty + D.offT;
  const double* __restrict__ a = alphabuf + D.offP;
  double s = 0.0;
  if (v < m) {
    const double xv = vx[D.offV + v], yv = vy[D.offV + v];
    for (int c = q; c < n; c += 4) s += corr(cov, dist(xv - X[c], yv - Y[c]), ir) * a[c];
  }
  red[q][l] = s;
  __syncthreads();
  if (q == 0 && v < m) {
    const double p = (red[0][l] + red[1][l]) + (red[2][l] + red[3][l]);
    const double e = p - yV[D.offV + v];
    yhat[D.offV + v] = p;
    err[D.offV + v] = e * e;
  }
}

// ---------------------------------------------------------------------------
// Per-subset SSPE and the global sum (eq. (7), Algorithm 1's final step).
// One workgroup; thread t owns subsets t, t+256, ... in index order, sums
// each subset's errors in order with Neumaier compensation, then the 256
// partial (hi, lo) pairs are combined by a fixed tree.  The result does not
// depend on launch order or batch composition.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void two_sum(double a, double b, double& s, double& e) {
  s = a + b;
  const double bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

__global__ __launch_bounds__(256) void k_reduce(const SubsetDesc* __restrict__ desc, int S,
                                                const double* __restrict__ err,
                                                const int32_t* __restrict__ status,
                                                const int32_t* __restrict__ active,
                                                double* __restrict__ per_subset,
                                                double* __restrict__ out_total,
                                                int32_t* __restrict__ out_nbad) {
  __shared__ double hi[256], lo[256];
  __shared__ int nb[256];
  const int tid = threadIdx.x;
  double th = 0.0, tl = 0.0;
  int bad = 0;
  for (int i = tid; i < S; i += 256) {
    const SubsetDesc D = desc[i];
    double zi = 0.0, zc = 0.0;
    if (active[i]) {
      for (int v = 0; v < D.m; ++v) {
        double s, e;
        two_sum(zi, err[D.offV + v], s, e);
        zi = s;
        zc += e;
      }
      if (status[i]) ++bad;
    }
    const double z = zi + zc;
    per_subset[i] = z;
    double s, e;
    two_sum(th, z, s, e);
    th = s;
    tl += e;
  }
  hi[tid] = th;
  lo[tid] = tl;
  nb[tid] = bad;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (tid < off) {
      double s, e;
      two_sum(hi[tid], hi[tid + off], s, e);
      hi[tid] = s;
      lo[tid] = lo[tid] + lo[tid + off] + e;
      nb[tid] += nb[tid + off];
    }
    __syncthreads();
  }
  if (tid == 0) {
    out_total[0] = hi[0] + lo[0];
    out_nbad[0] = nb[0];
  }
}

// ------------------------------------------------------------- launchers --
template <typename T>
static hipError_t fwd_launch(const Launch& Lc, const int32_t* order, int n_items, const T* Lbuf,
                             const double* Inv, const double* rt, const double* rp, double* z,
                             double* rhs2) {
  if (n_items <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_trsv_fwd<T>, dim3(n_items), dim3(256), 0, Lc.stream, Lc.desc, order, Lbuf, Inv,
                     rt, rp, z, rhs2);
  return hipGetLastError();
}
hipError_t launch_trsv_fwd_f32(const Launch& L, const int32_t* order, int n_items, const float* Lbuf,
                               const double* Inv, const double* rt, const double* rp, double* z,
                               double* rhs2) {
  return fwd_launch<float>(L, order, n_items, Lbuf, Inv, rt, rp, z, rhs2);
}
hipError_t launch_trsv_fwd_f64(const Launch& L, const int32_t* order, int n_items, const double* Lbuf,
                               const double* Inv, const double* rt, const double* rp, double* z,
                               double* rhs2) {
  return fwd_launch<double>(L, order, n_items, Lbuf, Inv, rt, rp, z, rhs2);
}

template <typename T>
static hipError_t bwd_launch(const Launch& Lc, const int32_t* order, int n_items, const T* Lbuf,
                             const double* Inv, const double* z, double* x, double* acc) {
  if (n_items <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_trsv_bwd<T>, dim3(n_items), dim3(256), 0, Lc.stream, Lc.desc, order, Lbuf, Inv,
                     z, x, acc);
  return hipGetLastError();
}
hipError_t launch_trsv_bwd_f32(const Launch& L, const int32_t* order, int n_items, const float* Lbuf,
                               const double* Inv, const double* z, double* x, double* acc) {
  return bwd_launch<float>(L, order, n_items, Lbuf, Inv, z, x, acc);
}
hipError_t launch_trsv_bwd_f64(const Launch& L, const int32_t* order, int n_items, const double* Lbuf,
                               const double* Inv, const double* z, double* x, double* acc) {
  return bwd_launch<double>(L, order, n_items, Lbuf, Inv, z, x, acc);
}

hipError_t launch_residual(const Launch& Lc, const int2* items, int n_items, const double* tx,
                           const double* ty, const double* yT, const double* alpha, double* r) {
  if (n_items <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_residual, dim3(n_items), dim3(256), 0, Lc.stream, Lc.desc, items, Lc.theta, tx,
                     ty, yT, alpha, r);
  return hipGetLastError();
}

hipError_t launch_predict_val(const Launch& Lc, const int2* items, int n_items, const double* tx,
                              const double* ty, const double* vx, const double* vy,
                              const double* yV, const double* alpha, double* yhat, double* err) {
  if (n_items <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_predict_val, dim3(n_items), dim3(256), 0, Lc.stream, Lc.desc, items, Lc.theta,
                     tx, ty, vx, vy, yV, alpha, yhat, err);
  return hipGetLastError();
}

hipError_t launch_reduce(hipStream_t s, const SubsetDesc* desc, int S, const double* err,
                         const int32_t* status, const int32_t* active, double* per_subset,
                         double* out_total, int32_t* out_nbad) {
  hipLaunchKernelGGL(k_reduce, dim3(1), dim3(256), 0, s, desc, S, err, status, active, per_subset,
                     out_total, out_nbad);
  return hipGetLastError();
}

}  // namespace pcv
