// Kriging of arbitrary query locations from resident FP64 factors
// (eq. (3) of arXiv:1912.13132 for the mean; the simple-kriging variance
// sigma^2 (1 - k^T (Sigma + lambda I)^{-1} k) for the uncertainty the paper
// motivates in Sec. 1 and Sec. 4.1).
//
// Item = (subset, up to 64 queries routed to it).  Thread (q, g): q = query
// slot, g = one of 4 row groups.  The mean sums k_c alpha_c over columns
// c = g mod 4.  The variance needs w = L^{-1} k for every query: a blocked
// forward substitution over the item's 64 right-hand sides, with the
// cross-covariance block generated on the fly and the solved rows kept in a
// scratch panel W (npad x 64).
#include "pcv_device.h"

namespace pcv {

__device__ __forceinline__ double corr64(int cov, double d, double inv_range) {
  const double t = d * inv_range;
  const double e = exp(-t);
  return cov == 1 ? (1.0 + t) * e : e;
}

__global__ __launch_bounds__(256) void k_krige(const SubsetDesc* __restrict__ desc,
                                               const ThetaDev* __restrict__ theta,
                                               const KrigeItem* __restrict__ items,
                                               const double* __restrict__ tx,
                                               const double* __restrict__ ty,
                                               const double* __restrict__ L64,
                                               const double* __restrict__ Invbuf,
                                               const double* __restrict__ alphabuf,
                                               const double* __restrict__ qx,
                                               const double* __restrict__ qy,
                                               const int32_t* __restrict__ qorig,
                                               double* __restrict__ Wscratch,
                                               double* __restrict__ mean,
                                               double* __restrict__ var, int32_t want_var,
                                               int32_t obs_noise) {
  __shared__ double red[4][64];
  __shared__ double t[TB][65];
  const KrigeItem it = items[blockIdx.x];
  const SubsetDesc D = desc[it.sidx];
  const int n = D.n, npad = D.npad, nb = npad / TB;
  const int tid = threadIdx.x, g = tid >> 6, q = tid & 63;
  const bool qv = q < it.nq;
  const int cov = theta->cov;
  const double ir = theta->inv_range;
  const double* __restrict__ X = tx + D.offT;
  const double* __restrict__ Y = ty + D.offT;
  const double* __restrict__ a = alphabuf + D.offP;
  const double xq = qv ? qx[it.q0 + q] : 0.0, yq = qv ? qy[it.q0 + q] : 0.0;

  // mean = k^T alpha
  double s = 0.0;
  if (qv)
    for (int c = g; c < n; c += 4) {
      const double dx = xq - X[c], dy = yq - Y[c];
      s += corr64(cov, sqrt(dx * dx + dy * dy), ir) * a[c];
    }
  red[g][q] = s;
  __syncthreads();
  if (g == 0 && qv) mean[qorig[it.q0 + q]] = (red[0][q] + red[1][q]) + (red[2][q] + red[3][q]);
  if (!want_var) return;

  // w = L^{-1} k, blocked by TB rows; W[k][q] row-major with 64 columns
  const double* __restrict__ L = L64 + D.offL;
  const double* __restrict__ Inv = Invbuf + D.offInv;
  double* __restrict__ W = Wscratch + it.woff;
  double w2 = 0.0;
  for (int J = 0; J < nb; ++J) {
    const int c0 = J * TB;
    double acc[16];
#pragma unroll
    for (int rr = 0; rr < 16; ++rr) {
      const int row = c0 + 16 * g + rr;
      double kv = 0.0;
      if (row < n && qv) {
        const double dx = xq - X[row], dy = yq - Y[row];
        kv = corr64(cov, sqrt(dx * dx + dy * dy), ir);
      }
      acc[rr] = kv;
    }
    for (int k = 0; k < c0; ++k) {
      const double wk = W[(int64_t)k * 64 + q];
#pragma unroll
      for (int rr = 0; rr < 16; ++rr) acc[rr] -= L[packed_rowoff(c0 + 16 * g + rr) + k] * wk;
    }
    __syncthreads();
#pragma unroll
    for (int rr = 0; rr < 16; ++rr) t[16 * g + rr][q] = acc[rr];
    __syncthreads();
    const double* I0 = Inv + (int64_t)J * TB * TB;
#pragma unroll 4
    for (int rr = 0; rr < 16; ++rr) {
      const int r = 16 * g + rr;
      double v = 0.0;
      for (int j = 0; j <= r; ++j) v += I0[r * TB + j] * t[j][q];
      W[(int64_t)(c0 + r) * 64 + q] = v;
      w2 += v * v;
    }
    __syncthreads();
  }
  red[g][q] = w2;
  __syncthreads();
  if (g == 0 && qv) {
    const double s2 = theta->sigma2;
    double v = s2 * (1.0 - ((red[0][q] + red[1][q]) + (red[2][q] + red[3][q])));
    if (obs_noise) v += s2 * theta->lambda;
    var[qorig[it.q0 + q]] = v;
  }
}

hipError_t launch_krige(hipStream_t s, const SubsetDesc* desc, const ThetaDev* theta,
                        const KrigeItem* items, int n_items, const double* tx, const double* ty,
                        const double* L64, const double* Inv, const double* alpha, const double* qx,
                        const double* qy, const int32_t* qorig, double* Wscratch, double* mean,
                        double* var, int32_t want_var, int32_t obs_noise) {
  if (n_items <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_krige, dim3(n_items), dim3(256), 0, s, desc, theta, items, tx, ty, L64, Inv,
                     alpha, qx, qy, qorig, Wscratch, mean, var, want_var, obs_noise);
  return hipGetLastError();
}

}  // namespace pcv
