// Kriging of arbitrary query locations from resident FP64 factors
// (eq. (3) of arXiv:1912.13132 for the mean; the simple-kriging variance
// sigma^2 (1 - k^T (Sigma + lambda I)^{-1} k) for the uncertainty the paper
// motivates in Sec. 1 and Sec. 4.1).
//
// Item = (subset, up to KRIGE_Q queries routed to it), one workgroup of four
// waves.  The variance needs w = L^{-1} k for every query: a blocked forward
// substitution over the item's right-hand sides, with k generated on the
// fly.  For block row J, lane l owns row 64 J + l and streams that row of L
// (contiguous in the packed layout), while the four waves split the column
// blocks left of the diagonal: wave g takes blocks c = g, g+4, ... and
// multiplies them with the already solved w of those columns, staged in its
// own LDS buffer (every lane reads the same entry: a broadcast).  The four
// partial sums are combined in a fixed order, the diagonal block is solved
// with its precomputed inverse, and the solved rows go to a scratch panel
// (npad x KRIGE_Q per item) for the following block rows.  The mean k^T
// alpha uses the same k entries.  Every query is handled by fixed lanes in
// a fixed order, so its result does not depend on the other queries of its
// item.
#include "pcv_device.h"

namespace pcv {

namespace {

constexpr int KQ = KRIGE_Q;     // queries per item
constexpr int QW = KQ / 4;      // queries per wave in the row phases
constexpr int LDQ = KQ + 2;     // LDS row stride (doubles)

__device__ __forceinline__ double corr64(int cov, double d, double inv_range) {
  const double t = d * inv_range;
  const double e = exp(-t);
  return cov == 1 ? (1.0 + t) * e : e;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

}  // namespace

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
                                               const int32_t* __restrict__ qflag,
                                               double* __restrict__ Wscratch,
                                               double* __restrict__ mean,
                                               double* __restrict__ var) {
  __shared__ double Ws[4][TB * LDQ];  // per wave: staged w of one column block, then partial sums
  __shared__ double T[TB * LDQ];      // right-hand side of the diagonal block
  __shared__ double Q[2][KQ];         // query coordinates
  const KrigeItem it = items[blockIdx.x];
  const SubsetDesc D = desc[it.sidx];
  const int n = D.n, nb = D.npad / TB;
  const int tid = threadIdx.x, g = tid >> 6, l = tid & 63;
  const int cov = theta[D.th].cov;
  const double ir = theta[D.th].inv_range;
  const double* __restrict__ X = tx + D.offT;
  const double* __restrict__ Y = ty + D.offT;
  const double* __restrict__ a = alphabuf + D.offP;
  const bool want_var = (it.flags & KRIGE_VAR) != 0;
  if (tid < KQ) {
    const bool v = tid < it.nq;
    Q[0][tid] = v ? qx[it.q0 + tid] : 0.0;
    Q[1][tid] = v ? qy[it.q0 + tid] : 0.0;
  }
  __syncthreads();

  // wave g answers queries [QW g, QW g + QW) in the row phases
  double msum[QW], w2[QW];
#pragma unroll
  for (int k = 0; k < QW; ++k) msum[k] = w2[k] = 0.0;

  const double* __restrict__ L = L64 + D.offL;
  const double* __restrict__ Inv = Invbuf + D.offInv;
  double* __restrict__ W = Wscratch + it.woff;
  double* __restrict__ S = Ws[g];

  for (int J = 0; J < nb; ++J) {
    const int row = J * TB + l;
    if (want_var) {
      // partial sums of L[row][c-block] w[c-block] over this wave's blocks
      double acc[KQ];
#pragma unroll
      for (int q = 0; q < KQ; ++q) acc[q] = 0.0;
      const double* __restrict__ Lr = L + packed_rowoff(row);
      for (int c = g; c < J; c += 4) {
        const double* __restrict__ Wc = W + (int64_t)c * TB * KQ;
#pragma unroll
        for (int e = 0; e < KQ; ++e) {
          const int idx = e * 64 + l;  // element (idx / KQ, idx % KQ) of the 64 x KQ block
          S[(idx / KQ) * LDQ + idx % KQ] = Wc[idx];
        }
        __builtin_amdgcn_wave_barrier();
        const double2* __restrict__ Lc = reinterpret_cast<const double2*>(Lr + c * TB);
#pragma unroll 4
        for (int cc = 0; cc < TB / 2; ++cc) {
          const double2 lv = Lc[cc];
          const double* s0 = S + (2 * cc) * LDQ;
#pragma unroll
          for (int q = 0; q < KQ; ++q) acc[q] = fma(lv.x, s0[q], acc[q]);
#pragma unroll
          for (int q = 0; q < KQ; ++q) acc[q] = fma(lv.y, s0[LDQ + q], acc[q]);
        }
        __builtin_amdgcn_wave_barrier();
      }
#pragma unroll
      for (int q = 0; q < KQ; ++q) S[l * LDQ + q] = acc[q];
      __syncthreads();
    }
    // k for row `row` and this wave's queries; mean and right-hand side
    const bool real = row < n;
    const double xr = real ? X[row] : 0.0, yr = real ? Y[row] : 0.0, ar = real ? a[row] : 0.0;
#pragma unroll
    for (int k = 0; k < QW; ++k) {
      const int q = QW * g + k;
      double kv = 0.0;
      if (real) {
        const double dx = Q[0][q] - xr, dy = Q[1][q] - yr;
        kv = corr64(cov, sqrt(dx * dx + dy * dy), ir);
      }
      msum[k] = fma(kv, ar, msum[k]);
      if (want_var)
        T[l * LDQ + q] = kv - ((Ws[0][l * LDQ + q] + Ws[1][l * LDQ + q]) + (Ws[2][l * LDQ + q] + Ws[3][l * LDQ + q]));
    }
    if (!want_var) continue;
    __syncthreads();
    // diagonal block: w[row] = sum_{j <= l} Inv[l][j] T[j]
    const double* __restrict__ Ir = Inv + (int64_t)J * TB * TB + l * TB;
    double wv[QW];
#pragma unroll
    for (int k = 0; k < QW; ++k) wv[k] = 0.0;
    for (int j = 0; j <= l; ++j) {
      const double iv = Ir[j];
#pragma unroll
      for (int k = 0; k < QW; ++k) wv[k] = fma(iv, T[j * LDQ + QW * g + k], wv[k]);
    }
#pragma unroll
    for (int k = 0; k < QW; ++k) {
      W[(int64_t)row * KQ + QW * g + k] = wv[k];
      w2[k] = fma(wv[k], wv[k], w2[k]);
    }
    // solved rows visible to every wave before the next block row
    __syncthreads();
  }

#pragma unroll
  for (int k = 0; k < QW; ++k) {
    const int q = QW * g + k;
    const double m = wave_sum(msum[k]);
    const double s2w = wave_sum(w2[k]);
    if (l == 0 && q < it.nq) {
      const int32_t f = qflag[it.q0 + q];
      const int32_t o = qorig[it.q0 + q];
      mean[o] = m;
      if (f & KRIGE_VAR) {
        const double s2 = theta[D.th].sigma2;
        double v = s2 * (1.0 - s2w);
        if (f & KRIGE_OBS_NOISE) v += s2 * theta[D.th].lambda;
        var[o] = v;
      }
    }
  }
}

hipError_t launch_krige(hipStream_t s, const SubsetDesc* desc, const ThetaDev* theta,
                        const KrigeItem* items, int n_items, const double* tx, const double* ty,
                        const double* L64, const double* Inv, const double* alpha, const double* qx,
                        const double* qy, const int32_t* qorig, const int32_t* qflag,
                        double* Wscratch, double* mean, double* var) {
  if (n_items <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_krige, dim3(n_items), dim3(256), 0, s, desc, theta, items, tx, ty, L64, Inv,
                     alpha, qx, qy, qorig, qflag, Wscratch, mean, var);
  return hipGetLastError();
}

}  // namespace pcv
