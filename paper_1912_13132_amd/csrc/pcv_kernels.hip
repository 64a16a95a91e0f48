// Device kernels of one theta-evaluation of the parallel CV loss
// (Gerber & Nychka, arXiv:1912.13132).
//
//   k_potrf<T>      covariance tiles (Sec. 3 / eq. (1)) generated in registers,
//                   blocked left-looking Cholesky of Sigma + lambda I
//                   (the (Sigma + lambda I)^{-1} of eq. (3)); tile updates on
//                   MFMA in T, diagonal blocks factored and inverted in FP64
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
// Blocked left-looking Cholesky, one workgroup (4 waves) per subset.
//
// For every column block J (TB columns) and every chunk of CHUNK rows at or
// below the diagonal block, the chunk of M = Sigma + lambda I is generated in
// the MFMA accumulators, the update  - sum_{K<J} L_{rows,K} L_{J,K}^T  is
// accumulated on MFMA from LDS-staged 128-byte row segments, and:
//   - the diagonal block (wave 0 of the first chunk) goes to LDS in FP64,
//     is factored there and inverted (FP64), log-pivots summed for log det;
//   - every other row block is written back and multiplied on MFMA by the
//     transposed inverse of the diagonal factor (the panel triangular solve).
// Wave w owns rows [64w, 64w+64) of the chunk and all TB columns: 4 x 4
// accumulator tiles of 16 x 16.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256, 1) void k_potrf(const SubsetDesc* __restrict__ desc,
                                                  const int32_t* __restrict__ order,
                                                  const ThetaDev* __restrict__ theta,
                                                  const T* __restrict__ cx, const T* __restrict__ cy,
                                                  T* __restrict__ Lbuf, double* __restrict__ Invbuf,
                                                  double* __restrict__ logdet,
                                                  int32_t* __restrict__ status) {
  typedef typename Mfma<T>::acc_t acc_t;
  typedef typename Vec16<T>::type vec_t;
  constexpr int KC = Tile<T>::KC;
  constexpr int LD = Tile<T>::LD;
  constexpr int VW = Vec16<T>::W;
  constexpr int STAGE_BYTES = (CHUNK + TB) * LD * (int)sizeof(T);
  constexpr int DG_BYTES = TB * (TB + 1) * 8;
  constexpr int U_BYTES = STAGE_BYTES > DG_BYTES ? STAGE_BYTES : DG_BYTES;
  __shared__ __attribute__((aligned(16))) char smem_u[U_BYTES];
  __shared__ double InvD[TB][TB + 1];
  __shared__ double red[4][TB];

  T* As = reinterpret_cast<T*>(smem_u);       // [CHUNK][LD]
  T* Bs = As + CHUNK * LD;                     // [TB][LD]
  double(*Dg)[TB + 1] = reinterpret_cast<double(*)[TB + 1]>(smem_u);

  const int sidx = order[blockIdx.x];
  const SubsetDesc D = desc[sidx];
  const int n = D.n, npad = D.npad, nb = npad / TB;
  T* __restrict__ L = Lbuf + D.offL;
  double* __restrict__ Inv = Invbuf + D.offInv;
  const T* __restrict__ X = cx + D.offT;
  const T* __restrict__ Y = cy + D.offT;
  const int cov = theta->cov;
  const T ir = (T)theta->inv_range;
  const T lam = (T)theta->lambda;

  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  const int lr = l & 15, lk = l >> 4;
  // staging map: thread -> (row within 32-row group, 16-byte column slot)
  const int srow = tid >> 3, scol = (tid & 7) * VW;

  double ld_acc = 0.0;
  int bad = 0;

  for (int J = 0; J < nb; ++J) {
    const int c0 = J * TB;
    for (int r0 = c0; r0 < npad; r0 += CHUNK) {
      __syncthreads();  // previous chunk's writes visible, LDS free
      const int wr0 = r0 + 64 * w;
      const bool wact = wr0 < npad;
      acc_t acc[4][4];

      // ---- covariance tile: M[row][col] for the wave's 64 x TB block
      if (wact) {
#pragma unroll
        for (int bj = 0; bj < 4; ++bj) {
          const int col = c0 + 16 * bj + lr;
          const T xc = col < n ? X[col] : (T)0, yc = col < n ? Y[col] : (T)0;
#pragma unroll
          for (int bi = 0; bi < 4; ++bi) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int row = wr0 + 16 * bi + Mfma<T>::crow(lk, v);
              T val;
              if (row < n && col < n) {
                const T xr = X[row], yr = Y[row];
                val = corr(cov, dist(xr - xc, yr - yc), ir) + (row == col ? lam : (T)0);
              } else {
                val = row == col ? (T)1 : (T)0;
              }
              acc[bi][bj][v] = val;
            }
          }
        }
      }

      // ---- update: acc -= L[rows, 0:c0] * L[c0:c0+TB, 0:c0]^T
      vec_t pa[8], pb[2];
      auto prefetch = [&](int k0) {
#pragma unroll
        for (int s = 0; s < 8; ++s) {
          const int row = r0 + 32 * s + srow;
          if (row < npad)
            pa[s] = *reinterpret_cast<const vec_t*>(L + packed_rowoff(row) + k0 + scol);
          else
            pa[s] = vec_t{};
        }
#pragma unroll
        for (int s = 0; s < 2; ++s) {
          const int row = c0 + 32 * s + srow;
          pb[s] = *reinterpret_cast<const vec_t*>(L + packed_rowoff(row) + k0 + scol);
        }
      };
      if (c0 > 0) prefetch(0);
      for (int k0 = 0; k0 < c0; k0 += KC) {
        __syncthreads();
#pragma unroll
        for (int s = 0; s < 8; ++s) {
          const T* p = reinterpret_cast<const T*>(&pa[s]);
#pragma unroll
          for (int e = 0; e < VW; ++e) As[(32 * s + srow) * LD + scol + e] = -p[e];
        }
#pragma unroll
        for (int s = 0; s < 2; ++s) {
          const T* p = reinterpret_cast<const T*>(&pb[s]);
#pragma unroll
          for (int e = 0; e < VW; ++e) Bs[(32 * s + srow) * LD + scol + e] = p[e];
        }
        __syncthreads();
        if (k0 + KC < c0) prefetch(k0 + KC);
        if (wact) {
#pragma unroll
          for (int kk = 0; kk < KC / 4; ++kk) {
            T a[4], b[4];
#pragma unroll
            for (int bi = 0; bi < 4; ++bi) a[bi] = As[(64 * w + 16 * bi + lr) * LD + 4 * kk + lk];
#pragma unroll
            for (int bj = 0; bj < 4; ++bj) b[bj] = Bs[(16 * bj + lr) * LD + 4 * kk + lk];
#pragma unroll
            for (int bi = 0; bi < 4; ++bi)
#pragma unroll
              for (int bj = 0; bj < 4; ++bj) acc[bi][bj] = Mfma<T>::mma(a[bi], b[bj], acc[bi][bj]);
          }
        }
      }

      // ---- diagonal block: FP64 factor + inverse in LDS
      if (r0 == c0) {
        __syncthreads();
        if (w == 0) {
#pragma unroll
          for (int bi = 0; bi < 4; ++bi)
#pragma unroll
            for (int bj = 0; bj < 4; ++bj)
#pragma unroll
              for (int v = 0; v < 4; ++v) Dg[16 * bi + Mfma<T>::crow(lk, v)][16 * bj + lr] = (double)acc[bi][bj][v];
        }
        __syncthreads();
        for (int j = 0; j < TB; ++j) {
          if (tid == 0) {
            double d = Dg[j][j];
            if (!(d > 0.0) || !(d < 1e300)) {
              if (!bad) bad = c0 + j + 1;
              d = 1.0;
            }
            const double s = sqrt(d);
            Dg[j][j] = s;
            if (c0 + j < n) ld_acc += 2.0 * log(s);
          }
          __syncthreads();
          const double piv = Dg[j][j];
          if (tid > j && tid < TB) Dg[tid][j] /= piv;
          __syncthreads();
          const int m = TB - 1 - j;
          for (int e = tid; e < m * m; e += 256) {
            const int i = j + 1 + e / m, k = j + 1 + e % m;
            if (k <= i) Dg[i][k] -= Dg[i][j] * Dg[k][j];
          }
          __syncthreads();
        }
        // inverse of the lower-triangular factor, row by row:
        // Inv[i][c] = (delta_ic - sum_{c<=k<i} Dg[i][k] Inv[k][c]) / Dg[i][i]
        {
          const int c = tid & 63, q = tid >> 6;
          for (int i = 0; i < TB; ++i) {
            double s = 0.0;
            for (int k = c + q; k < i; k += 4) s += Dg[i][k] * InvD[k][c];
            red[q][c] = s;
            __syncthreads();
            if (q == 0) {
              double v = 0.0;
              if (c <= i) {
                const double t = (c == i ? 1.0 : 0.0) - (red[0][c] + red[1][c] + red[2][c] + red[3][c]);
                v = t / Dg[i][i];
              }
              InvD[i][c] = v;
            }
            __syncthreads();
          }
        }
        // write L_JJ (T) and Inv_J (FP64)
        for (int e = tid; e < TB * TB; e += 256) {
          const int i = e / TB, j = e % TB;
          L[packed_rowoff(c0 + i) + c0 + j] = j <= i ? (T)Dg[i][j] : (T)0;
          Inv[(int64_t)J * TB * TB + e] = InvD[i][j];
        }
      }

      // ---- panel triangular solve for the rows below the diagonal block:
      //      L[rows, J] = Aupd[rows, J] * Inv_J^T
      const bool offdiag = wact && !(r0 == c0 && w == 0);
      if (offdiag) {
#pragma unroll
        for (int bi = 0; bi < 4; ++bi)
#pragma unroll
          for (int bj = 0; bj < 4; ++bj)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int row = wr0 + 16 * bi + Mfma<T>::crow(lk, v);
              L[packed_rowoff(row) + c0 + 16 * bj + lr] = acc[bi][bj][v];
            }
      }
      const bool any_below = (r0 != c0) || (r0 + 64 < npad);
      if (any_below) {
#pragma unroll
        for (int bi = 0; bi < 4; ++bi)
#pragma unroll
          for (int bj = 0; bj < 4; ++bj) acc[bi][bj] = acc_t{};
        for (int k0 = 0; k0 < TB; k0 += KC) {
          __syncthreads();  // written rows visible; LDS free
#pragma unroll
          for (int s = 0; s < 8; ++s) {
            const int row = r0 + 32 * s + srow;
            vec_t v = vec_t{};
            if (row < npad) v = *reinterpret_cast<const vec_t*>(L + packed_rowoff(row) + c0 + k0 + scol);
            const T* p = reinterpret_cast<const T*>(&v);
#pragma unroll
            for (int e = 0; e < VW; ++e) As[(32 * s + srow) * LD + scol + e] = p[e];
          }
          __syncthreads();
          if (offdiag) {
#pragma unroll
            for (int kk = 0; kk < KC / 4; ++kk) {
              T a[4], b[4];
#pragma unroll
              for (int bi = 0; bi < 4; ++bi) a[bi] = As[(64 * w + 16 * bi + lr) * LD + 4 * kk + lk];
#pragma unroll
              for (int bj = 0; bj < 4; ++bj) b[bj] = (T)InvD[16 * bj + lr][k0 + 4 * kk + lk];
#pragma unroll
              for (int bi = 0; bi < 4; ++bi)
#pragma unroll
                for (int bj = 0; bj < 4; ++bj) acc[bi][bj] = Mfma<T>::mma(a[bi], b[bj], acc[bi][bj]);
            }
          }
        }
        __syncthreads();  // all staging reads done before overwriting
        if (offdiag) {
#pragma unroll
          for (int bi = 0; bi < 4; ++bi)
#pragma unroll
            for (int bj = 0; bj < 4; ++bj)
#pragma unroll
              for (int v = 0; v < 4; ++v) {
                const int row = wr0 + 16 * bi + Mfma<T>::crow(lk, v);
                L[packed_rowoff(row) + c0 + 16 * bj + lr] = acc[bi][bj][v];
              }
        }
      }
    }
  }
  if (tid == 0) {
    logdet[sidx] = ld_acc;
    status[sidx] = bad;
  }
}

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
static hipError_t potrf_launch(const Launch& Lc, const int32_t* order, int n_items, const T* cx,
                               const T* cy, T* Lbuf, double* Inv, double* logdet, int32_t* status) {
  if (n_items <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_potrf<T>, dim3(n_items), dim3(256), 0, Lc.stream, Lc.desc, order, Lc.theta, cx,
                     cy, Lbuf, Inv, logdet, status);
  return hipGetLastError();
}
hipError_t launch_potrf_f32(const Launch& L, const int32_t* order, int n_items, const float* cx,
                            const float* cy, float* Lbuf, double* Inv, double* logdet,
                            int32_t* status) {
  return potrf_launch<float>(L, order, n_items, cx, cy, Lbuf, Inv, logdet, status);
}
hipError_t launch_potrf_f64(const Launch& L, const int32_t* order, int n_items, const double* cx,
                            const double* cy, double* Lbuf, double* Inv, double* logdet,
                            int32_t* status) {
  return potrf_launch<double>(L, order, n_items, cx, cy, Lbuf, Inv, logdet, status);
}

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
