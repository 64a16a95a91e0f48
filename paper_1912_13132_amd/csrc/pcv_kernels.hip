// Device kernels of one theta-evaluation of the parallel CV loss
// (Gerber & Nychka, arXiv:1912.13132).
//
//   (the factorisation k_potrf<T> lives in pcv_potrf.hip)
//   k_trsv_fwd<T>   forward substitution L z = b (FP64 accumulation)
//   k_trsv_bwd<T>   backward substitution L^T x = z, optionally alpha += x
//                   (both right-looking over 64-column blocks, see below)
//   k_residual_*    r = y_T - (Sigma + lambda I) alpha in FP64, the matrix
//                   regenerated from FP64 coordinates (refinement residual;
//                   symmetric tiles, fixed-order partial sums)
//   k_refine_gate   which subsets take a refinement sweep after the first
//   k_predict_val   kriging predictor eq. (3) at the validation points and
//                   squared errors of eq. (4), FP64
//   k_subset_sspe,  per-subset SSPE z_i and the sum of eq. (7) / Algorithm 1
//   k_reduce_total  (fixed-order compensated FP64 sums)
#include <type_traits>

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
// e^{-t}, t >= 0, in FP64.  t is clamped to 740 (e^{-740} < 1e-321: such
// entries are negligible).  t = k ln 2 + f with k the integer nearest to
// t / ln 2 and |f| <= ln 2 / 2, ln 2 split into a high part with trailing
// zero bits (k ln2_hi is exact for |k| < 2^21) and a low part; e^{-f} by its
// Taylor polynomial of degree 13 (truncation below 1e-17 relative), times
// 2^{-k}.  No range checks are needed for this argument range.
__device__ __forceinline__ double exp_neg(double t) {
  constexpr double LOG2E = 1.4426950408889634074;
  constexpr double LN2_HI = 6.93147180369123816490e-01;
  constexpr double LN2_LO = 1.90821492927058770002e-10;
  t = fmin(t, 740.0);
  const double k = rint(t * LOG2E);
  const double g = -fma(-k, LN2_LO, fma(-k, LN2_HI, t));  // -f
  double p = 1.0 / 6227020800.0;                          // 1 / 13!
  p = fma(p, g, 1.0 / 479001600.0);
  p = fma(p, g, 1.0 / 39916800.0);
  p = fma(p, g, 1.0 / 3628800.0);
  p = fma(p, g, 1.0 / 362880.0);
  p = fma(p, g, 1.0 / 40320.0);
  p = fma(p, g, 1.0 / 5040.0);
  p = fma(p, g, 1.0 / 720.0);
  p = fma(p, g, 1.0 / 120.0);
  p = fma(p, g, 1.0 / 24.0);
  p = fma(p, g, 1.0 / 6.0);
  p = fma(p, g, 0.5);
  p = fma(p, g, 1.0);
  p = fma(p, g, 1.0);
  return ldexp(p, -(int)k);
}
// sqrt(x), x >= 0, in FP64: the hardware reciprocal square root estimate
// (relative error about 2^-23), one coupled Newton step for sqrt(x) and
// 1 / (2 sqrt(x)), then a residual correction.  x is raised to 1e-300
// first, so that x = 0 gives 1e-150, where e^{-d / theta} is exactly 1.
__device__ __forceinline__ double sqrt_pos(double x) {
  x = fmax(x, 1e-300);
  const double y = __builtin_amdgcn_rsq(x);
  double s = x * y, h = 0.5 * y;
  const double r = fma(-s, h, 0.5);
  s = fma(s, r, s);
  h = fma(h, r, h);
  const double d = fma(-s, s, x);
  return fma(d, h, s);
}
__device__ __forceinline__ double corr(int cov, double d, double inv_range) {
  const double t = d * inv_range;
  const double e = exp_neg(t);
  return cov == 1 ? (1.0 + t) * e : e;
}
__device__ __forceinline__ float dist(float x, float y) { return sqrtf(x * x + y * y); }
__device__ __forceinline__ double dist(double x, double y) { return sqrt_pos(x * x + y * y); }

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
// Triangular solves with the packed factor, one workgroup of 512 threads per
// subset, FP64 accumulation.  Right-looking by 64-column blocks: the 64 x 64
// inverse of the diagonal block is staged in LDS, the block's unknowns are
// formed from it, and every thread then subtracts their contribution from the
// partial sums it owns (kept in registers):
//   forward  L z = b:   the rows below the block stream their segments
//                       L[r, c0:c0+64] (256 bytes in FP32), one 16-byte
//                       part per lane, summed across lanes (see below);
//   backward L^T x = z: thread owns column quads q = tid + 512 i (columns
//                       4q..4q+3), streams L[c0+k, 4q:4q+4] for the block's
//                       64 rows (coalesced across threads).
// MR / MQ bound the rows / quads per thread (npad <= 512 MR).
// ---------------------------------------------------------------------------
constexpr int SNT = 512;

template <typename T>
struct SVec;
template <>
struct SVec<float> {
  typedef float4 type;
  static constexpr int W = 4;
};
template <>
struct SVec<double> {
  typedef double2 type;
  static constexpr int W = 2;
};

__device__ __forceinline__ void stage_inv(double (*IL)[65], const double* __restrict__ Iblk, int tid) {
  for (int e = tid; e < 2048; e += SNT) {
    const double2 v = reinterpret_cast<const double2*>(Iblk)[e];
    const int i = (2 * e) >> 6, j = (2 * e) & 63;
    IL[i][j] = v.x;
    IL[i][j + 1] = v.y;
  }
}

// Forward pass, rows below block J: LPR lanes cover one row's 64-column
// segment of L with a 16-byte load each, so one load instruction of a wave
// reads RPW whole segments (coalesced), and the segment's dot product with
// z_J is summed over the LPR lanes by a fixed butterfly.  The partial sum
// t_r of row r = RPP P + RPW w + g (pass P, wave w, lane group g) lives in
// lane P mod LPR of that group, slot P / LPR.
template <typename T, int MR>
__global__ __launch_bounds__(512, (MR <= 8 && sizeof(T) == 4) ? 4 : 2) void k_trsv_fwd(const SubsetDesc* __restrict__ desc,
                                                     const int32_t* __restrict__ order,
                                                     const T* __restrict__ Lbuf,
                                                     const double* __restrict__ Invbuf,
                                                     const double* __restrict__ rhs_train,
                                                     const double* __restrict__ rhs_pad,
                                                     double* __restrict__ zbuf,
                                                     double* __restrict__ rhs2out,
                                                     const int32_t* __restrict__ gate) {
  typedef typename SVec<T>::type vec_t;
  constexpr int VW = SVec<T>::W;
  constexpr int LPR = TB / VW;           // lanes per row segment: 16 (FP32), 32 (FP64)
  constexpr int RPW = 64 / LPR;          // row segments per wave and load
  constexpr int RPP = (SNT / 64) * RPW;  // rows per pass of the workgroup
  static_assert(RPP * LPR == SNT, "one slot covers SNT rows");
  __shared__ double IL[64][65];
  __shared__ double tJ[64], zJ[64];
  __shared__ double b2s[SNT / 64];
  const int sidx = order[blockIdx.x];
  if (gate && !gate[sidx]) return;  // a refinement sweep this subset does not take
  const SubsetDesc D = desc[sidx];
  const int n = D.n, npad = D.npad, nb = npad / TB;
  const T* __restrict__ L = Lbuf + D.offL;
  const double* __restrict__ Inv = Invbuf + D.offInv;
  double* __restrict__ z = zbuf + D.offP;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, g = lane / LPR, l = lane % LPR;
  double t[MR];
  double b2 = 0.0;
#pragma unroll
  for (int i = 0; i < MR; ++i) {
    const int row = RPP * (i * LPR + l) + RPW * w + g;
    double b = 0.0;
    if (row < npad) b = rhs_pad ? rhs_pad[D.offP + row] : (row < n ? rhs_train[D.offT + row] : 0.0);
    t[i] = b;
    b2 += b * b;
  }
  for (int J = 0; J < nb; ++J) {
    const int c0 = J * TB;
    stage_inv(IL, Inv + (int64_t)J * TB * TB, tid);
#pragma unroll
    for (int i = 0; i < MR; ++i) {
      const int row = RPP * (i * LPR + l) + RPW * w + g;
      if (row >= c0 && row < c0 + TB) tJ[row - c0] = t[i];
    }
    __syncthreads();
    if (tid < TB) {
      double s = 0.0;
      for (int j = 0; j <= tid; ++j) s += IL[tid][j] * tJ[j];
      zJ[tid] = s;
      z[c0 + tid] = s;
    }
    __syncthreads();
    double zl[VW];
#pragma unroll
    for (int u = 0; u < VW; ++u) zl[u] = zJ[VW * l + u];
    const int P0 = (c0 + TB) / RPP, P1 = npad / RPP;
#pragma unroll
    for (int i = 0; i < MR; ++i) {
      const int pa = max(P0, i * LPR), pb = min(P1, (i + 1) * LPR);
      // four passes per step, their loads issued together; a pass beyond pb
      // reloads pass P's row and its sum is dropped
#pragma unroll 1
      for (int P = pa; P < pb; P += 4) {
        vec_t v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int row = RPP * (P + k < pb ? P + k : P) + RPW * w + g;
          v[k] = *reinterpret_cast<const vec_t*>(L + packed_rowoff32(row) + c0 + VW * l);
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const T* e = reinterpret_cast<const T*>(&v[k]);
          double a = 0.0;
#pragma unroll
          for (int u = 0; u < VW; ++u) a += (double)e[u] * zl[u];
#pragma unroll
          for (int off = LPR / 2; off > 0; off >>= 1) a += __shfl_xor(a, off, 64);
          if (P + k < pb && l == P + k - i * LPR) t[i] -= a;
        }
      }
    }
    __syncthreads();
  }
  if (rhs2out) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) b2 += __shfl_xor(b2, off, 64);
    if ((tid & 63) == 0) b2s[tid >> 6] = b2;
    __syncthreads();
    if (tid == 0) {
      double s = 0.0;
      for (int k = 0; k < SNT / 64; ++k) s += b2s[k];
      rhs2out[sidx] = s;
    }
  }
}

// Backward-pass update for subsets of at most SNT padded rows (at most
// SNT / 4 column quads): RS threads share a quad, each summing TB / RS of
// the block's rows, so that a thread waits for a quarter of the loads; the
// partial sums go to red[(split * QP + quad) * 4 + u] (QP = SNT / RS).
template <typename T, int RS>
__device__ __forceinline__ void bwd_update_split(const T* __restrict__ L, int c0, int tid,
                                                 const double* __restrict__ xJ, double* __restrict__ red) {
  typedef typename std::conditional<sizeof(T) == 4, float4, double4>::type q_t;
  constexpr int QP = SNT / RS, RR = TB / RS;
  const int q = tid % QP, sp = tid / QP, c = 4 * q;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  if (c < c0) {
#pragma unroll 4
    for (int r = 0; r < RR; ++r) {
      const int k = sp * RR + r;
      const q_t v = *reinterpret_cast<const q_t*>(L + packed_rowoff32(c0 + k) + c);
      const double xr = xJ[k];
      a0 += (double)v.x * xr;
      a1 += (double)v.y * xr;
      a2 += (double)v.z * xr;
      a3 += (double)v.w * xr;
    }
  }
  double* o = red + 4 * (sp * QP + q);
  o[0] = a0;
  o[1] = a1;
  o[2] = a2;
  o[3] = a3;
}

template <typename T, int MQ>
__global__ __launch_bounds__(512, MQ <= 2 ? 4 : 2) void k_trsv_bwd(const SubsetDesc* __restrict__ desc,
                                                     const int32_t* __restrict__ order,
                                                     const T* __restrict__ Lbuf,
                                                     const double* __restrict__ Invbuf,
                                                     const double* __restrict__ zbuf,
                                                     double* __restrict__ xbuf,
                                                     double* __restrict__ alpha_accum,
                                                     const int32_t* __restrict__ gate) {
  typedef typename std::conditional<sizeof(T) == 4, float4, double4>::type q_t;
  __shared__ double IL[64][65];
  __shared__ double tJ[64], xJ[64];
  const int sidx = order[blockIdx.x];
  if (gate && !gate[sidx]) return;
  const SubsetDesc D = desc[sidx];
  const int npad = D.npad, nb = npad / TB;
  const T* __restrict__ L = Lbuf + D.offL;
  const double* __restrict__ Inv = Invbuf + D.offInv;
  const double* __restrict__ z = zbuf + D.offP;
  double* __restrict__ x = xbuf + D.offP;
  const int tid = threadIdx.x;
  double t[MQ][4];
#pragma unroll
  for (int i = 0; i < MQ; ++i) {
    const int c = 4 * (tid + SNT * i);
#pragma unroll
    for (int u = 0; u < 4; ++u) t[i][u] = c + u < npad ? z[c + u] : 0.0;
  }
  for (int J = nb - 1; J >= 0; --J) {
    const int c0 = J * TB;
    stage_inv(IL, Inv + (int64_t)J * TB * TB, tid);
#pragma unroll
    for (int i = 0; i < MQ; ++i) {
      const int c = 4 * (tid + SNT * i);
      if (c >= c0 && c < c0 + TB) {
#pragma unroll
        for (int u = 0; u < 4; ++u) tJ[c - c0 + u] = t[i][u];
      }
    }
    __syncthreads();
    if (tid < TB) {
      double s = 0.0;
      for (int i = tid; i < TB; ++i) s += IL[i][tid] * tJ[i];
      xJ[tid] = s;
      x[c0 + tid] = s;
      if (alpha_accum) alpha_accum[D.offP + c0 + tid] += s;
    }
    __syncthreads();
    if (MQ <= 2 && npad <= SNT) {
      // small subset: four threads per column quad; the partial sums reuse
      // IL (the block's inverse is no longer read) and the quad's owner
      // (thread q, slot 0) adds them in a fixed order
      constexpr int RS = 4, QP = SNT / RS;
      double* red = &IL[0][0];
      bwd_update_split<T, RS>(L, c0, tid, xJ, red);
      __syncthreads();
      if (tid < QP && 4 * tid < c0) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          double a = 0.0;
#pragma unroll
          for (int sp = 0; sp < RS; ++sp) a += red[4 * (sp * QP + tid) + u];
          t[0][u] -= a;
        }
      }
    } else {
#pragma unroll
      for (int i = 0; i < MQ; ++i) {
        const int c = 4 * (tid + SNT * i);
        if (c < c0) {
          double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
#pragma unroll 8
          for (int r = 0; r < TB; ++r) {
            const q_t v = *reinterpret_cast<const q_t*>(L + packed_rowoff32(c0 + r) + c);
            const double xr = xJ[r];
            a0 += (double)v.x * xr;
            a1 += (double)v.y * xr;
            a2 += (double)v.z * xr;
            a3 += (double)v.w * xr;
          }
          t[i][0] -= a0;
          t[i][1] -= a1;
          t[i][2] -= a2;
          t[i][3] -= a3;
        }
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Refinement residual r = y_T - (Sigma + lambda I) alpha in FP64, the matrix
// regenerated from FP64 coordinates.  Sigma is symmetric, so every entry is
// generated once: the workgroup of row block I visits tiles (I, J), J <= I
// (wave w takes J = w, w + 4, ...; lane (ri, cj) an 8 x 8 sub-tile), and
// forms both Sigma_IJ alpha_J (row sums, kept) and Sigma_IJ^T alpha_I (column
// sums for block J, written to a partial buffer).  A second kernel adds the
// partials in a fixed order, so the result does not depend on scheduling.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256, 3) void k_residual_tiles(const SubsetDesc* __restrict__ desc,
                                                        const int2* __restrict__ items,
                                                        const ThetaDev* __restrict__ theta,
                                                        const double* __restrict__ tx,
                                                        const double* __restrict__ ty,
                                                        const double* __restrict__ alphabuf,
                                                        double* __restrict__ rrow,
                                                        double* __restrict__ pcol,
                                                        const int32_t* __restrict__ gate) {
  __shared__ double red[4][64];
  const int2 it = items[blockIdx.x];
  if (gate && !gate[it.x]) return;
  const SubsetDesc D = desc[it.x];
  const int I = it.y, n = D.n;
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  const int ri = l >> 3, cj = l & 7;
  const int cov = theta[D.th].cov;
  const double ir = theta[D.th].inv_range;
  const double* __restrict__ X = tx + D.offT;
  const double* __restrict__ Y = ty + D.offT;
  const double* __restrict__ a = alphabuf + D.offP;
  double xi[8], yi[8], ai[8];
  bool vi[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int row = 64 * I + 8 * ri + u;
    vi[u] = row < n;
    const int rc = vi[u] ? row : 0;
    xi[u] = X[rc];
    yi[u] = Y[rc];
    ai[u] = vi[u] ? a[row] : 0.0;
  }
  double rowacc[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) rowacc[u] = 0.0;
  for (int J = w; J <= I; J += 4) {
    double xj[8], yj[8], aj[8];
    bool vj[8];
#pragma unroll
    for (int v = 0; v < 8; ++v) {
      const int col = 64 * J + 8 * cj + v;
      vj[v] = col < n;
      const int cc = vj[v] ? col : 0;
      xj[v] = X[cc];
      yj[v] = Y[cc];
      aj[v] = vj[v] ? a[col] : 0.0;
    }
    double rp[8], cp[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) rp[u] = cp[u] = 0.0;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
#pragma unroll
      for (int v = 0; v < 8; ++v) {
        // rows and columns beyond n carry the first point's coordinates and
        // alpha = 0, so they add exact zeros to the other side's sums (their
        // own sums are never read): no mask is needed
        const double dx = xi[u] - xj[v], dy = yi[u] - yj[v];
        const double c = corr(cov, dist(dx, dy), ir);
        rp[u] += c * aj[v];
        cp[v] += c * ai[u];
      }
      // one sub-tile row at a time: bounds the exponentials in flight
      asm volatile("" : "+v"(rp[u]), "+v"(cp[0]), "+v"(cp[1]), "+v"(cp[2]), "+v"(cp[3]), "+v"(cp[4]),
                   "+v"(cp[5]), "+v"(cp[6]), "+v"(cp[7]));
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      double t = rp[u];
      t += __shfl_xor(t, 1, 64);
      t += __shfl_xor(t, 2, 64);
      t += __shfl_xor(t, 4, 64);
      rowacc[u] += t;
    }
    if (J < I) {
#pragma unroll
      for (int v = 0; v < 8; ++v) {
        double t = cp[v];
        t += __shfl_xor(t, 8, 64);
        t += __shfl_xor(t, 16, 64);
        t += __shfl_xor(t, 32, 64);
        cp[v] = t;
      }
      if (ri == 0) {
        double* dst = pcol + D.offPC + ((int64_t)I * (I - 1) / 2 + J) * 64 + 8 * cj;
#pragma unroll
        for (int v = 0; v < 8; ++v) dst[v] = cp[v];
      }
    }
  }
  if (cj == 0) {
#pragma unroll
    for (int u = 0; u < 8; ++u) red[w][8 * ri + u] = rowacc[u];
  }
  __syncthreads();
  if (tid < 64) rrow[D.offP + 64 * I + tid] = (red[0][tid] + red[1][tid]) + (red[2][tid] + red[3][tid]);
}

// r_j = y_j - lambda alpha_j - (row sums of block J) - sum_{I > J} (column
// sums of tile (I, J)), added in increasing I.  Item = (subset, row block J).
__global__ __launch_bounds__(64) void k_residual_reduce(const SubsetDesc* __restrict__ desc,
                                                        const int2* __restrict__ items,
                                                        const ThetaDev* __restrict__ theta,
                                                        const double* __restrict__ yT,
                                                        const double* __restrict__ alphabuf,
                                                        const double* __restrict__ rrow,
                                                        const double* __restrict__ pcol,
                                                        double* __restrict__ rbuf,
                                                        const int32_t* __restrict__ gate) {
  const int2 it = items[blockIdx.x];
  if (gate && !gate[it.x]) return;
  const SubsetDesc D = desc[it.x];
  const int J = it.y, n = D.n, nb = D.npad / TB;
  const int row = 64 * J + threadIdx.x;
  double r = 0.0;
  if (row < n) {
    double s = rrow[D.offP + row];
    for (int I = J + 1; I < nb; ++I) s += pcol[D.offPC + ((int64_t)I * (I - 1) / 2 + J) * 64 + threadIdx.x];
    r = yT[D.offT + row] - theta[D.th].lambda * alphabuf[D.offP + row] - s;
  }
  rbuf[D.offP + row] = r;
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
  const int cov = theta[D.th].cov;
  const double ir = theta[D.th].inv_range;
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
    yhat[D.offE + v] = p;
    err[D.offE + v] = e * e;
  }
}

// ---------------------------------------------------------------------------
// Per-subset SSPE and the global sum (eq. (7), Algorithm 1's final step), in
// two launches.  k_subset_sspe: one wave per (theta slot, subset); lane l
// adds errors l, l + 64, ... with Neumaier compensation, then the 64 (hi, lo)
// pairs are combined by a fixed butterfly (two_sum gives the exact error in
// either operand order, so every lane ends with the same pair).
// k_reduce_total: one workgroup per theta slot; thread t adds subsets t,
// t + 256, ... in index order, then a fixed tree.  The result does not
// depend on launch order or batch composition.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void two_sum(double a, double b, double& s, double& e) {
  s = a + b;
  const double bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

__global__ __launch_bounds__(256) void k_subset_sspe(const SubsetDesc* __restrict__ desc, int S, int n_desc,
                                                     const double* __restrict__ err,
                                                     int32_t* __restrict__ status,
                                                     const int32_t* __restrict__ active,
                                                     const double* __restrict__ rhs2,
                                                     const double* __restrict__ ynorm2, double tol2,
                                                     double* __restrict__ per_subset) {
  const int k = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int l = threadIdx.x & 63;
  if (k >= n_desc) return;  // the whole wave
  const int i = k % S;
  const bool act = active[i] != 0;
  const SubsetDesc D = desc[k];
  double hi = 0.0, lo = 0.0;
  if (act)
    for (int v = l; v < D.m; v += 64) {
      double s, e;
      two_sum(hi, err[D.offE + v], s, e);
      hi = s;
      lo += e;
    }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const double oh = __shfl_xor(hi, off, 64), ol = __shfl_xor(lo, off, 64);
    double s, e;
    two_sum(hi, oh, s, e);
    hi = s;
    lo = (lo + ol) + e;
  }
  if (l == 0) {
    per_subset[k] = hi + lo;
    // a mixed-precision subset whose residual before the last correction
    // was not small enough is re-run in FP64 like a broken-down one
    if (act && rhs2 && status[k] == 0 && rhs2[k] > tol2 * ynorm2[i]) status[k] = PCV_STATUS_STAGNATED;
  }
}

__global__ __launch_bounds__(256) void k_reduce_total(int S, const int32_t* __restrict__ status,
                                                      const int32_t* __restrict__ active,
                                                      const double* __restrict__ per_subset,
                                                      double* __restrict__ out_total,
                                                      int32_t* __restrict__ out_nbad) {
  __shared__ double hi[256], lo[256];
  __shared__ int nb[256];
  const int tid = threadIdx.x;
  const int base = blockIdx.x * S;  // this theta slot's descriptors
  double th = 0.0, tl = 0.0;
  int bad = 0;
  for (int i = tid; i < S; i += 256) {
    const int k = base + i;
    if (active[i] && status[k]) ++bad;
    double s, e;
    two_sum(th, per_subset[k], s, e);
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
    out_total[blockIdx.x] = hi[0] + lo[0];
    out_nbad[blockIdx.x] = nb[0];
  }
}

// ---------------------------------------------------------------------------
// Quadratic term of the subset likelihood (eq. (2)): y_T^T alpha with
// alpha = M^{-1} y_T, one workgroup per subset, fixed-order sums.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_quad(const SubsetDesc* __restrict__ desc,
                                              const int32_t* __restrict__ order,
                                              const double* __restrict__ yT,
                                              const double* __restrict__ alphabuf,
                                              double* __restrict__ quad) {
  __shared__ double red[256];
  const int sidx = order[blockIdx.x];
  const SubsetDesc D = desc[sidx];
  const int tid = threadIdx.x;
  double s = 0.0;
  for (int r = tid; r < D.n; r += 256) s = fma(yT[D.offT + r], alphabuf[D.offP + r], s);
  red[tid] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (tid < off) red[tid] += red[tid + off];
    __syncthreads();
  }
  if (tid == 0) quad[sidx] = red[0];
}

// ---------------------------------------------------------------------------
// GLS mean coefficients (Sec. 5, eq. (8)) of one subset from W = M^{-1} X
// and alpha = M^{-1} y: beta solves (X^T W) beta = X^T alpha.  The p x p
// system (p <= GLS_MAXP) is factored by one thread.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wsum64(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__global__ __launch_bounds__(256) void k_gls(const SubsetDesc* __restrict__ desc,
                                             const int32_t* __restrict__ order, int p, int64_t nP,
                                             const double* __restrict__ Xp,
                                             const double* __restrict__ Wp,
                                             const double* __restrict__ alphabuf,
                                             double* __restrict__ beta, int32_t* __restrict__ status) {
  constexpr int NA = GLS_MAXP * (GLS_MAXP + 1) / 2 + GLS_MAXP;
  __shared__ double part[4][NA];
  const int sidx = order[blockIdx.x];
  const SubsetDesc D = desc[sidx];
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  double acc[NA];
#pragma unroll
  for (int e = 0; e < NA; ++e) acc[e] = 0.0;
  for (int r = tid; r < D.n; r += 256) {
    double x[GLS_MAXP], wv[GLS_MAXP];
#pragma unroll
    for (int j = 0; j < GLS_MAXP; ++j) {
      x[j] = j < p ? Xp[(int64_t)j * nP + D.offP + r] : 0.0;
      wv[j] = j < p ? Wp[(int64_t)j * nP + D.offP + r] : 0.0;
    }
    const double a = alphabuf[D.offP + r];
    int e = 0;
#pragma unroll
    for (int j = 0; j < GLS_MAXP; ++j) {
#pragma unroll
      for (int k = 0; k <= j; ++k, ++e) acc[e] = fma(x[j], wv[k], acc[e]);
    }
#pragma unroll
    for (int j = 0; j < GLS_MAXP; ++j, ++e) acc[e] = fma(x[j], a, acc[e]);
  }
#pragma unroll
  for (int e = 0; e < NA; ++e) {
    const double v = wsum64(acc[e]);
    if (l == 0) part[w][e] = v;
  }
  __syncthreads();
  if (tid != 0) return;
  double A[GLS_MAXP][GLS_MAXP], b[GLS_MAXP];
  int e = 0;
  for (int j = 0; j < GLS_MAXP; ++j)
    for (int k = 0; k <= j; ++k, ++e) A[j][k] = (part[0][e] + part[1][e]) + (part[2][e] + part[3][e]);
  for (int j = 0; j < GLS_MAXP; ++j, ++e) b[j] = (part[0][e] + part[1][e]) + (part[2][e] + part[3][e]);
  // Cholesky of the p x p normal matrix, then two triangular solves
  int bad = 0;
  for (int j = 0; j < p; ++j) {
    double d = A[j][j];
    for (int k = 0; k < j; ++k) d -= A[j][k] * A[j][k];
    if (!(d > 0.0)) {
      bad = j + 1;
      break;
    }
    d = sqrt(d);
    A[j][j] = d;
    for (int i = j + 1; i < p; ++i) {
      double s = A[i][j];
      for (int k = 0; k < j; ++k) s -= A[i][k] * A[j][k];
      A[i][j] = s / d;
    }
  }
  status[sidx] = bad;
  if (bad) {
    for (int j = 0; j < p; ++j) beta[(int64_t)sidx * p + j] = __builtin_nan("");
    return;
  }
  for (int j = 0; j < p; ++j) {
    double s = b[j];
    for (int k = 0; k < j; ++k) s -= A[j][k] * b[k];
    b[j] = s / A[j][j];
  }
  for (int j = p - 1; j >= 0; --j) {
    double s = b[j];
    for (int k = j + 1; k < p; ++k) s -= A[k][j] * b[k];
    b[j] = s / A[j][j];
  }
  for (int j = 0; j < p; ++j) beta[(int64_t)sidx * p + j] = b[j];
}

// ------------------------------------------------------------- launchers --
template <typename T>
static hipError_t fwd_launch(const Launch& Lc, const int32_t* order, int n_items, int max_npad, const T* Lbuf,
                             const double* Inv, const double* rt, const double* rp, double* z,
                             double* rhs2, const int32_t* gate) {
  if (n_items <= 0) return hipSuccess;
  // slots per thread = npad / 512 at most; the 32-slot variant (subsets above
  // 8,192 padded rows) spills part of its registers
  if (max_npad <= 4096)
    hipLaunchKernelGGL((k_trsv_fwd<T, 8>), dim3(n_items), dim3(SNT), 0, Lc.stream, Lc.desc, order, Lbuf, Inv,
                       rt, rp, z, rhs2, gate);
  else if (max_npad <= 8192)
    hipLaunchKernelGGL((k_trsv_fwd<T, 16>), dim3(n_items), dim3(SNT), 0, Lc.stream, Lc.desc, order, Lbuf, Inv,
                       rt, rp, z, rhs2, gate);
  else
    hipLaunchKernelGGL((k_trsv_fwd<T, 32>), dim3(n_items), dim3(SNT), 0, Lc.stream, Lc.desc, order, Lbuf, Inv,
                       rt, rp, z, rhs2, gate);
  return hipGetLastError();
}
hipError_t launch_trsv_fwd_f32(const Launch& L, const int32_t* order, int n_items, int max_npad,
                               const float* Lbuf, const double* Inv, const double* rt, const double* rp,
                               double* z, double* rhs2, const int32_t* gate) {
  return fwd_launch<float>(L, order, n_items, max_npad, Lbuf, Inv, rt, rp, z, rhs2, gate);
}
hipError_t launch_trsv_fwd_f64(const Launch& L, const int32_t* order, int n_items, int max_npad,
                               const double* Lbuf, const double* Inv, const double* rt, const double* rp,
                               double* z, double* rhs2, const int32_t* gate) {
  return fwd_launch<double>(L, order, n_items, max_npad, Lbuf, Inv, rt, rp, z, rhs2, gate);
}

template <typename T>
static hipError_t bwd_launch(const Launch& Lc, const int32_t* order, int n_items, int max_npad, const T* Lbuf,
                             const double* Inv, const double* z, double* x, double* acc, const int32_t* gate) {
  if (n_items <= 0) return hipSuccess;
  if (max_npad <= 4096)
    hipLaunchKernelGGL((k_trsv_bwd<T, 2>), dim3(n_items), dim3(SNT), 0, Lc.stream, Lc.desc, order, Lbuf, Inv,
                       z, x, acc, gate);
  else
    hipLaunchKernelGGL((k_trsv_bwd<T, 8>), dim3(n_items), dim3(SNT), 0, Lc.stream, Lc.desc, order, Lbuf, Inv,
                       z, x, acc, gate);
  return hipGetLastError();
}
hipError_t launch_trsv_bwd_f32(const Launch& L, const int32_t* order, int n_items, int max_npad,
                               const float* Lbuf, const double* Inv, const double* z, double* x, double* acc,
                               const int32_t* gate) {
  return bwd_launch<float>(L, order, n_items, max_npad, Lbuf, Inv, z, x, acc, gate);
}
hipError_t launch_trsv_bwd_f64(const Launch& L, const int32_t* order, int n_items, int max_npad,
                               const double* Lbuf, const double* Inv, const double* z, double* x, double* acc,
                               const int32_t* gate) {
  return bwd_launch<double>(L, order, n_items, max_npad, Lbuf, Inv, z, x, acc, gate);
}

hipError_t launch_residual(const Launch& Lc, const int2* tile_items, int n_tile_items, const int2* row_items,
                           int n_row_items, const double* tx, const double* ty, const double* yT,
                           const double* alpha, double* rrow, double* pcol, double* r, const int32_t* gate) {
  if (n_tile_items <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_residual_tiles, dim3(n_tile_items), dim3(256), 0, Lc.stream, Lc.desc, tile_items,
                     Lc.theta, tx, ty, alpha, rrow, pcol, gate);
  hipLaunchKernelGGL(k_residual_reduce, dim3(n_row_items), dim3(64), 0, Lc.stream, Lc.desc, row_items,
                     Lc.theta, yT, alpha, rrow, pcol, r, gate);
  return hipGetLastError();
}

// Before sweep it >= 1 of the refinement, for the descriptors k = order[j],
// j < n: a subset takes the sweep only if it took sweep it - 1 and the
// residual that sweep measured, ||r||^2 = rhs2[k], is above tol^2 ||y_T||^2
// (gate[k] = 1, else 0); nsweep[k] counts the sweeps it takes (set at it = 1,
// so nothing needs clearing).  Descriptor k belongs to subset k % S.
__global__ __launch_bounds__(256) void k_refine_gate(int n, const int32_t* __restrict__ order, int S, int it,
                                                     const double* __restrict__ rhs2,
                                                     const double* __restrict__ ynorm2, double tol2,
                                                     int32_t* __restrict__ gate, int32_t* __restrict__ nsweep) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const int k = order[j];
  const int32_t done = it == 1 ? 1 : nsweep[k];
  const bool take = done == it && rhs2[k] > tol2 * ynorm2[k % S];
  gate[k] = take ? 1 : 0;
  nsweep[k] = take ? it + 1 : done;
}

hipError_t launch_refine_gate(hipStream_t s, int n, const int32_t* order, int S, int it, const double* rhs2,
                              const double* ynorm2, double tol, int32_t* gate, int32_t* nsweep) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_refine_gate, dim3((n + 255) / 256), dim3(256), 0, s, n, order, S, it, rhs2, ynorm2,
                     tol * tol, gate, nsweep);
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

hipError_t launch_gls(hipStream_t s, const SubsetDesc* desc, const int32_t* order, int n_items, int p,
                      int64_t nP, const double* Xp, const double* Wp, const double* alpha, double* beta,
                      int32_t* status) {
  if (n_items <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gls, dim3(n_items), dim3(256), 0, s, desc, order, p, nP, Xp, Wp, alpha, beta, status);
  return hipGetLastError();
}

hipError_t launch_quad(hipStream_t s, const SubsetDesc* desc, const int32_t* order, int n_items,
                       const double* yT, const double* alpha, double* quad) {
  if (n_items <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_quad, dim3(n_items), dim3(256), 0, s, desc, order, yT, alpha, quad);
  return hipGetLastError();
}

hipError_t launch_reduce(hipStream_t s, const SubsetDesc* desc, int S, int n_theta, const double* err,
                         int32_t* status, const int32_t* active, const double* rhs2,
                         const double* ynorm2, double tol, double* per_subset, double* out_total,
                         int32_t* out_nbad) {
  const int n_desc = S * n_theta;
  hipLaunchKernelGGL(k_subset_sspe, dim3((n_desc + 3) / 4), dim3(256), 0, s, desc, S, n_desc, err, status, active,
                     rhs2, ynorm2, tol * tol, per_subset);
  hipLaunchKernelGGL(k_reduce_total, dim3(n_theta), dim3(256), 0, s, S, status, active, per_subset, out_total,
                     out_nbad);
  return hipGetLastError();
}

// Testing hook: exp_neg and sqrt_pos on n values.
__global__ __launch_bounds__(256) void k_math_check(int64_t n, const double* __restrict__ t,
                                                    const double* __restrict__ x, double* __restrict__ e,
                                                    double* __restrict__ r) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) {
    e[i] = exp_neg(t[i]);
    r[i] = sqrt_pos(x[i]);
  }
}
hipError_t launch_math_check(hipStream_t s, int64_t n, const double* t, const double* x, double* e, double* r) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_math_check, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, t, x, e, r);
  return hipGetLastError();
}

}  // namespace pcv
