// Batched blocked Cholesky of the subset matrices M_i = Sigma_i(theta) +
// lambda I (the (Sigma + lambda I)^{-1} of eq. (3), arXiv:1912.13132), one
// workgroup per subset: 8 waves (one workgroup per compute unit) or, for
// small FP32 subsets, 4 waves with 64-column panels (two per compute unit),
// or for the smallest 2 waves with 64-row chunks (four per compute unit).
//
// Left-looking over column panels of PB columns (PB = 128 for FP32, 64 for
// FP64 and for the small shape).  For every panel J and every chunk of 32
// rows per wave at or below the diagonal, each wave keeps the TRANSPOSED
// chunk C^T (PB x 32) in MFMA accumulators:
//   1. C^T is initialised with the covariance (Sec. 3, exponential or
//      Matern-3/2) of the chunk rows and panel columns, generated from the
//      subset's centred coordinates (padded to npad with points at infinity,
//      whose entries are 0, so padding rows form an identity block); lambda
//      (and the padding's unit diagonal) is set by index when the diagonal
//      block is moved to FP64;
//   2. C^T -= L_J L_R^T over all previous columns, on MFMA from 128-byte row
//      segments staged through two LDS buffers (loads for stage k+2 in flight
//      while stage k is consumed; conflict-free 16-byte operand reads; one
//      barrier per stage, between its two operand halves, so that each
//      half's operands are read while the other half's MFMAs run);
//   3. the diagonal 64 x 64 blocks of the panel are factored in FP64 in LDS
//      (blocked in 16 x 16 tiles), inverted in FP64 into the free upper half
//      of the same array, and the inverse is kept in LDS;
//   4. the panel triangular solve X^T = L_JJ^{-1} C^T runs on MFMA with the
//      accumulators themselves as the B operand (the contraction index is
//      permuted to follow the accumulator layout), block row by block row
//      from the bottom, in place: no transpose through memory;
//   5. for FP32 panels the second 64-column half is first updated with the
//      first half's solved columns (again from the accumulators), then
//      factored and solved the same way;
//   6. the finished rows are written to the packed tile-row factor.
// The inverses of the diagonal blocks are also written (FP64) for the
// triangular solves, and 2 sum log L_jj (FP64) for log det.
// A cooperative launch (COOP) can give its largest subsets several 8-wave
// workgroups each: the row chunks of every panel are dealt out among them,
// with per-subset counters in device memory ordering the diagonal chunk
// before the others' solves and each panel before the next one's update.
#include <type_traits>

#include "pcv_device.h"

namespace pcv {
namespace potrf {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename T>
struct Cfg;
template <>
struct Cfg<float> {
  typedef f32x4 acc_t;
  static constexpr int PB = 128;  // panel width
  static constexpr int KC = 32;   // staged k per step (128 bytes of a row)
  static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // accumulator element v of lane group g sits in row crow(g, v) of a 16x16 tile
  static __device__ __forceinline__ int crow(int g, int v) { return 4 * g + v; }
};
template <>
struct Cfg<double> {
  typedef f64x4 acc_t;
  static constexpr int PB = 64;
  static constexpr int KC = 16;
  static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int crow(int g, int v) { return 4 * v + g; }
};

// Correlation of Sec. 3 (exponential) or Matern-3/2.  Padding points carry
// infinite coordinates: their distance to anything is inf or NaN, and the
// entry is then exactly 0.
// The FP32 tiles only feed the factor that preconditions the FP64
// refinement (whose residual uses the exact FP64 covariance), so the
// hardware exp2 and square root (about 1 ulp) are used here.
__device__ __forceinline__ float corr_t(int cov, float d, float ir) {
  const float t = d * ir;
  const float e = __builtin_amdgcn_exp2f(-1.44269504088896341f * t);
  const float c = cov == 1 ? (1.0f + t) * e : e;
  return d < INFINITY ? c : 0.0f;
}
__device__ __forceinline__ double corr_t(int cov, double d, double ir) {
  const double t = d * ir;
  const double e = exp(-t);
  const double c = cov == 1 ? (1.0 + t) * e : e;
  return d < INFINITY ? c : 0.0;
}

__device__ __forceinline__ float fsqrt_t(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double fsqrt_t(double x) { return sqrt(x); }

// The four accumulator-row entries crow(g, 0..3) of a 16-wide LDS row segment.
__device__ __forceinline__ void load_crow4(const float* row, int g, float (&a)[4]) {
  const float4 v = *reinterpret_cast<const float4*>(row + 4 * g);
  a[0] = v.x;
  a[1] = v.y;
  a[2] = v.z;
  a[3] = v.w;
}
__device__ __forceinline__ void load_crow4(const double* row, int g, double (&a)[4]) {
#pragma unroll
  for (int v = 0; v < 4; ++v) a[v] = row[4 * v + g];
}

// Barrier that orders LDS only: unlike __syncthreads() it does not wait for
// outstanding global loads, so prefetches stay in flight across it.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

constexpr int WR = 32;    // chunk rows per wave
// Diagonal of the y_T row: far above any |L^{-1} y_T|^2 part its block
// subtracts, so that its pivot stays positive and the padding rows below it
// keep zero entries in its column (a pivot there that fails anyway is set to
// 1 and not reported: the row is not part of the subset matrix).
constexpr double VDIAG = 1e200;
constexpr int NBJ = WR / 16;
constexpr int LDD = 65;   // FP64 diagonal array row stride (doubles)

// Workgroup shape: NTH threads (NTH / 64 waves) per subset.  512: panels of
// Cfg<T>::PB columns and 256-row chunks, one workgroup per compute unit (the
// large subsets).  256: 64-column panels and 128-row chunks in at most 80 KB
// of LDS, so that two workgroups share a compute unit and one's diagonal
// block latency overlaps the other's MFMA work.  128 (TINY): 64-column
// panels and 64-row chunks (the first chunk of a panel is its diagonal
// block) in 40 KB of LDS: each wave keeps the inverse tiles its triangular
// solves read in registers instead of LDS, and the FP64 work tiles of the
// diagonal block share the stage buffers' space, so that four workgroups
// share a compute unit and their diagonal blocks overlap each other's MFMA
// work (the smallest subsets).
template <typename T, int NTH>
struct Shape {
  static constexpr int NT = NTH;
  static constexpr int NW = NTH / 64;
  static constexpr bool TINY = NTH == 128;
  static constexpr int PB = NTH == 512 ? Cfg<T>::PB : 64;
  static constexpr int KC = Cfg<T>::KC;
  static constexpr int RCH = NW * WR;         // chunk rows
  static constexpr int VW = 16 / sizeof(T);   // elements per 16-byte vector
  static constexpr int LDK = KC + VW;         // staged row stride (144 bytes)
  static constexpr int LDI = 64 + VW;         // inverse row stride
  static constexpr int NSUB = PB / 64;
  static constexpr int NINV = TINY ? 0 : NSUB;  // inverse blocks kept in LDS
  static constexpr int STAGE = (PB + RCH) * LDK * (int)sizeof(T);
  static constexpr int L21 = 64 * LDI * (int)sizeof(T);
  static constexpr int DG = 64 * LDD * 8;
  static constexpr int TBB = 3 * 16 * 17 * 8;  // FP64 work tiles of the diagonal block
  static constexpr int DGT = TINY ? DG + TBB : DG;
  static constexpr int U0 = 2 * STAGE > DGT ? 2 * STAGE : DGT;  // two stage buffers
  static constexpr int U = NSUB == 2 && L21 > U0 ? L21 : U0;
};

// In-register triangular solve on one 64-column sub-panel (accumulator block
// rows B0..B0+3):  X^T = Inv * C^T, Inv lower triangular (LDS, row stride
// LDI).  Output block row bo needs input block rows bk <= bo, so block rows
// are produced from the bottom up and written in place.
template <typename T, int B0, int NBI, int NB>
__device__ __forceinline__ void trsm_regs(typename Cfg<T>::acc_t (&acc)[NBI][NB], const T* Inv, int lr,
                                          int g) {
  typedef typename Cfg<T>::acc_t acc_t;
  constexpr int LDI = 64 + 16 / (int)sizeof(T);
#pragma unroll
  for (int bo = 3; bo >= 0; --bo) {
    acc_t tmp[NB];
#pragma unroll
    for (int bj = 0; bj < NB; ++bj) tmp[bj] = acc_t{};
#pragma unroll
    for (int bk = 0; bk <= bo; ++bk) {
      T a[4];
      load_crow4(Inv + (16 * bo + lr) * LDI + 16 * bk, g, a);
#pragma unroll
      for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int bj = 0; bj < NB; ++bj) tmp[bj] = Cfg<T>::mma(a[v], acc[B0 + bk][bj][v], tmp[bj]);
    }
#pragma unroll
    for (int bj = 0; bj < NB; ++bj) acc[B0 + bo][bj] = tmp[bj];
  }
}

// The same solve with the inverse tiles held in registers: inv[bo (bo + 1) / 2
// + bk][v] = Inv[16 bo + lr][16 bk + crow(g, v)] (zero above the diagonal).
template <typename T, int B0, int NBI, int NB>
__device__ __forceinline__ void trsm_regs_r(typename Cfg<T>::acc_t (&acc)[NBI][NB], const T (&inv)[10][4]) {
  typedef typename Cfg<T>::acc_t acc_t;
#pragma unroll
  for (int bo = 3; bo >= 0; --bo) {
    acc_t tmp[NB];
#pragma unroll
    for (int bj = 0; bj < NB; ++bj) tmp[bj] = acc_t{};
#pragma unroll
    for (int bk = 0; bk <= bo; ++bk)
#pragma unroll
      for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int bj = 0; bj < NB; ++bj)
          tmp[bj] = Cfg<T>::mma(inv[bo * (bo + 1) / 2 + bk][v], acc[B0 + bk][bj][v], tmp[bj]);
#pragma unroll
    for (int bj = 0; bj < NB; ++bj) acc[B0 + bo][bj] = tmp[bj];
  }
}

// FP64 factorisation of the 64 x 64 block in Dg (lower part), in place,
// followed by the inverse of the factor, stored transposed in the free upper
// part: Inv[i][c] (i >= c) lives at Dg[c][i + 1].  Adds 2 sum log L_jj over
// rows < nreal to ld and records the first failing pivot (1-based global
// row) in bad (thread 0's copies).  All NW waves of the workgroup take part
// (NW >= 2).
//
// Blocked in 16 x 16 tiles.  For each tile column kb:
//   1. wave 0 factors and inverts the diagonal tile together in registers,
//      four entries per lane: at pivot j the pivot comes by readlane, the
//      lane's own row entry by a quad broadcast (DPP), the column-j entries
//      and the inverse's row j by lane shuffles; the inverse is built as the
//      product of the elementary inverses of the columns (row j scaled by
//      1/L_jj, the rows below eliminated with it);
//   2. the tiles below: X_I = A_Ik L_kk^{-T}, one FP64 MFMA tile per wave,
//      and beside them row kb of the inverse off the diagonal, one tile per
//      wave: Inv_kb,J = -Inv_kb,kb * sum_{J<=K<kb} L_kb,K Inv_K,J (two MFMA
//      products), from the leaf of this step and the rows of earlier steps;
//   3. the trailing lower block triangle: A_IK -= X_I X_K^T, one MFMA tile
//      per wave.
__device__ __forceinline__ double rlane(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// quad_perm DPP control that broadcasts lane q of every group of four
constexpr int QP(int q) { return q | q << 2 | q << 4 | q << 6; }
template <int CTRL>
__device__ __forceinline__ double qbcast(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)b, CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
// value of lane (l & ~3) | q in every lane l (q known after unrolling)
__device__ __forceinline__ double qbcast(double v, int q) {
  switch (q) {
    case 0: return qbcast<QP(0)>(v);
    case 1: return qbcast<QP(1)>(v);
    case 2: return qbcast<QP(2)>(v);
    default: return qbcast<QP(3)>(v);
  }
}

template <int NW>
__device__ void diag_factor_invert(double (*Dg)[LDD], double (*Tb)[16][17], int nreal, int grow0,
                                   double& ld, int& bad) {
  typedef double f64x4_t __attribute__((ext_vector_type(4)));
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  const int li = l & 15, kq = l >> 4;  // MFMA operand lane roles: index li, k slice kq
  for (int kb = 0; kb < 4; ++kb) {
    const int k0 = 16 * kb;
    // ---- leaf: factor and invert the diagonal tile in wave 0
    // 1. diagonal tile, wave 0: lane l holds entries (r, c) = (l / 4, l % 4 + 4 u)
    //    of the tile in registers through the 16 pivot steps: the pivot by
    //    readlane, A[r][j] from the lane's quad and A[c][j] from lane 4 c + j % 4
    //    by lane shuffles; then the factored tile goes back to LDS.
    if (w == 0) {
      const int r = l >> 2, cq = l & 3;
      double a[4], x[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        a[u] = Dg[k0 + r][k0 + cq + 4 * u];
        x[u] = r == cq + 4 * u ? 1.0 : 0.0;
      }
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int uj = j >> 2, qj = j & 3;
        // operands of this pivot that need no pivot value: issued first
        double xj[4], acj[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          xj[u] = __shfl(x[u], 4 * j + cq, 64);
          acj[u] = __shfl(a[uj], 4 * (cq + 4 * u) + qj, 64);
        }
        const double arj = qbcast(a[uj], qj);
        double p = rlane(a[uj], 4 * j + qj);
        const bool ok = p > 0.0 && p < 1e300;
        if (!ok) p = 1.0;
        if (l == 0 && !ok && !bad && k0 + j < nreal) bad = grow0 + k0 + j + 1;
        double isp = __builtin_amdgcn_rsq(p);
        isp = isp * (1.5 - 0.5 * p * isp * isp);
        isp = isp * (1.5 - 0.5 * p * isp * isp);
        const double sp = p * isp, ip = isp * isp;
        const double arjp = arj * ip;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int c = cq + 4 * u;
          const double upd = fma(-arjp, acj[u], a[u]);
          if (c == j && r >= j) a[u] = r == j ? sp : arj * isp;
          if (c > j && r >= c) a[u] = upd;
          // inverse: row j scaled, the rows below eliminated with it
          x[u] = r == j ? x[u] * isp : (r > j ? fma(-arjp, xj[u], x[u]) : x[u]);
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int c = cq + 4 * u;
        if (r >= c) {
          Dg[k0 + r][k0 + c] = a[u];
          Dg[k0 + c][k0 + r + 1] = x[u];
        }
      }
      __builtin_amdgcn_wave_barrier();
      // log det of the tile's real rows
      double t = (l < 16 && k0 + l < nreal) ? 2.0 * log(Dg[k0 + l][k0 + l]) : 0.0;
#pragma unroll
      for (int off = 8; off > 0; off >>= 1) t += __shfl_xor(t, off, 64);
      if (tid == 0) ld += t;
    }
    __syncthreads();
    // ---- tiles below, X_I = A_I,k L_kk^{-T}, wave w -> block row kb + 1 + w; and
    //      row kb of the inverse, Inv_kb,J = -Inv_kb,kb sum_{K=J}^{kb-1} L_kb,K Inv_K,J
    //      for J < kb, wave 3 - kb + J: both need only this step's leaf and the
    //      earlier steps
    for (int t = w; t < 3; t += NW) {
      if (t < 3 - kb) {
        const int I = kb + 1 + t;
        f64x4_t acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
          const int m = 4 * ks + kq;
          const double av = Dg[16 * I + li][k0 + m];
          const double bv = m <= li ? Dg[k0 + m][k0 + li + 1] : 0.0;
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) Dg[16 * I + 4 * v + kq][k0 + li] = acc[v];
      } else {
        const int I = kb, J = t - (3 - kb);
        f64x4_t acc = {0.0, 0.0, 0.0, 0.0};
        for (int K = J; K < I; ++K) {
#pragma unroll
          for (int ks = 0; ks < 4; ++ks) {
            const int m = 4 * ks + kq;
            const double av = Dg[16 * I + li][16 * K + m];
            const double bv = (K > J || m >= li) ? Dg[16 * J + li][16 * K + m + 1] : 0.0;
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
          }
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) Tb[J][4 * v + kq][li] = acc[v];
        __builtin_amdgcn_wave_barrier();
        f64x4_t acc2 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
          const int m = 4 * ks + kq;
          const double av = m <= li ? -Dg[16 * I + m][16 * I + li + 1] : 0.0;
          const double bv = Tb[J][m][li];
          acc2 = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc2, 0, 0, 0);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) Dg[16 * J + li][16 * I + 4 * v + kq + 1] = acc2[v];
      }
    }
    __syncthreads();
    if (kb == 3) break;
    // ---- trailing update of the lower block triangle: A_IK -= X_I X_K^T
    {
      const int t = 3 - kb;
      const int npairs = t * (t + 1) / 2;
      for (int pw = w; pw < npairs; pw += NW) {
        // pair index -> (I, K), K <= I, both in kb+1..3
        int I = kb + 1, K = kb + 1, q = pw;
        while (q > I - (kb + 1)) {
          q -= I - kb;
          ++I;
        }
        K = kb + 1 + q;
        f64x4_t acc;
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[v] = Dg[16 * I + 4 * v + kq][16 * K + li];
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
          const int m = 4 * ks + kq;
          const double av = -Dg[16 * I + li][k0 + m];
          const double bv = Dg[16 * K + li][k0 + m];
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v)
          if (I != K || li <= 4 * v + kq) Dg[16 * I + 4 * v + kq][16 * K + li] = acc[v];
      }
    }
    __syncthreads();
  }
}

// ---- several workgroups on one subset
// A cooperative launch gives a large subset several workgroups ("ranks"):
// in every panel rank r takes the row chunks whose index within the panel is
// r modulo the rank count, so rank 0 always holds the diagonal chunk.  Each
// chunk's arithmetic is the same as with one workgroup, so the factor is the
// same bit for bit.  Per subset, three counters in device memory (zeroed
// before the launch): the panels whose diagonal chunk is stored (written by
// rank 0), the rank-panels finished (every rank adds one per panel) and an
// error word.  Waits are polled by thread 0 with a bounded count: a wait that
// runs out marks the subset (status PCV_STATUS_SYNC_TIMEOUT) and the rank
// carries on without waiting again, so every wave reaches the end.
constexpr int COOP_SPIN = 1 << 21;  // polls, each about a microsecond or more

// Thread 0 waits until *ctr >= target (agent-scope acquire); then the whole
// workgroup continues with an acquire fence of its own.
__device__ __forceinline__ void wg_wait(int32_t* ctr, int32_t target, int& tmo, int32_t* err) {
  if (threadIdx.x == 0 && !tmo) {
    int it = 0;
    while (__hip_atomic_load(ctr, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (++it > COOP_SPIN) {
        tmo = 1;
        __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
      __builtin_amdgcn_s_sleep(8);
    }
  }
  __syncthreads();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}
// Every thread's earlier global stores are made visible at agent scope, then
// thread 0 sets *ctr = value (set) or adds one (!set) with release order.
__device__ __forceinline__ void wg_signal(int32_t* ctr, int32_t value, bool set) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __syncthreads();
  if (threadIdx.x == 0) {
    if (set)
      __hip_atomic_store(ctr, value, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    else
      __hip_atomic_fetch_add(ctr, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
}

__global__ void k_fill_i32(int32_t* __restrict__ p, int n, int32_t v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// After a factorisation with the y_T row: z = L^{-1} y_T (FP64, padded with
// zeros to npad) from row n, then row n and its row of the diagonal-block
// inverse are reset to those of a padding row (unit diagonal, zeros).
template <typename T>
__global__ __launch_bounds__(256) void k_take_z(const SubsetDesc* __restrict__ desc,
                                                const int32_t* __restrict__ order, T* __restrict__ Lbuf,
                                                double* __restrict__ Invbuf, double* __restrict__ zbuf) {
  const SubsetDesc D = desc[order[blockIdx.x]];
  const int n = D.n, npad = D.npad;
  if (n <= 0 || n >= npad) return;
  T* __restrict__ row = Lbuf + D.offL + packed_rowoff32(n);
  double* __restrict__ z = zbuf + D.offP;
  for (int i = threadIdx.x; i < npad; i += 256) {
    if (i < n) {
      z[i] = (double)row[i];
      row[i] = (T)0;
    } else {
      z[i] = 0.0;
      if (i == n) row[i] = (T)1;
    }
  }
  double* __restrict__ inv = Invbuf + D.offInv + (int64_t)(n / 64) * 4096 + (n % 64) * 64;
  for (int j = threadIdx.x; j < 64; j += 256) inv[j] = j == n % 64 ? 1.0 : 0.0;
}

template <typename T, int NTH, bool COOP>
__global__ __launch_bounds__(NTH, 2) void k_potrf(const SubsetDesc* __restrict__ desc,
                                                 const int32_t* __restrict__ order,
                                                 const ThetaDev* __restrict__ theta,
                                                 const T* __restrict__ cx, const T* __restrict__ cy,
                                                 const T* __restrict__ cyv,
                                                 T* __restrict__ Lbuf, double* __restrict__ Invbuf,
                                                 double* __restrict__ logdet,
                                                 int32_t* __restrict__ status,
                                                 const int32_t* __restrict__ coop_info, int n_coop,
                                                 int32_t* __restrict__ coop_sync) {
  typedef typename Cfg<T>::acc_t acc_t;
  typedef Shape<T, NTH> SM;
  constexpr int NT = SM::NT, RCH = SM::RCH;
  constexpr int PB = SM::PB, KC = SM::KC, VW = SM::VW, LDK = SM::LDK, LDI = SM::LDI;
  constexpr int NBI = PB / 16;                    // accumulator block rows (panel columns)
  constexpr int NVEC = (PB + RCH) * (KC / VW);    // 16-byte vectors per stage
  constexpr int VPR = KC / VW;                    // vectors per row (4)
  typedef typename std::conditional<sizeof(T) == 4, float4, double2>::type vec_t;

  __shared__ __attribute__((aligned(16))) char smem_u[SM::U];
  __shared__ __attribute__((aligned(16))) T InvS[SM::NINV > 0 ? SM::NINV : 1][SM::NINV > 0 ? 64 * LDI : 1];
  __shared__ double TbS[SM::TINY ? 1 : 3][16][17];
  __shared__ T colx[PB], coly[PB];  // the current panel's column coordinates
  __shared__ T colv[PB];            // ... and their y_T values (row n, when cyv is given)

  T* Ps = reinterpret_cast<T*>(smem_u);    // [PB][LDK]  panel rows (negated)
  T* L21s = reinterpret_cast<T*>(smem_u);  // [64][LDI]  -L21 (second half update)
  double(*Dg)[LDD] = reinterpret_cast<double(*)[LDD]>(smem_u);
  // FP64 work tiles of the diagonal block: behind Dg in the TINY shape
  double(*Tb)[16][17] = SM::TINY ? reinterpret_cast<double(*)[16][17]>(smem_u + SM::DG) : TbS;
  // TINY: the inverse tiles of the current panel that this wave's solves read
  T invr[SM::TINY ? 10 : 1][4];

  // rank of this workgroup among the nwg that share the subset; blocks past
  // the cooperative ones (and every block without COOP) work alone
  int rank = 0, nwg = 1;
  int32_t* sy = nullptr;
  if constexpr (COOP) {
    if ((int)blockIdx.x < n_coop) {
      const int32_t info = coop_info[blockIdx.x];
      rank = info & 255;
      nwg = (info >> 8) & 255;
      sy = coop_sync + 4 * (info >> 16);
      if (nwg == 0) return;
    }
  }
  int tmo = 0;  // thread 0: a wait ran out

  const int sidx = order[blockIdx.x];
  const SubsetDesc D = desc[sidx];
  const int n = D.n, npad = D.npad;
  T* __restrict__ L = Lbuf + D.offL;
  double* __restrict__ Inv = Invbuf + D.offInv;
  const T* __restrict__ X = cx + D.offX;  // padded coordinates (npad entries)
  const T* __restrict__ Y = cy + D.offX;
  // With cyv, the training values y_T ride along as row n (the first padding
  // row): entries y_j in columns j < n, a large diagonal.  The left-looking
  // updates and panel solves then leave (L^{-1} y_T)_j in that row, the
  // forward substitution of the solve of eq. (3); rows < n never read it,
  // so their factor is unchanged.  The row is moved out afterwards.
  const int cov = theta[D.th].cov;
  const T ir = (T)theta[D.th].inv_range;
  const double lam64 = theta[D.th].lambda;

  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  const int lr = l & 15, g = l >> 4;

  double ld = 0.0;
  int bad = 0;
  // rows at or past nlive are padding rows: their covariance entries are 0
  // and so are their factor entries left of the diagonal (no row of the
  // subset matrix reaches them), so a wave whose rows all lie there writes
  // zeros without computing them (the y_T row, n, is live)
  const int nlive = cyv ? n + 1 : n;

  for (int c0 = 0, panel = 0; c0 < npad; c0 += PB, ++panel) {
    const bool two = (SM::NSUB == 2) && (c0 + 128 <= npad);
    // cooperative ranks: the previous panel's rows are all stored (checked
    // before the first update of this panel), this panel's diagonal inverse
    // is in LDS (rank 0 makes it; the others read it once per panel)
    bool synced = !COOP || nwg == 1 || c0 == 0;
    bool inv_ready = !COOP || rank == 0;
    __syncthreads();  // previous panel done with colx / coly
    if (tid < PB) {
      const int col = min(c0 + tid, npad - 1);
      colx[tid] = X[col];
      coly[tid] = Y[col];
      colv[tid] = cyv ? cyv[(X - cx) + col] : (T)0;
    }
    for (int r0 = c0 + RCH * rank; r0 < npad; r0 += RCH * nwg) {
      const bool first = (r0 == c0);
      const int wr0 = r0 + WR * w;          // this wave's first row
      const bool wact = wr0 < npad;
      const bool wlive = wr0 < nlive;
      // In the first chunk, waves 0,1 hold the diagonal block of the first
      // 64 columns, waves 2,3 the second 64 rows of the panel.
      const int wpos = first ? w : 8;     // 8 = an ordinary row block
      acc_t acc[NBI][NBJ];
      __syncthreads();  // previous chunk finished with LDS and global writes

      // ---- 1. covariance: acc[bi][bj][v] = c(|s_row - s_col|) for row = wr0 + 16 bj + lr,
      //      col = c0 + 16 bi + crow(g, v).  Padding points are at infinity, so
      //      their entries are exactly 0; the nugget and the padding's unit
      //      diagonal are set on the diagonal blocks in FP64 (step 3).
      if (wlive) {
        T xr[NBJ], yr[NBJ];
#pragma unroll
        for (int bj = 0; bj < NBJ; ++bj) {
          const int row = wr0 + 16 * bj + lr;
          xr[bj] = X[row];
          yr[bj] = Y[row];
        }
#pragma unroll
        for (int bi = 0; bi < NBI; ++bi) {
          T tv[NBJ][4];
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int cl = 16 * bi + Cfg<T>::crow(g, v);
            const T xc = colx[cl], yc = coly[cl];
#pragma unroll
            for (int bj = 0; bj < NBJ; ++bj) {
              const T dx = xr[bj] - xc, dy = yr[bj] - yc;
              tv[bj][v] = corr_t(cov, fsqrt_t(dx * dx + dy * dy), ir);
            }
          }
#pragma unroll
          for (int bj = 0; bj < NBJ; ++bj) acc[bi][bj] = acc_t{tv[bj][0], tv[bj][1], tv[bj][2], tv[bj][3]};
        }
      } else if (wact) {
#pragma unroll
        for (int bi = 0; bi < NBI; ++bi)
#pragma unroll
          for (int bj = 0; bj < NBJ; ++bj) acc[bi][bj] = acc_t{};
      }

      if constexpr (COOP) {
        if (!synced) {
          wg_wait(sy + 1, nwg * panel, tmo, sy + 2);
          synced = true;
        }
      }

      // ---- 2. update: C^T -= L[c0:c0+PB, 0:c0] L[rows, 0:c0]^T
      //      Two LDS stage buffers and one barrier per stage, placed between
      //      the stage's two halves (q = 0, 1) of operand columns.  First half
      //      of stage k: the MFMAs on the q = 0 operands (read before) while
      //      the q = 1 operands are read, stage k + 1 is stored into the other
      //      buffer and stage k + 2 is requested from memory.  Barrier: stage
      //      k + 1 complete.  Second half: the MFMAs on the q = 1 operands
      //      while the q = 0 operands of stage k + 1 are read.  No wave waits
      //      on LDS before its MFMAs, and the stores drain behind them.
      if (c0 > 0) {
        // staging map: vector vi = tid + NT s -> (row vi / VPR, 16-byte column
        // slot vi % VPR); rows [0, PB) are panel rows (stored negated), the
        // rest chunk rows.  Rows past npad read row npad - 1 instead: they
        // only feed accumulators that are never used (chunk rows of waves
        // past the matrix, the second half of a half-width last panel).
        static_assert(NVEC % NT == 0 && (PB * VPR) % NT == 0, "stage rows split evenly");
        constexpr int VPT = NVEC / NT;
        int goff[VPT];
#pragma unroll
        for (int s = 0; s < VPT; ++s) {
          const int vi = tid + NT * s;
          const int row = vi / VPR, cv = vi % VPR;
          const int grow = row < PB ? c0 + row : r0 + (row - PB);
          goff[s] = packed_rowoff32(min(grow, npad - 1)) + cv * VW;
        }
        vec_t st[VPT];
        auto gload = [&](int k0) {
#pragma unroll
          for (int s = 0; s < VPT; ++s) st[s] = *reinterpret_cast<const vec_t*>(L + goff[s] + k0);
        };
        auto lstore = [&](T* buf) {
#pragma unroll
          for (int s = 0; s < VPT; ++s) {
            const int vi = tid + NT * s;
            const int row = vi / VPR, cv = vi % VPR;
            vec_t v = st[s];
            if (NT * s < PB * VPR) {  // a panel row
              T* p = reinterpret_cast<T*>(&v);
#pragma unroll
              for (int e = 0; e < VW; ++e) p[e] = -p[e];
            }
            *reinterpret_cast<vec_t*>(buf + row * LDK + cv * VW) = v;
          }
        };
        // lane group g takes k = g (KC/4) + q VW + s: one 16-byte read per
        // operand block and half, VW MFMA steps per read
        static_assert(KC == 8 * VW, "two operand halves per stage");
        constexpr int SBUF = (PB + RCH) * LDK;  // elements per stage buffer
        vec_t pa0[NBI], rb0[NBJ], pa1[NBI], rb1[NBJ];
        // (the loop is free of branches around memory operations, so that
        // the waits the compiler places before each half's MFMAs cover only
        // the operands that half uses: the last stage stores and loads a
        // spare stage)
        auto rd = [&](const T* buf, int q, vec_t (&pa)[NBI], vec_t (&rb)[NBJ]) {
          const T* Rk = buf + PB * LDK;
#pragma unroll
          for (int bj = 0; bj < NBJ; ++bj)
            rb[bj] = *reinterpret_cast<const vec_t*>(Rk + (WR * w + 16 * bj + lr) * LDK + g * (KC / 4) + q * VW);
#pragma unroll
          for (int bi = 0; bi < NBI; ++bi)
            pa[bi] = *reinterpret_cast<const vec_t*>(buf + (16 * bi + lr) * LDK + g * (KC / 4) + q * VW);
        };
        auto mm = [&](const vec_t (&pa)[NBI], const vec_t (&rb)[NBJ]) {
#pragma unroll
          for (int h = 0; h < NBI; h += 4)
#pragma unroll
            for (int s = 0; s < VW; ++s)
#pragma unroll
              for (int b = 0; b < 4; ++b)
#pragma unroll
                for (int bj = 0; bj < NBJ; ++bj)
                  acc[h + b][bj] = Cfg<T>::mma(reinterpret_cast<const T*>(&pa[h + b])[s],
                                               reinterpret_cast<const T*>(&rb[bj])[s], acc[h + b][bj]);
        };
        // Instruction order inside each half (the two waves of a SIMD run in
        // step, so memory instructions issued between MFMAs are hidden behind
        // the other wave's MFMAs): first half, one LDS read after every two
        // MFMAs, then the LDS stores and the memory loads between pairs of
        // MFMAs; second half, one LDS read after every three MFMAs.  The
        // scheduling fences keep the halves apart.  (Measured against one
        // MFMA per memory instruction: 93.0 -> 89.2 ms on 2,304 subsets of
        // 2,250 points.)
        constexpr int NRD = NBI + NBJ;  // LDS reads per half
        auto order_first_half = [] {
#pragma unroll
          for (int i = 0; i < NRD; ++i) {
            __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);  // MFMA
            __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);  // LDS read
          }
#pragma unroll
          for (int i = 0; i < VPT; ++i) {
            __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);
            __builtin_amdgcn_sched_group_barrier(0x200, 1, 0);  // LDS write
            __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);
            __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);  // memory read
          }
        };
        auto order_second_half = [] {
#pragma unroll
          for (int i = 0; i < NRD; ++i) {
            __builtin_amdgcn_sched_group_barrier(0x008, 3, 0);
            __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
          }
        };
        const int nst = c0 / KC;
        gload(0);
        lds_barrier();  // LDS free (previous phase done with smem_u)
        lstore(Ps);
        if (nst > 1) gload(KC);
        lds_barrier();
        if (wlive) {
          rd(Ps, 0, pa0, rb0);
          for (int k = 0; k < nst; ++k) {
            const T* Bk = Ps + (k & 1) * SBUF;
            T* Bn = Ps + ((k + 1) & 1) * SBUF;
            rd(Bk, 1, pa1, rb1);
            lstore(Bn);
            gload(min(k + 2, nst - 1) * KC);
            mm(pa0, rb0);
            order_first_half();
            __builtin_amdgcn_sched_barrier(0);
            lds_barrier();
            __builtin_amdgcn_sched_barrier(0);
            rd(Bn, 0, pa0, rb0);
            mm(pa1, rb1);
            order_second_half();
            __builtin_amdgcn_sched_barrier(0);
          }
        } else {
          // waves without live rows: their share of the staging only
          for (int k = 0; k < nst; ++k) {
            lstore(Ps + ((k + 1) & 1) * SBUF);
            gload(min(k + 2, nst - 1) * KC);
            lds_barrier();
          }
        }
      }

      // the y_T row (a padding row, so its covariance entries are 0): add
      // y_j after the update, in the one lane row of the one wave that holds it
      if (cyv && wact && n >= wr0 && n < wr0 + WR) {
        const int rn = n - wr0;
#pragma unroll
        for (int bj = 0; bj < NBJ; ++bj)
          if ((rn >> 4) == bj && lr == (rn & 15)) {
#pragma unroll
            for (int bi = 0; bi < NBI; ++bi)
#pragma unroll
              for (int v = 0; v < 4; ++v) acc[bi][bj][v] += colv[16 * bi + Cfg<T>::crow(g, v)];
          }
      }

      if constexpr (COOP) {
        if (!inv_ready) {
          // rank 0 has stored this panel's diagonal chunk (factor rows and
          // the FP64 inverses): take the inverses as rank 0 holds them
          wg_wait(sy, panel + 1, tmo, sy + 2);
          for (int e = tid; e < 64 * 64; e += NT) {
            const int i = e >> 6, j = e & 63;
            InvS[0][i * LDI + j] = (T)Inv[(int64_t)(c0 / 64) * 4096 + e];
            if constexpr (SM::NSUB == 2) {
              if (two) InvS[1][i * LDI + j] = (T)Inv[(int64_t)(c0 / 64 + 1) * 4096 + e];
            }
          }
          __syncthreads();
          inv_ready = true;
        }
      }

      // ---- 3/4. first sub-panel: diagonal block (first chunk), then solve
      if (first) {
        __syncthreads();
        if (wpos < 2) {
#pragma unroll
          for (int bi = 0; bi < 4; ++bi)
#pragma unroll
            for (int bj = 0; bj < NBJ; ++bj)
#pragma unroll
              for (int v = 0; v < 4; ++v)
                Dg[WR * wpos + 16 * bj + lr][16 * bi + Cfg<T>::crow(g, v)] = (double)acc[bi][bj][v];
        }
        __syncthreads();
        if (tid < 64) Dg[tid][tid] = c0 + tid < n ? Dg[tid][tid] + lam64 : (cyv && c0 + tid == n ? VDIAG : 1.0);
        __syncthreads();
        diag_factor_invert<SM::NW>(Dg, Tb, n - c0, c0, ld, bad);
        for (int e = tid; e < 64 * 64; e += NT) {
          const int i = e >> 6, j = e & 63;
          L[packed_rowoff32(c0 + i) + c0 + j] = j <= i ? (T)Dg[i][j] : (T)0;
          const double iv = j <= i ? Dg[j][i + 1] : 0.0;
          Inv[(int64_t)(c0 / 64) * 4096 + e] = iv;
          if constexpr (SM::NINV > 0) InvS[0][i * LDI + j] = (T)iv;
        }
        if constexpr (SM::TINY) {
#pragma unroll
          for (int bo = 0; bo < 4; ++bo)
#pragma unroll
            for (int bk = 0; bk <= bo; ++bk)
#pragma unroll
              for (int v = 0; v < 4; ++v) {
                const int row = 16 * bo + lr, col = 16 * bk + Cfg<T>::crow(g, v);
                invr[bo * (bo + 1) / 2 + bk][v] = col <= row ? (T)Dg[col][row + 1] : (T)0;
              }
        }
        __syncthreads();
      }
      if constexpr (SM::TINY) {
        if (wlive && wpos >= 2) trsm_regs_r<T, 0, NBI, NBJ>(acc, invr);
      } else {
        if (wlive && wpos >= 2) trsm_regs<T, 0, NBI, NBJ>(acc, InvS[0], lr, g);
      }

      if constexpr (SM::NSUB == 2) {
        if (two) {
          // ---- 5. second half: C2^T -= L21 X0^T, then factor / solve
          __syncthreads();
          if (first) {
            if (wpos == 2 || wpos == 3) {
#pragma unroll
              for (int bi = 0; bi < 4; ++bi)
#pragma unroll
                for (int bj = 0; bj < NBJ; ++bj)
#pragma unroll
                  for (int v = 0; v < 4; ++v) {
                    const int i = WR * (wpos - 2) + 16 * bj + lr, k = 16 * bi + Cfg<T>::crow(g, v);
                    L21s[i * LDI + k] = -acc[bi][bj][v];
                  }
            }
          } else {
            for (int e = tid; e < 64 * 16; e += NT) {
              const int i = e >> 4, k4 = (e & 15) * 4;
              const float4 v = *reinterpret_cast<const float4*>(
                  reinterpret_cast<const float*>(L) + packed_rowoff32(c0 + 64 + i) + c0 + k4);
              float* q = reinterpret_cast<float*>(L21s) + i * LDI + k4;
              q[0] = -v.x;
              q[1] = -v.y;
              q[2] = -v.z;
              q[3] = -v.w;
            }
          }
          __syncthreads();
          if (wlive && wpos >= 2) {
#pragma unroll
            for (int bi = 0; bi < 4; ++bi) {
#pragma unroll
              for (int bk = 0; bk < 4; ++bk) {
                T a[4];
                load_crow4(L21s + (16 * bi + lr) * LDI + 16 * bk, g, a);
#pragma unroll
                for (int v = 0; v < 4; ++v)
#pragma unroll
                  for (int bj = 0; bj < NBJ; ++bj)
                    acc[4 + bi][bj] = Cfg<T>::mma(a[v], acc[bk][bj][v], acc[4 + bi][bj]);
              }
            }
          }
          if (first) {
            __syncthreads();
            if (wpos == 2 || wpos == 3) {
#pragma unroll
              for (int bi = 0; bi < 4; ++bi)
#pragma unroll
                for (int bj = 0; bj < NBJ; ++bj)
#pragma unroll
                  for (int v = 0; v < 4; ++v)
                    Dg[WR * (wpos - 2) + 16 * bj + lr][16 * bi + Cfg<T>::crow(g, v)] = (double)acc[4 + bi][bj][v];
            }
            __syncthreads();
            if (tid < 64)
              Dg[tid][tid] = c0 + 64 + tid < n ? Dg[tid][tid] + lam64 : (cyv && c0 + 64 + tid == n ? VDIAG : 1.0);
            __syncthreads();
            diag_factor_invert<SM::NW>(Dg, Tb, n - c0 - 64, c0 + 64, ld, bad);
            for (int e = tid; e < 64 * 64; e += NT) {
              const int i = e >> 6, j = e & 63;
              L[packed_rowoff32(c0 + 64 + i) + c0 + 64 + j] = j <= i ? (T)Dg[i][j] : (T)0;
              const double iv = j <= i ? Dg[j][i + 1] : 0.0;
              Inv[(int64_t)(c0 / 64 + 1) * 4096 + e] = iv;
              InvS[1][i * LDI + j] = (T)iv;
            }
            __syncthreads();
          }
          if (wlive && wpos >= 4) trsm_regs<T, 4, NBI, NBJ>(acc, InvS[1], lr, g);
        }
      }

      // ---- 6. store the finished rows
      if (wact && wpos >= 2) {
        const int nbs = (wpos < 4) ? 4 : (two ? NBI : 4);
#pragma unroll
        for (int bi = 0; bi < NBI; ++bi) {
          if (bi < nbs) {
#pragma unroll
            for (int bj = 0; bj < NBJ; ++bj) {
              const int row = wr0 + 16 * bj + lr;
              T* dst = L + packed_rowoff32(row) + c0 + 16 * bi;
              if constexpr (sizeof(T) == 4) {
                *reinterpret_cast<acc_t*>(dst + 4 * g) = acc[bi][bj];
              } else {
#pragma unroll
                for (int v = 0; v < 4; ++v) dst[Cfg<T>::crow(g, v)] = acc[bi][bj][v];
              }
            }
          }
        }
      }
      if constexpr (COOP) {
        if (first && nwg > 1) wg_signal(sy, panel + 1, true);  // diagonal chunk stored
      }
    }
    if constexpr (COOP) {
      // arrive once per panel, and only after the previous panel's arrivals
      // are all in, so that a count of nwg * p means panels < p are done
      if (nwg > 1) {
        if (!synced) wg_wait(sy + 1, nwg * panel, tmo, sy + 2);
        wg_signal(sy + 1, 0, false);
      }
    }
  }
  if constexpr (COOP) {
    if (nwg > 1 && rank != 0) return;
    if (nwg > 1) {
      // every rank done: a wait that ran out anywhere is in the error word
      wg_wait(sy + 1, nwg * ((npad + PB - 1) / PB), tmo, sy + 2);
      if (tid == 0 && (tmo || __hip_atomic_load(sy + 2, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT)))
        bad = PCV_STATUS_SYNC_TIMEOUT;
    }
  }
  if (tid == 0) {
    logdet[sidx] = ld;
    status[sidx] = bad;
  }
}

}  // namespace potrf

template <typename T>
static hipError_t take_z(const Launch& Lc, const int32_t* order, int n_items, const T* cv, T* Lbuf, double* Inv,
                         double* zout) {
  if (!cv || n_items <= 0) return hipGetLastError();
  hipLaunchKernelGGL(potrf::k_take_z<T>, dim3(n_items), dim3(256), 0, Lc.stream, Lc.desc, order, Lbuf, Inv, zout);
  return hipGetLastError();
}

template <typename T>
static hipError_t potrf2_launch(const Launch& Lc, const int32_t* order, int n_items, const T* cx,
                                const T* cy, const T* cv, double* zout, T* Lbuf, double* Inv, double* logdet,
                                int32_t* status, const CoopPlan* cp) {
  if (n_items <= 0) return hipSuccess;
  if (cp && cp->n_blocks > 0) {
    if (cp->n_blocks > n_items || cp->n_slots <= 0 || !cp->info || !cp->sync) return hipErrorInvalidValue;
    const int nz = 4 * cp->n_slots;
    hipLaunchKernelGGL(potrf::k_fill_i32, dim3((nz + 255) / 256), dim3(256), 0, Lc.stream, cp->sync, nz, 0);
    if (cv && (!cp->subsets || cp->n_subsets <= 0)) return hipErrorInvalidValue;
    hipLaunchKernelGGL((potrf::k_potrf<T, 512, true>), dim3(n_items), dim3(512), 0, Lc.stream, Lc.desc, order,
                       Lc.theta, cx, cy, cv, Lbuf, Inv, logdet, status, cp->info, cp->n_blocks, cp->sync);
    return take_z<T>(Lc, cp->subsets, cp->n_subsets, cv, Lbuf, Inv, zout);
  } else {
    hipLaunchKernelGGL((potrf::k_potrf<T, 512, false>), dim3(n_items), dim3(512), 0, Lc.stream, Lc.desc, order,
                       Lc.theta, cx, cy, cv, Lbuf, Inv, logdet, status, nullptr, 0, nullptr);
  }
  return take_z<T>(Lc, order, n_items, cv, Lbuf, Inv, zout);
}
hipError_t launch_potrf_f32(const Launch& L, const int32_t* order, int n_items, int max_npad, const float* cx,
                            const float* cy, const float* cv, double* zout, float* Lbuf, double* Inv,
                            double* logdet, int32_t* status, const CoopPlan* cp, int small_npad, int tiny_npad) {
  if (cv && !zout) return hipErrorInvalidValue;
  if (n_items > 0 && max_npad <= tiny_npad) {
    if (cp && cp->n_blocks > 0) return hipErrorInvalidValue;  // cooperative ranks use 8-wave workgroups
    hipLaunchKernelGGL((potrf::k_potrf<float, 128, false>), dim3(n_items), dim3(128), 0, L.stream, L.desc, order,
                       L.theta, cx, cy, cv, Lbuf, Inv, logdet, status, nullptr, 0, nullptr);
    return take_z<float>(L, order, n_items, cv, Lbuf, Inv, zout);
  }
  if (n_items > 0 && max_npad <= small_npad) {
    if (cp && cp->n_blocks > 0) return hipErrorInvalidValue;  // cooperative ranks use 8-wave workgroups
    hipLaunchKernelGGL((potrf::k_potrf<float, 256, false>), dim3(n_items), dim3(256), 0, L.stream, L.desc, order,
                       L.theta, cx, cy, cv, Lbuf, Inv, logdet, status, nullptr, 0, nullptr);
    return take_z<float>(L, order, n_items, cv, Lbuf, Inv, zout);
  }
  return potrf2_launch<float>(L, order, n_items, cx, cy, cv, zout, Lbuf, Inv, logdet, status, cp);
}
hipError_t launch_potrf_f64(const Launch& L, const int32_t* order, int n_items, const double* cx,
                            const double* cy, const double* cv, double* zout, double* Lbuf, double* Inv,
                            double* logdet, int32_t* status, const CoopPlan* cp) {
  if (cv && !zout) return hipErrorInvalidValue;
  return potrf2_launch<double>(L, order, n_items, cx, cy, cv, zout, Lbuf, Inv, logdet, status, cp);
}

}  // namespace pcv
