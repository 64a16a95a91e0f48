// Shared definitions of the device path (kernels and their host launchers).
// gfx950 only: 64-wide wavefronts, MFMA 16x16x4 for FP32 and FP64.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pcv {

// Tile / block size of the blocked factorisation and of the solves.  Every
// subset is padded to a multiple of TB with points at +infinity: their
// covariance with everything is exactly 0, the factorisation gives them a
// unit diagonal, their right-hand side is 0, so the real part of every
// result is unchanged.
constexpr int TB = 64;
// Subset status codes: 0 = fine, k > 0 = pivot k-1 not positive,
// PCV_STATUS_STAGNATED = mixed-precision refinement did not converge.
constexpr int32_t PCV_STATUS_STAGNATED = -1;
// PCV_STATUS_SYNC_TIMEOUT = a workgroup of a cooperative factorisation waited
// past its bound for another (the factor is not usable; FP64 re-run).
constexpr int32_t PCV_STATUS_SYNC_TIMEOUT = -2;

// Per-subset descriptor.  Offsets are element offsets into the packed
// device arrays.
struct SubsetDesc {
  int64_t offT;    // training panel (coordinates, y_T)          [n]
  int64_t offV;    // validation panel (coordinates, y_V, errors) [m]
  int64_t offP;    // padded vectors (z, alpha, r, x)              [npad]
  int64_t offL;    // packed tile-row lower factor                 [packed_size(npad)]
  int64_t offInv;  // inverse diagonal blocks, FP64                [npad * TB]
  int64_t offPC;   // residual column partials, FP64               [TB * nb (nb - 1) / 2]
  int64_t offX;    // padded factorisation coordinates            [npad]
  int64_t offE;    // validation predictions / squared errors     [m]
  int32_t n, m, npad;
  int32_t th;      // theta slot: kernels read theta[th]
  // Several theta values are evaluated in one launch by replicating the
  // descriptors per theta slot: the per-theta workspace offsets (offP, offL,
  // offInv, offPC, offE) move to that slot's copy of the buffers, the input
  // offsets (offT, offV, offX) stay.
};

// The evaluated parameters, read by every kernel from device memory so that
// one captured sequence serves any theta.
struct ThetaDev {
  int32_t cov;
  int32_t pad;
  double range;
  double inv_range;
  double lambda;
  double sigma2;
};

// Packed tile-row lower storage: row r of block I = r / TB holds columns
// [0, (I+1) TB) contiguously.  Row-major inside a block row, so any
// segment of a row that lies on or below the diagonal block is contiguous.
__host__ __device__ inline int64_t packed_rowoff(int r) {
  const int64_t I = r / TB;
  return (int64_t)TB * TB * (I * (I + 1) / 2) + (int64_t)(r % TB) * (I + 1) * TB;
}
// 32-bit form for indexing inside one subset (npad <= 16384 keeps it < 2^31).
__host__ __device__ inline int packed_rowoff32(int r) {
  const int I = r / TB;
  return TB * TB * (I * (I + 1) / 2) + (r % TB) * (I + 1) * TB;
}
__host__ __device__ inline int64_t packed_size(int npad) {
  const int64_t nb = npad / TB;
  return (int64_t)TB * TB * (nb * (nb + 1) / 2);
}

}  // namespace pcv

// Host-side launchers implemented in pcv_kernels.hip.
namespace pcv {
struct Launch {
  hipStream_t stream;
  const SubsetDesc* desc;
  const ThetaDev* theta;
};
// Cooperative factorisation: blocks 0 .. n_blocks - 1 of the launch share
// subsets, info[b] = rank | nwg << 8 | slot << 16 (rank < nwg <= 255: the
// block is rank `rank` of the nwg on subset order[b]; slot < n_slots picks
// its 4 counters in sync, zeroed by the launcher).  The other blocks work
// alone.  The ranks of a subset must be able to run at the same time: the
// launcher's caller keeps the cooperative blocks first and at most one per
// compute unit.
struct CoopPlan {
  const int32_t* info;
  int n_blocks;
  int32_t* sync;
  int n_slots;
  const int32_t* subsets;  // the launch's subsets, each once (the order list
  int n_subsets;           // repeats shared ones), for the y_T row's move-out
};
// max_npad: the largest padded size among the listed subsets.  FP32 launches
// with max_npad <= small_npad use workgroups of 4 waves (64-column panels,
// two per compute unit), the others 8 waves; FACTOR_SMALL_NPAD is the
// measured crossover for uniform sizes (4 waves faster up to n = 1,250,
// equal at 1,400, slower from 1,500).  n_items counts launch blocks (with
// cp, the cooperative blocks included; cp needs the 8-wave shape).
constexpr int FACTOR_SMALL_NPAD = 1408;
// ... and those whose largest subset has npad <= tiny_npad 2-wave
// workgroups (64-column panels, 64-row chunks, four per compute unit);
// measured on uniform sizes: faster up to n = 600, equal at 700, slower
// from 800.
constexpr int FACTOR_TINY_NPAD = 704;
// cv (may be null): the subsets' y_T values in the coordinates' padded
// layout; then each subset's first padding row (row n) carries them through
// the factorisation and zout receives z = L^{-1} y_T (FP64, at offP, zeros
// from n to npad), the forward substitution of the solve, while the factor
// comes out as without them.  Needs npad > n for every subset with n > 0.
hipError_t launch_potrf_f32(const Launch& L, const int32_t* order, int n_items, int max_npad, const float* cx,
                            const float* cy, const float* cv, double* zout, float* Lbuf, double* Inv,
                            double* logdet, int32_t* status, const CoopPlan* cp = nullptr,
                            int small_npad = FACTOR_SMALL_NPAD, int tiny_npad = FACTOR_TINY_NPAD);
hipError_t launch_potrf_f64(const Launch& L, const int32_t* order, int n_items, const double* cx,
                            const double* cy, const double* cv, double* zout, double* Lbuf, double* Inv,
                            double* logdet, int32_t* status, const CoopPlan* cp = nullptr);
// max_npad: the largest padded size among the launched subsets (selects the
// per-thread register budget of the solve kernels).
// gate (may be null): per descriptor, 0 = skip this subset (a refinement
// sweep it does not take), see launch_refine_gate.
hipError_t launch_trsv_fwd_f32(const Launch& L, const int32_t* order, int n_items, int max_npad,
                               const float* Lbuf, const double* Inv, const double* rhs_train,
                               const double* rhs_pad, double* z, double* rhs2, const int32_t* gate = nullptr);
hipError_t launch_trsv_fwd_f64(const Launch& L, const int32_t* order, int n_items, int max_npad,
                               const double* Lbuf, const double* Inv, const double* rhs_train,
                               const double* rhs_pad, double* z, double* rhs2, const int32_t* gate = nullptr);
hipError_t launch_trsv_bwd_f32(const Launch& L, const int32_t* order, int n_items, int max_npad,
                               const float* Lbuf, const double* Inv, const double* z, double* x,
                               double* alpha_accum, const int32_t* gate = nullptr);
hipError_t launch_trsv_bwd_f64(const Launch& L, const int32_t* order, int n_items, int max_npad,
                               const double* Lbuf, const double* Inv, const double* z, double* x,
                               double* alpha_accum, const int32_t* gate = nullptr);
// Refinement residual r = y_T - (Sigma + lambda I) alpha, each symmetric entry
// generated once: tile items (subset, row block I) sorted by work, and row
// items (subset, row block) for the fixed-order reduction.
hipError_t launch_residual(const Launch& L, const int2* tile_items, int n_tile_items, const int2* row_items,
                           int n_row_items, const double* tx, const double* ty, const double* yT,
                           const double* alpha, double* rrow, double* pcol, double* r,
                           const int32_t* gate = nullptr);
// Before refinement sweep it >= 1, for the descriptors k = order[j], j < n:
// gate[k] = 1 where descriptor k (subset k % S) took sweep it - 1 and that
// sweep's squared residual norm rhs2[k] exceeds tol^2 ynorm2[k % S];
// nsweep[k] = sweeps descriptor k takes.
hipError_t launch_refine_gate(hipStream_t s, int n, const int32_t* order, int S, int it, const double* rhs2,
                              const double* ynorm2, double tol, int32_t* gate, int32_t* nsweep);
hipError_t launch_predict_val(const Launch& L, const int2* items, int n_items, const double* tx,
                              const double* ty, const double* vx, const double* vy,
                              const double* yV, const double* alpha, double* yhat, double* err);
// Kriging of query points from resident FP64 factors (mean and variance).
constexpr int KRIGE_Q = 16;  // queries per kriging item
struct KrigeItem {
  int32_t sidx;    // subset
  int32_t q0;      // first query (in the grouped query arrays)
  int32_t nq;      // queries in this item (<= KRIGE_Q)
  int32_t flags;   // KRIGE_VAR: some query of the item wants its variance
  int64_t woff;    // scratch offset (npad x KRIGE_Q doubles), used with KRIGE_VAR
};
// Per-query flags (and KRIGE_VAR per item).
constexpr int32_t KRIGE_VAR = 1;        // write the kriging variance
constexpr int32_t KRIGE_OBS_NOISE = 2;  // add the nugget variance sigma^2 lambda
// Grouped query j (centred coordinates qx/qy[j], flags qflag[j]) writes
// mean[qorig[j]] and, with KRIGE_VAR, var[qorig[j]].
hipError_t launch_krige(hipStream_t s, const SubsetDesc* desc, const ThetaDev* theta,
                        const KrigeItem* items, int n_items, const double* tx, const double* ty,
                        const double* L64, const double* Inv, const double* alpha, const double* qx,
                        const double* qy, const int32_t* qorig, const int32_t* qflag,
                        double* Wscratch, double* mean, double* var);
// GLS coefficients (p <= GLS_MAXP covariates): X and W = M^{-1} X as p
// padded vectors of nP entries each (column j at j * nP + offP); beta
// [S][p]; status[i] = j + 1 when the normal matrix is not positive
// definite at column j (beta then NaN).
constexpr int GLS_MAXP = 8;
hipError_t launch_gls(hipStream_t s, const SubsetDesc* desc, const int32_t* order, int n_items, int p,
                      int64_t nP, const double* Xp, const double* Wp, const double* alpha, double* beta,
                      int32_t* status);
// quad[order[k]] = y_T^T alpha of subset order[k], k < n_items.
hipError_t launch_quad(hipStream_t s, const SubsetDesc* desc, const int32_t* order, int n_items,
                       const double* yT, const double* alpha, double* quad);
// Per-subset SSPE and the global loss (fixed-order compensated sums), count
// of subsets with nonzero status, for n_theta theta slots of S descriptors
// each (slot t: descriptors t S .. t S + S - 1, outputs out_total[t],
// out_nbad[t]).  With rhs2 non-null, an active subset with
// rhs2 > tol^2 * ynorm2 gets status PCV_STATUS_STAGNATED first.
hipError_t launch_reduce(hipStream_t s, const SubsetDesc* desc, int S, int n_theta, const double* err,
                         int32_t* status, const int32_t* active, const double* rhs2,
                         const double* ynorm2, double tol, double* per_subset_sspe,
                         double* out_total, int32_t* out_nbad);
// Testing hook: e[i] = e^{-t[i]} and r[i] = sqrt(x[i]) by the FP64 device
// functions of the residual and the kriging of validation points.
hipError_t launch_math_check(hipStream_t s, int64_t n, const double* t, const double* x, double* e, double* r);
}  // namespace pcv
