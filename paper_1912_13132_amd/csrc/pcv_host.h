// Host-side state of a resident problem and the internal entry points
// behind the C ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/pcv.h"
#include "pcv_device.h"

struct pcv_problem {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  pcv_options opt{};

  int64_t n = 0;
  int32_t S = 0;
  std::vector<pcv::SubsetDesc> desc;
  std::vector<int32_t> active;      // subset has >= 1 validation point
  std::vector<int32_t> order_eval;  // active subsets, largest n^3 first
  std::vector<int32_t> order_all;   // subsets with >= 1 training point, largest first
  std::vector<int2> row_items_eval; // (subset, 64-row block) over order_eval
  std::vector<int2> tile_items;     // (subset, row block I), by decreasing I (residual tiles)
  std::vector<int2> val_items;      // (subset, 64-point validation block)
  std::vector<double> core_rect;    // S x 4, empty when not given
  std::vector<double> centroid;     // S x 2
  std::vector<double> ynorm2;       // S: ||y_T||^2
  int64_t nnzT = 0, nnzV = 0, nP = 0, nL = 0, nInv = 0, n_val_total = 0;
  int32_t max_train = 0;
  int32_t max_npad = 0;
  int32_t n_active = 0;

  // device copies
  pcv::SubsetDesc* d_desc = nullptr;
  int32_t* d_order_eval = nullptr;
  int32_t* d_order_all = nullptr;
  int32_t* d_active = nullptr;
  int2* d_row_items = nullptr;
  int2* d_tile_items = nullptr;
  double *d_rrow = nullptr, *d_pcol = nullptr;
  int64_t nPC = 0;
  int2* d_val_items = nullptr;
  double *d_tx = nullptr, *d_ty = nullptr, *d_yT = nullptr, *d_ynorm2 = nullptr;
  // factorisation coordinates, padded to npad per subset with +inf (offP)
  double *d_px64 = nullptr, *d_py64 = nullptr;
  float *d_px32 = nullptr, *d_py32 = nullptr;
  double *d_vx = nullptr, *d_vy = nullptr, *d_yV = nullptr;
  double *d_z = nullptr, *d_x = nullptr, *d_alpha = nullptr, *d_r = nullptr, *d_rhs2 = nullptr;
  double *d_yhat = nullptr, *d_err = nullptr;
  double *d_logdet = nullptr, *d_sspe = nullptr;
  int32_t* d_status = nullptr;
  pcv::ThetaDev* d_theta = nullptr;
  double* d_total = nullptr;
  int32_t* d_nbad = nullptr;
  float* d_L32 = nullptr;
  double* d_L64 = nullptr;
  double* d_Inv = nullptr;
  // FP64 factors kept for prediction (pcv_factor); separate from the
  // evaluation workspace so that evaluations do not disturb them
  double* d_Lf = nullptr;
  double* d_Invf = nullptr;
  double* d_alpha_fact = nullptr;
  double* d_zf = nullptr;
  double* d_logdetf = nullptr;
  int32_t* d_statusf = nullptr;
  pcv::ThetaDev* d_theta_fact = nullptr;

  // pinned host mirrors
  pcv::ThetaDev* h_theta = nullptr;
  double* h_total = nullptr;
  int32_t* h_nbad = nullptr;

  size_t dev_bytes = 0;
  std::vector<void*> allocs;
  hipEvent_t ev[8] = {};
  bool events = false;

  bool factored = false;
  pcv_theta fact_theta{};
};

namespace pcv {
extern thread_local std::string g_err;
pcv_status fail(pcv_status s, const std::string& msg);
pcv_status problem_build(pcv_problem* p, int64_t n, const double* locs, const double* y, int32_t S,
                         const int64_t* train_ptr, const int32_t* train_idx, const int64_t* val_ptr,
                         const int32_t* val_idx, const double* core_rect);
void problem_free(pcv_problem* p);
pcv_status eval_impl(pcv_problem* p, const pcv_theta& th, double* loss, pcv_eval_report* rep);
pcv_status factor_impl(pcv_problem* p, const pcv_theta& th);
pcv_status predict_impl(pcv_problem* p, int64_t q, const double* qlocs, double* mean, double* var,
                        int32_t obs_noise, int32_t* owner);
}  // namespace pcv
