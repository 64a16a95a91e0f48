// Host-side state of a resident problem and the internal entry points
// behind the C ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <utility>
#include <vector>

#include "../../include/pcv.h"
#include "pcv_device.h"

namespace pcv {
// Host plan of one kriging launch: queries grouped by owning subset, in
// 64-query items.  Input j of the plan is query j of the caller's list.
struct KrigePlan {
  std::vector<double> qx, qy;      // grouped, centred on the subset centroid
  std::vector<int32_t> qorig;      // grouped -> input index
  std::vector<int32_t> qflag;      // grouped flags (KRIGE_VAR | KRIGE_OBS_NOISE)
  std::vector<KrigeItem> items;
  int64_t w_doubles = 0;           // variance scratch
  std::vector<int32_t> cnt, pos;   // counting-sort work arrays (size S)
};
}  // namespace pcv

// Bucket grid over the core rectangles for routing query locations
// (built once per problem when core rectangles are given).
struct pcv_router {
  int G = 0;
  double xmin = 0, ymin = 0, xmax = 0, ymax = 0, bw = 0, bh = 0;
  std::vector<int32_t> ptr, list;  // CSR: cores touching bucket b
};

// Workspace for evaluating several theta values in one launch per kernel:
// B theta slots, the descriptors replicated per slot (see SubsetDesc), and
// per group size nb <= B the item lists over (slot, subset) pairs and the
// captured graph.
struct pcv_batch_plan {
  int nb = 0;
  int32_t* d_order = nullptr;
  int2 *d_row_items = nullptr, *d_tile_items = nullptr, *d_val_items = nullptr;
  int n_order = 0, n_row = 0, n_tile = 0, n_val = 0;
  hipGraphExec_t graph = nullptr;
};
struct pcv_batch {
  int B = 0;
  pcv::SubsetDesc* d_desc = nullptr;
  void* d_L = nullptr;  // FP32 (mixed) or FP64 factors, B copies
  double *d_Inv = nullptr, *d_z = nullptr, *d_x = nullptr, *d_alpha = nullptr, *d_r = nullptr;
  double *d_rrow = nullptr, *d_pcol = nullptr, *d_rhs2 = nullptr, *d_yhat = nullptr, *d_err = nullptr;
  double *d_logdet = nullptr, *d_sspe = nullptr, *d_quad = nullptr, *d_total = nullptr;
  int32_t *d_status = nullptr, *d_nbad = nullptr;
  int32_t *d_gate = nullptr, *d_nsweep = nullptr;  // refinement sweeps taken, per descriptor
  pcv::ThetaDev* d_theta = nullptr;
  pcv::ThetaDev* h_theta = nullptr;  // pinned [B]
  double* h_total = nullptr;         // pinned [B]
  int32_t* h_nbad = nullptr;         // pinned [B]
  pcv_batch_plan plans[2];
};

// A contiguous group of order_eval and its slices of the item lists: subsets
// order_eval[o0, o0 + cnt), row and tile items [r0, r0 + nr), validation
// items [v0, v0 + nv).
struct pcv_group {
  int32_t o0 = 0, cnt = 0;
  int32_t r0 = 0, nr = 0;
  int32_t v0 = 0, nv = 0;
};

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
  std::vector<int2> tile_items;     // (subset, row block I), by decreasing I within each
                                    // group of the schedule (residual tiles)
  std::vector<int2> val_items;      // (subset, 64-point validation block)
  std::vector<double> core_rect;    // S x 4, empty when not given
  pcv_router router;
  std::vector<double> centroid;     // S x 2
  std::vector<double> ynorm2;       // S: ||y_T||^2
  std::vector<int64_t> train_ptr;   // S + 1 (training CSR, kept for covariates)
  std::vector<int32_t> train_idx;
  int64_t nnzT = 0, nnzV = 0, nP = 0, nL = 0, nInv = 0, n_val_total = 0;
  int32_t max_train = 0;
  int32_t max_npad = 0;
  int32_t n_active = 0;
  // Evaluation schedule.  g_all covers every evaluated subset; groups split
  // order_eval into consecutive groups of whole rounds of one factorisation
  // work-group per compute unit (the last group holds the remainder).  The
  // factorisations run group after group on the problem's stream; each
  // group's solves, refinement and kriging follow on one of two further
  // streams, beside the next group's factorisation, so that the remainder
  // group does not leave most compute units idle.
  // The post streams are made at the first evaluation that uses them.  A
  // problem served by a pcv_server evaluates on its one stream (served), so
  // that the server's kriging streams keep hardware queues of their own.
  pcv_group g_all;
  std::vector<pcv_group> groups;
  bool served = false;
  int32_t n_cu = 0;                 // compute units of the device
  hipStream_t post_stream[2] = {};
  std::vector<hipEvent_t> ev_fact;
  hipEvent_t ev_post[2] = {};
  // The first factorisation launch of an evaluation (coop_group_cnt subsets
  // of order_eval) with its largest subsets shared by several work-groups:
  // coop_order lists the launch's blocks (coop_blocks shared ones first,
  // then the other subsets alone), coop_info each shared block's rank, rank
  // count and counter slot (coop_slots of them).  Empty when no subset is
  // shared.
  int32_t coop_group_cnt = 0;
  int32_t coop_blocks = 0, coop_slots = 0;
  std::vector<int32_t> coop_order, coop_info;
  int32_t *d_coop_order = nullptr, *d_coop_info = nullptr, *d_coop_sync = nullptr;
  bool coop_now = false;  // the current evaluation's first launch is shared
  // Launch shapes and schedule (defaults, or the autotuner's choice): FP32
  // factorisations whose schedule group's largest subset pads to at most
  // tune_small_npad rows use 4-wave work-groups; tune_two_groups turns the
  // two-group schedule on; opt.max_wg_per_subset bounds the sharing.
  int32_t tune_small_npad = pcv::FACTOR_SMALL_NPAD;
  bool tune_two_groups = true;

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
  // y_T in the same padded layout (zeros in padding): the factorisation's
  // y_T row (forward substitution)
  double* d_pv64 = nullptr;
  float* d_pv32 = nullptr;
  double *d_vx = nullptr, *d_vy = nullptr, *d_yV = nullptr;
  double *d_z = nullptr, *d_x = nullptr, *d_alpha = nullptr, *d_r = nullptr, *d_rhs2 = nullptr;
  double *d_yhat = nullptr, *d_err = nullptr;
  double *d_logdet = nullptr, *d_sspe = nullptr, *d_quad = nullptr;
  int32_t* d_status = nullptr;
  int32_t* d_bad = nullptr;         // subsets re-run in FP64
  // mixed path: FP64 factors of the re-run subsets only, packed one after
  // the other (grow-only), and descriptors pointing into it
  double* d_L64fb = nullptr;
  int64_t L64fb_cap = 0;
  pcv::SubsetDesc* d_desc_fb = nullptr;
  int32_t *d_gate = nullptr, *d_nsweep = nullptr;  // refinement sweeps taken, per subset
  // error estimate (opt.est_error): predictions, squared errors, per-subset
  // SSPE and total from alpha after one more sweep; allocated on first use
  double *d_est_yhat = nullptr, *d_est_err = nullptr, *d_est_sspe = nullptr, *d_est_total = nullptr;
  int32_t* d_est_nbad = nullptr;
  // captured theta-evaluation: [0] as planned, [1] with one work-group per
  // subset (used while another shared launch is in flight on the device)
  hipGraphExec_t graph_exec[2] = {};
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
  pcv::ThetaDev* d_theta_fact = nullptr;      // [S]: slot 0, or slot i per subset
  pcv::SubsetDesc* d_desc_local = nullptr;    // descriptors with th = i
  const pcv::SubsetDesc* d_desc_fact = nullptr;  // descriptors the factors were made with

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

  pcv_batch batch;

  // host buffers of pcv_predict_noalloc, reused from call to call
  pcv::KrigePlan na_plan;
  std::vector<int32_t> na_owner;
  std::vector<std::pair<int32_t, int32_t>> na_groups;
  std::vector<double> na_q;
};

namespace pcv {
extern thread_local std::string g_err;
pcv_status fail(pcv_status s, const std::string& msg);
pcv_status problem_build(pcv_problem* p, int64_t n, const double* locs, const double* y, int32_t S,
                         const int64_t* train_ptr, const int32_t* train_idx, const int64_t* val_ptr,
                         const int32_t* val_idx, const double* core_rect);
void problem_free(pcv_problem* p);
pcv_status eval_impl(pcv_problem* p, const pcv_theta& th, double* loss, pcv_eval_report* rep);
// n_theta evaluations, batched B at a time when the workspace allows.
// per_subset_sspe (may be null): [n_theta][S] local losses.
pcv_status eval_batch_impl(pcv_problem* p, int32_t n_theta, const pcv_theta* thetas, double* losses,
                           pcv_eval_report* rep, double* per_subset_sspe = nullptr);
pcv_status factor_impl(pcv_problem* p, const pcv_theta* th, bool local);
pcv_status gls_impl(pcv_problem* p, int32_t ncov, const double* X, double* beta, int32_t* status);
// Single-stream evaluation schedule while a server holds the problem (on)
// or the two-stream schedule again (off); drops the captured evaluation.
pcv_status set_served(pcv_problem* p, bool on);
// Sharing plan of the first factorisation launch (coop_* fields) for the
// current schedule groups and max_wg_per_subset; host side only.
void plan_coop(pcv_problem* p);
// Launch shapes and schedule of later evaluations (drops the captured ones).
pcv_status apply_tuning(pcv_problem* p, int32_t small_npad, int32_t max_wg, bool two_groups);
pcv_status autotune_impl(pcv_problem* p, const pcv_theta& th, const char* cache_path, int32_t reps,
                         pcv_tune_report* rep);
pcv_status predict_impl(pcv_problem* p, int64_t q, const double* qlocs, double* mean, double* var,
                        int32_t obs_noise, int32_t* owner, bool dev_out = false);
// predict_impl with every device buffer in the library's fixed scratch array
pcv_status predict_noalloc_impl(pcv_problem* p, int64_t q, const double* qlocs, double* mean, double* var,
                                int32_t obs_noise, int32_t* owner, bool dev_out);
pcv_status server_create(pcv_server** out, pcv_problem* p, size_t mem_budget, int32_t max_inflight,
                         int32_t n_slots);
pcv_status server_submit_predict(pcv_server* s, int64_t q, const double* ql, double* mean, double* var,
                                 int32_t obs_noise, pcv_ticket* ticket);
pcv_status server_submit_eval(pcv_server* s, const pcv_theta& th, double* loss, pcv_ticket* ticket);
pcv_status server_wait(pcv_server* s, pcv_ticket t, double timeout_s);
pcv_status server_set_window(pcv_server* s, double seconds);
pcv_status server_report(pcv_server* s, pcv_server_report* out);
pcv_status server_destroy(pcv_server* s);
const pcv_problem* server_problem(const pcv_server* s);

pcv_status part_divide(int64_t n, const double* locs, const double* domain, int32_t m, double delta,
                       double* core_rect);
pcv_status part_subsets(int64_t n, const double* locs, int32_t S, const double* core_rect, double delta,
                        const uint8_t* is_val, int32_t* owner, int64_t* memberships, int64_t* train_ptr,
                        int32_t* train_idx, int64_t* val_ptr, int32_t* val_idx);

// Owning subset of each query location (half-open cores, nearest core
// outside all of them; nearest training centroid without core rectangles).
void route(const pcv_problem* p, int64_t q, const double* ql, int32_t* owner);

// owner[j] is the subset of query j; flags[j] its flags (or `flag_all` when
// flags is null).  Items get scratch only when they need the variance.
void plan_krige(const pcv_problem* p, int64_t q, const double* ql, const int32_t* owner,
                const int32_t* flags, int32_t flag_all, KrigePlan& plan);
}  // namespace pcv
