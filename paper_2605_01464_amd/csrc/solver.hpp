// Solver driver: context, workspace, method chains and the solve loop.
#pragma once

#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/qpinv.h"
#include "common.hpp"
#include "qgemm.hpp"

namespace qp {

// Grow-only named device allocations, freed with the context.  In arena mode (allocation-free solves)
// the same named requests are carved, 256-byte aligned, from a caller-provided region instead: no
// allocation, and a request that does not fit throws EINVAL.
struct Workspace {
  struct Buf {
    void* p = nullptr;
    size_t bytes = 0;
  };
  std::map<std::string, Buf> bufs;
  char* arena = nullptr;
  size_t arena_cap = 0, arena_used = 0;
  std::map<std::string, Buf> arena_bufs;
  void* get(const std::string& key, size_t bytes);
  void begin_arena(void* base, size_t cap);
  void end_arena();
  void release();
  ~Workspace() { release(); }
};

struct Options {
  int side = QPINV_SIDE_AUTO;
  int power_steps = 8;
  uint64_t power_seed = 0x5EED;
  int autotune = 0;
  int f64_finish_iters = 2;
  int f64_refined = 1;  // 1: FP64 finish updates with FP64 residual and sum, FP32 polynomial (NS, HPI, QSAI, QHPI19)
  int finish_method = QPINV_NS;  // method of the FP64 finish updates (-1: the solve's own method)
  int penrose_finish = 0;        // FP64 projection of the returned iterate: 0 none, 1 X A X, 2 (X A)^H X (A X)^H
  int small_path = 1;            // single solves of at most 128 per side in one launch (small.hip) when eligible
  int small_gram = 1;            // one-launch FP64 solves: the Gram matrix formed during the set-up (small.hip)
  int fault_small_giveup = 0;    // test hook: the one-launch solve starts with its barrier's give-up flag raised
  double mixed_switch = 1e-2;
  int mixed_rnorm_steps = 6;
  int max_bf16_iters = 8;
  int mixed_split = 1;  // ladder: products of its FP32 phase and finish as three BF16 products (P_BF16X3)
  int verbose = 0;
  int gemm_timing = 0;
  int force_cfg[4] = {-1, -1, -1, -1};  // per product precision: tile configuration for every product, -1 = choose
  int batched_cfg = -1;             // batched kernel configuration, -1 = tuned or default
  int batched_dynamic = 1;          // phase-synchronous batched form: dynamic (1) or static (0) item dealing
};

struct MlpState;      // scaling network (mlp.hip)
struct BatchedState;  // batched persistent solver (batched.hip)

struct Ctx {
  int device = 0;
  Options opt;
  Workspace ws;
  GemmScratch scratch;
  double* dsc = nullptr;  // device scalars
  double* hsc = nullptr;  // pinned host scalars
  static constexpr size_t kStageBytes = 32768;
  void* hstage = nullptr;  // pinned host staging area for small parameter blocks (kStageBytes)
  std::map<std::tuple<int, int64_t, int64_t, int64_t>, int> tuned;
  MlpState* mlp = nullptr;
  BatchedState* batched = nullptr;
  std::map<std::vector<int64_t>, int> batched_tuned;  // batch signature -> tile configuration
  bool no_alloc = false;  // allocation-free call in progress: no autotuning, no product timing, no growth
  bool split_f32 = false;  // a ladder solve in progress computes its FP32-storage products as P_BF16X3
  void* small_state = nullptr;  // the small solve's record whose barrier words hold a known count and a clear flag
  unsigned int small_bar_base = 0;  // the arrival count those barrier words hold
  void* small_params_dev = nullptr;         // the small solve's parameter block in device memory, and
  std::vector<unsigned char> small_params;  // the bytes it holds (copied again only when they change)
  double flops = 0.0;  // running count of algorithmic product flops
  // event pairs around product launches (option gemm_timing)
  std::vector<std::pair<hipEvent_t, hipEvent_t>> events;
  std::vector<double> event_flops;
  std::vector<int> event_key;  // prec * 64 + tile configuration
  size_t events_used = 0;

  explicit Ctx(int dev);
  ~Ctx();
  int config_for(Prec p, int64_t M, int64_t N, int64_t K, hipStream_t s);
};

// A quaternion matrix with its shape and element type.
struct Mat {
  QView v;
  int64_t rows = 0, cols = 0;
  int dtype = QPINV_F32;
};

Mat from_abi(const qpinv_qmat& q);
void validate(const qpinv_qmat* q, const char* what);

// Workspace matrix of the given shape/type (ld padded to a multiple of 8 elements).
Mat ws_mat(Ctx& c, const std::string& key, int64_t rows, int64_t cols, int dtype);

// C = A B with epilogue (adds the flops to c.flops; uses tuned/default tile configuration).
void gemm(Ctx& c, Prec p, const Mat& A, const Mat& B, const Epilogue& e, hipStream_t s, double* red = nullptr);

// One iteration of `method` from Xc into Xn.  A and X share the element type of `p`'s storage.
// If red != nullptr, red (device, 2 doubles) receives {||Xn - Xc||^2, ||Xn||^2}.
// If Rout != nullptr it receives a view of R_j = I - (side product) (s x s) for norm estimates.
void chain(Ctx& c, int method, int order, int side, Prec p, const Mat& A, const Mat& Xc, const Mat& Xn, double* red,
           hipStream_t s, Mat* Rout = nullptr);

int solve(Ctx& c, int method, int order, const qpinv_qmat* A, int scaling, double alpha_or_mu, double tol,
          int max_iter, int stop, int precision, qpinv_qmat* X, qpinv_info* info, hipStream_t s);

// The same solve with every workspace buffer carved from the device's static no-allocation scratch (noalloc.hip).
int solve_noalloc(Ctx& c, int method, int order, const qpinv_qmat* A, int scaling, double alpha_or_mu, double tol,
                  int max_iter, int stop, int precision, qpinv_qmat* X, qpinv_info* info, hipStream_t s);

// One-launch solve of a small matrix (small.hip): eligibility and the solve (returns a status code).
bool small_eligible(const Ctx& c, int method, int order, int scaling, int stop, int precision, int64_t m, int64_t n);
int small_solve(Ctx& c, int method, int order, const Mat& A0, int scaling, double am, double tol, int max_iter,
                int stop, int precision, const Mat& Xout, qpinv_info& inf, hipStream_t s);

// Address of the device's no-allocation scratch, looked up once per device with that device current (noalloc.hip).
void* noalloc_scratch(int device);

// Upper bound of the workspace bytes one solve of an m x n matrix can request (noalloc.hip).
size_t noalloc_workspace_bound(int64_t m, int64_t n, int side, int precision, int out_dtype);

int solve_batched(Ctx& c, int method, int order, int batch, const qpinv_qmat* A, qpinv_qmat* X, int scaling,
                  const double* alpha, double tol, int max_iter, int stop, qpinv_info* infos, hipStream_t s);

void residuals(Ctx& c, const qpinv_qmat* A, const qpinv_qmat* X, double E_abs[4], double E_rel[4], hipStream_t s);

void features(Ctx& c, const Mat& A, int steps, double out[7], hipStream_t s);

// Per kernel (precision, tile configuration): rows of {prec, cfg, launches, flops, milliseconds} of the
// timed product launches since the last call; returns the row count (at most max_rows) and resets.
int gemm_stats(Ctx& c, double* out, int max_rows);

int autotune(Ctx& c, Prec p, int64_t M, int64_t N, int64_t K, double* best_ms, hipStream_t s);

// Normalised method parameters; throws EINVAL on a bad order.
void check_method(int method, int& order);

}  // namespace qp
