// Batched persistent solver (host interface).
#pragma once

#include <vector>

#include "common.hpp"

namespace qp {

// One matrix of a batch (device pointers, FP32 storage).  X_b is n x m.  The phase-synchronous kernel
// also reads the matrix's workspace offsets (elements into its float pool, double partial-sum array and
// double vector scratch) and the row strides of its s x s and n x m work buffers.
struct BDesc {
  const float* A;
  int64_t lda, psa;
  float* X;
  int64_t ldx, psx;
  int m, n;
  int64_t off = 0, poff = 0, doff = 0;
  int64_t lds = 0, pss = 0, ldw = 0, psw = 0;
  int64_t ldap = 0, psap = 0;  // copy of A with 16-byte aligned rows (ldap = 0: A itself is aligned)
};

// Per-matrix outcome written by the kernel.
struct BInfo {
  int iters, returned, reason, status;
  double alpha, dx_rel, sigma1_sq;
};

// Everything the captured graph bakes in.
struct BKey {
  int count = 0, D = 0, cfg = 0, method = 0, stop = 0, max_iter = 0, scaling = 0, power_steps = 0;
  int dyn = 1;  // phase-synchronous form: workgroups take work items from a counter (0: items g, g + G, ...)
  double tol = 0.0;
  unsigned long long seed = 0;
  bool operator==(const BKey& o) const {
    return count == o.count && D == o.D && cfg == o.cfg && method == o.method && stop == o.stop &&
           max_iter == o.max_iter && scaling == o.scaling && power_steps == o.power_steps && dyn == o.dyn &&
           tol == o.tol && seed == o.seed;
  }
};

// Device buffers, pinned staging buffers and the captured graph of the last batch signature.
struct BatchedState {
  BKey key;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t stream = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  BDesc* h_desc = nullptr;
  BInfo* h_info = nullptr;
  int* h_order = nullptr;
  double* h_alpha = nullptr;
  unsigned long long* h_trace = nullptr;
  int grid = 0;
  std::vector<void*> dev;
  // phase-synchronous configurations: capacities the captured graph was built for
  int64_t pool_cap = 0, part_cap = 0, dw_cap = 0;
  ~BatchedState();
};

// Phase-synchronous configurations keep every matrix's work buffers in one pool: fill the offsets and
// strides of `desc` and return the pool, partial-sum and vector scratch sizes (elements).
void batched_layout(std::vector<BDesc>& desc, int cfg, int64_t& pool, int64_t& part, int64_t& dwork);
bool batched_is_sync(int cfg);

// Upload the batch, replay (or build) the graph and wait for it; infos receives the outcomes.
void run_batched(BatchedState& st, const BKey& key, const std::vector<BDesc>& desc, const std::vector<int>& order,
                 const std::vector<double>& alphas, std::vector<BInfo>& infos, hipStream_t caller,
                 bool verbose = false);

int batched_num_configs();
const char* batched_config_name(int cfg);
// configurations used without autotuning: phase-synchronous 32 x 32 x 32 tiles, and the queue form
// with 64 x 64 tiles for batches beyond the phase-synchronous limit
constexpr int kBatchedDefaultSync = 5;
constexpr int kBatchedDefaultQueue = 2;

}  // namespace qp
