// Internal pieces shared by the C ABI sources: the handle types, device
// storage of a structure, and the batched launch of truncation items.
#pragma once
#include <memory>
#include <vector>

#include "api_util.h"
#include "planner.h"
#include "program.h"
#include "structure.h"

namespace hm {
hipError_t launch_trunc(const DTrunc* descs, const DTruncPart* parts, int count, double* pool, int64_t pool_doubles,
                        int* counter, int* status, double eps, int* size_log, const int* done, int run_id,
                        hipStream_t stream);
hipError_t launch_trunc_tall(const DTrunc* descs, const DTruncPart* parts, int count, double* pool,
                             int64_t pool_doubles, int* counter, int* status, double eps, int* size_log,
                             int* done, int run_id, hipStream_t stream, bool thin);
hipError_t launch_trunc_small(const DTrunc* descs, const DTruncPart* parts, int count, int* status, double eps,
                              int* size_log, int tpc, const DPredictor* pred, float* feat_log, int prec,
                              hipStream_t stream, int ntiny = 0);
MlpWeights hm_mlp_weights(const hm_mlp* n);

// Device storage for a structure: dense leaves first (contiguous), then the
// low-rank factors (A: rows x cap, B: cols x cap per block), ranks separately;
// everything zero.  dense_off (may be NULL) receives each block's offset in
// doubles.
std::shared_ptr<DevHMatrix> allocate(const AllocRef& alloc, std::shared_ptr<ClusterTree> ct, const BlockTree& bt,
                                     int kmax, std::vector<size_t>* dense_off);

// Workspace (doubles) that the register-resident and general truncation
// kernels may claim for one item of m x n with stacked rank l.
int64_t trunc_ws_doubles(int m, int n, int l);

// Runs a batch of independent truncation items (descriptors and parts built on
// the host) on the context's stream: small-block kernel for m, n <= 64, the
// register-resident and general kernels for the rest.  Reorders dt.  Waits for
// the stream; returns the status bits and adds the executed truncations to
// *executed (may be NULL).  pred (host, may be NULL) attaches the rank
// predictor to the small items.
int run_trunc_items(hm_ctx* ctx, std::vector<DTrunc>& dt, const std::vector<DTruncPart>& dp, double eps, int prec,
                    const DPredictor* pred, int64_t* executed, int64_t* accepted, int64_t* fell_back);

hm_status status_to_error(int bits);
double now_seconds();
}  // namespace hm

struct hm_matrix {
  std::shared_ptr<hm::DevHMatrix> M;
};

struct hm_plan {
  std::unique_ptr<hm::Program> P;
  hm::DPredictor* pred_dev = nullptr;  // device copy of the attached predictor
  std::vector<std::shared_ptr<hm::DevHMatrix>> targets;  // the matrices the plan writes (G of an H-LU, Z of a product)
  std::vector<std::unique_ptr<hm::PNode>> roots;
  hm::PlanCounts counts;
  double plan_seconds = 0;
  double phase_seconds[3] = {0, 0, 0};  // record, schedule, upload
  bool uploaded = false;
};
