// Register-resident truncation kernel for blocks larger than 64 x 64 with a
// stacked rank of at most 64 (see tall.h).  It is launched on the same items as
// the general kernel, after the one-wave kernel for stacked ranks of at most
// 16 (trunc_thin.hip); each marks the items it takes in `done`, and the
// kernels after it skip those.
#include <hip/hip_runtime.h>

#include "tall.h"

namespace hm {

__global__ __launch_bounds__(TALL_TB) void trunc_tall_kernel(const DTrunc* __restrict__ descs,
                                                             const DTruncPart* __restrict__ parts,
                                                             double* __restrict__ pool, long long pool_doubles,
                                                             unsigned long long* counter, int* status, double eps,
                                                             int* size_log, int* done, int run_id) {
  extern __shared__ double smem[];
  __shared__ TallShared sh;
  __shared__ int l_sh, skip_sh;
  __shared__ long long ws_sh;
  if (done[blockIdx.x] == run_id) return;  // done by trunc_thin_kernel
  const DTrunc d = descs[blockIdx.x];
  if ((d.flags & TRUNC_CLASS_CHECK) && d.m <= TRUNC_SMALL_MAX && d.n <= TRUNC_SMALL_MAX) return;  // small-block kernel's
  const int tid = threadIdx.x;
  if (tid < 64) {
    const StackCounts sc = stacked_counts(parts, d.part0, d.nparts, sh.k, sh.coff, sh.part);
    if (tid == 0) {
      l_sh = sc.l;
      skip_sh = ((d.flags & TRUNC_SKIP_IF_PART0_EMPTY) && sc.k0 == 0) ||
               ((d.flags & TRUNC_SKIP_IF_HEAD_EMPTY) && sc.l == sc.klast);
    }
  }
  __syncthreads();
  const int l = l_sh;
  if (skip_sh || l == 0 || !tall_fits(d.m, d.n, l)) return;  // other kernel (l == 0 included)
  if (tid == 0) {
    const long long need = tall_ws_need(d.m, d.n, l);
    const unsigned long long off = atomicAdd(counter, (unsigned long long)need);
    if ((long long)off + need > pool_doubles) {
      atomicOr(status, ST_WS_OVERFLOW);
      ws_sh = -1;
    } else {
      ws_sh = (long long)off;
    }
  }
  __syncthreads();
  if (ws_sh < 0) return;
  // mark the item: the general kernel, launched next on the same items, skips
  // it (it cannot decide by itself: this kernel changes the target's rank,
  // which is the column count of one of the item's parts)
  if (tid == 0) done[blockIdx.x] = run_id;
  tall_path(d, sh, d.nparts, l, pool + ws_sh, smem, status, eps, size_log);
}

hipError_t launch_trunc_thin(const DTrunc* descs, const DTruncPart* parts, int count, int* status, double eps,
                             int* size_log, int* done, int run_id, hipStream_t stream);

// With thin, the one-wave kernel first; then the register-resident kernel.
hipError_t launch_trunc_tall(const DTrunc* descs, const DTruncPart* parts, int count, double* pool,
                             int64_t pool_doubles, int* counter, int* status, double eps, int* size_log,
                             int* done, int run_id, hipStream_t stream, bool thin) {
  if (count <= 0) return hipSuccess;
  if (thin) {
    const hipError_t e = launch_trunc_thin(descs, parts, count, status, eps, size_log, done, run_id, stream);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(trunc_tall_kernel, dim3(count), dim3(TALL_TB), TALL_LDS_DOUBLES * 8, stream, descs, parts, pool,
                     (long long)pool_doubles, (unsigned long long*)counter, status, eps, size_log, done, run_id);
  return hipGetLastError();
}

}  // namespace hm
