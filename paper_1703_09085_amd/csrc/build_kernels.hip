// Device kernels of the H-matrix builders: entries of the kernel matrix
// 1/|x - y| (the sphere workload standing in for the boundary-element
// matrices of Sect. 7), and the lowering of truncation descriptors that a
// caller made on the device.
#include <hip/hip_runtime.h>

#include "../../include/hm.h"
#include "build_kernels.h"
#include "hm_types.h"

namespace hm {

// One 64 x 64 tile of a block per workgroup of 256 threads: lane r of the
// wave takes row r0 + r, the four waves take every fourth column.  Writes
// are coalesced along the columns (column-major storage).  The squared
// distance is summed over the axes in order without fused multiply-adds, and
// the entry is the correctly rounded 1 / sqrt of it; equal positions in
// cluster order (the same point) get the diagonal value.
__global__ __launch_bounds__(256) void kmat_eval_kernel(const KEvalTile* __restrict__ tiles,
                                                        const double* __restrict__ xs, long long n, int dim,
                                                        double diag) {
  const KEvalTile T = tiles[blockIdx.x];
  const int r = T.r0 + (threadIdx.x & 63);
  if (r >= T.m) return;
  const long long gi = (long long)T.ro + r;
  double xi[3] = {0.0, 0.0, 0.0};
  for (int d = 0; d < dim; ++d) xi[d] = xs[d * n + gi];
  const int cend = T.c0 + 64 < T.n ? T.c0 + 64 : T.n;
  for (int c = T.c0 + (threadIdx.x >> 6); c < cend; c += 4) {
    const long long gj = (long long)T.co + c;
    double v;
    if (gi == gj) {
      v = diag;
    } else {
      double d2 = 0.0;
      for (int d = 0; d < dim; ++d) {
        const double g = __dsub_rn(xi[d], xs[d * n + gj]);
        d2 = __dadd_rn(d2, __dmul_rn(g, g));
      }
      v = 1.0 / sqrt(d2);
    }
    T.out[r + (size_t)c * T.ld] = v;
  }
}

hipError_t launch_kmat_eval(const KEvalTile* tiles, int64_t ntiles, const double* xs, int64_t n, int dim, double diag,
                            hipStream_t stream) {
  for (int64_t t0 = 0; t0 < ntiles; t0 += (1 << 30)) {
    const int64_t cnt = ntiles - t0 < (1 << 30) ? ntiles - t0 : (1 << 30);
    hipLaunchKernelGGL(kmat_eval_kernel, dim3((unsigned)cnt), dim3(256), 0, stream, tiles + t0, xs, (long long)n,
                       dim, diag);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Lowering of caller-made descriptors (hm_trunc_desc, device memory) to the
// kernels' items: the update alpha A B^T and the current block C D^T as two
// parts of one truncation into (Cout, Dout).  Every truncation kernel is
// launched on every item and takes only those of its size class.  An item
// that is invalid or beyond the caller's bounds is turned into a no-op (an
// empty first part with the skip flag) and reported in the status word.
__global__ void lower_trunc_descs_kernel(const hm_trunc_desc* __restrict__ in, int count, int max_rows,
                                         int max_stack, DTrunc* __restrict__ dt, DTruncPart* __restrict__ dp,
                                         int* status) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const hm_trunc_desc h = in[i];
  const bool ok = h.m >= 1 && h.n >= 1 && h.m <= max_rows && h.n <= max_rows && h.k1 >= 0 && h.k2 >= 0 &&
                  h.k1 + h.k2 <= max_stack && h.kcap >= 0 && h.Cout && h.Dout && h.rank_out &&
                  (h.k1 == 0 || (h.A && h.B && h.lda >= h.m && h.ldb >= h.n)) &&
                  (h.k2 == 0 || (h.C && h.D && h.ldc >= h.m && h.ldd >= h.n));
  DTruncPart u{};
  u.A = h.A;
  u.B = h.B;
  u.alpha = h.alpha;
  u.lda = h.lda;
  u.ldb = h.ldb;
  u.rows = h.m;
  u.cols = h.n;
  u.k = {ok ? h.k1 : 0, 0, nullptr};
  DTruncPart z{};
  z.A = h.C;
  z.B = h.D;
  z.alpha = 1.0;
  z.lda = h.ldc;
  z.ldb = h.ldd;
  z.rows = h.m;
  z.cols = h.n;
  z.k = {ok ? h.k2 : 0, 0, nullptr};
  dp[2 * (size_t)i] = u;
  dp[2 * (size_t)i + 1] = z;
  DTrunc d{};
  d.C = h.Cout;
  d.D = h.Dout;
  d.rank = h.rank_out;
  d.m = ok ? h.m : 1;
  d.n = ok ? h.n : 1;
  d.ldc = d.m;
  d.ldd = d.n;
  d.cap = h.kcap;
  d.part0 = 2 * i;
  d.nparts = 2;
  d.lmax = ok ? h.k1 + h.k2 : 0;
  d.flags = TRUNC_SKIP_IF_PART0_EMPTY | TRUNC_CLASS_CHECK;
  d.log_idx = i;
  d.level = 0;
  d.kfix = -1;
  dt[i] = d;
  if (!ok) atomicOr(status, ST_BAD_DESC);
}

hipError_t launch_lower_trunc_descs(const hm_trunc_desc* in, int count, int max_rows, int max_stack, DTrunc* dt,
                                    DTruncPart* dp, int* status, hipStream_t stream) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(lower_trunc_descs_kernel, dim3((count + 255) / 256), dim3(256), 0, stream, in, count, max_rows,
                     max_stack, dt, dp, status);
  return hipGetLastError();
}

}  // namespace hm
