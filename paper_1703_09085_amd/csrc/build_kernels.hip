// Device kernels of the H-matrix builders: entries of the kernel matrix
// 1/|x - y| (the sphere workload standing in for the boundary-element
// matrices of Sect. 7), and the lowering of truncation descriptors that a
// caller made on the device.
#include <hip/hip_runtime.h>

#include <cmath>

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

// ---- boundary-element entries ------------------------------------------------
// Per triangle (cluster order): the 7 points of the degree-5 rule (Radon) as
// x, y, z (21 doubles), their weights times the area (7), the unit normal
// (3), the vertices (9).
void bem_triangle_table(const double* tri9, const int32_t* perm, int64_t n, double* out) {
  const double r15 = std::sqrt(15.0);
  const double b1 = (6.0 + r15) / 21.0, a1 = 1.0 - 2.0 * b1;
  const double b2 = (6.0 - r15) / 21.0, a2 = 1.0 - 2.0 * b2;
  const double w1 = (155.0 + r15) / 1200.0, w2 = (155.0 - r15) / 1200.0;
  const double lam[7][3] = {{1.0 / 3, 1.0 / 3, 1.0 / 3}, {a1, b1, b1}, {b1, a1, b1}, {b1, b1, a1},
                            {a2, b2, b2}, {b2, a2, b2}, {b2, b2, a2}};
  const double wq[7] = {0.225, w1, w1, w1, w2, w2, w2};
  for (int64_t p = 0; p < n; ++p) {
    const double* v = tri9 + (size_t)perm[p] * 9;
    double* o = out + (size_t)p * BEM_TRI_DOUBLES;
    const double e1[3] = {v[3] - v[0], v[4] - v[1], v[5] - v[2]};
    const double e2[3] = {v[6] - v[0], v[7] - v[1], v[8] - v[2]};
    const double c[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
    const double len = std::sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
    const double area = 0.5 * len;
    for (int q = 0; q < 7; ++q) {
      for (int d = 0; d < 3; ++d) o[3 * q + d] = lam[q][0] * v[d] + lam[q][1] * v[3 + d] + lam[q][2] * v[6 + d];
      o[21 + q] = wq[q] * area;
    }
    for (int d = 0; d < 3; ++d) o[28 + d] = c[d] / len;
    for (int d = 0; d < 9; ++d) o[31 + d] = v[d];
  }
}

// int over the triangle t (vertices t[31..39], normal t[28..30]) of
// 1/|x - y| dy, x in its plane: the sum over the counterclockwise edges a -> b
// of h log((r_b + s_b) / (r_a + s_a)), h the distance of x from the edge's
// line (positive inside), s the coordinate along the edge from the foot of x,
// r the distance from x.
__device__ double tri_inv_dist(const double* t, const double* x) {
  const double* nr = t + 28;
  double sum = 0.0;
  for (int e = 0; e < 3; ++e) {
    const double* a = t + 31 + 3 * e;
    const double* b = t + 31 + 3 * ((e + 1) % 3);
    double u[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
    const double len = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    for (int d = 0; d < 3; ++d) u[d] /= len;
    const double out[3] = {u[1] * nr[2] - u[2] * nr[1], u[2] * nr[0] - u[0] * nr[2], u[0] * nr[1] - u[1] * nr[0]};
    const double xa[3] = {a[0] - x[0], a[1] - x[1], a[2] - x[2]};
    const double xb[3] = {b[0] - x[0], b[1] - x[1], b[2] - x[2]};
    const double h = xa[0] * out[0] + xa[1] * out[1] + xa[2] * out[2];
    const double sa = xa[0] * u[0] + xa[1] * u[1] + xa[2] * u[2];
    const double sb = xb[0] * u[0] + xb[1] * u[1] + xb[2] * u[2];
    const double ra = sqrt(xa[0] * xa[0] + xa[1] * xa[1] + xa[2] * xa[2]);
    const double rb = sqrt(xb[0] * xb[0] + xb[1] * xb[1] + xb[2] * xb[2]);
    if (h != 0.0) sum += h * log((rb + sb) / (ra + sa));
  }
  return sum;
}

// One 64 x 64 tile per workgroup as kmat_eval_kernel; lane r of each wave
// holds the 7 points and weights of row triangle ro + r in registers.
__global__ __launch_bounds__(256) void bem_eval_kernel(const KEvalTile* __restrict__ tiles,
                                                       const double* __restrict__ tri, int layer) {
  const KEvalTile T = tiles[blockIdx.x];
  const int r = T.r0 + (threadIdx.x & 63);
  if (r >= T.m) return;
  const long long gi = (long long)T.ro + r;
  const double* ti = tri + gi * BEM_TRI_DOUBLES;
  double px[7], py[7], pz[7], wi[7];
  for (int q = 0; q < 7; ++q) {
    px[q] = ti[3 * q];
    py[q] = ti[3 * q + 1];
    pz[q] = ti[3 * q + 2];
    wi[q] = ti[21 + q];
  }
  const double inv4pi = 0.25 / 3.14159265358979323846;
  const int cend = T.c0 + 64 < T.n ? T.c0 + 64 : T.n;
  for (int c = T.c0 + (threadIdx.x >> 6); c < cend; c += 4) {
    const long long gj = (long long)T.co + c;
    const double* tj = tri + gj * BEM_TRI_DOUBLES;
    double v = 0.0;
    if (gi == gj) {
      if (layer == 0) {
        for (int a = 0; a < 7; ++a) {
          const double x[3] = {px[a], py[a], pz[a]};
          v += wi[a] * tri_inv_dist(tj, x);
        }
        v *= inv4pi;
      } else {
        double area = 0.0;
        for (int q = 0; q < 7; ++q) area += wi[q];  // the weights sum to the area
        v = 0.5 * area;
      }
    } else {
      const double nx = tj[28], ny = tj[29], nz = tj[30];
      for (int b = 0; b < 7; ++b) {
        const double yx = tj[3 * b], yy = tj[3 * b + 1], yz = tj[3 * b + 2], wb = tj[21 + b];
        double s = 0.0;
        for (int a = 0; a < 7; ++a) {
          const double dx = yx - px[a], dy = yy - py[a], dz = yz - pz[a];
          const double d2 = dx * dx + dy * dy + dz * dz;
          const double id = 1.0 / sqrt(d2);
          s += wi[a] * (layer == 0 ? id : (dx * nx + dy * ny + dz * nz) * id * id * id);
        }
        v += wb * s;
      }
      v *= inv4pi;
    }
    T.out[r + (size_t)c * T.ld] = v;
  }
}

hipError_t launch_bem_eval(const KEvalTile* tiles, int64_t ntiles, const double* tri, int layer, hipStream_t stream) {
  for (int64_t t0 = 0; t0 < ntiles; t0 += (1 << 30)) {
    const int64_t cnt = ntiles - t0 < (1 << 30) ? ntiles - t0 : (1 << 30);
    hipLaunchKernelGGL(bem_eval_kernel, dim3((unsigned)cnt), dim3(256), 0, stream, tiles + t0, tri, layer);
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
