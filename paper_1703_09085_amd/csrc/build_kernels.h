// Launchers of the builder kernels (build_kernels.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/hm.h"
#include "hm_types.h"

namespace hm {

// One 64 x 64 tile of a block of the kernel matrix: rows [r0, r0 + 64) and
// columns [c0, c0 + 64) (clipped to m x n) of the block whose first row and
// column are points ro and co in cluster order, written to out (leading
// dimension ld, column-major).
struct KEvalTile {
  double* out;
  int ld;
  int ro, co;
  int m, n;
  int r0, c0;
  int pad;
};

// xs: point coordinates in cluster order, dim arrays of n doubles.
hipError_t launch_kmat_eval(const KEvalTile* tiles, int64_t ntiles, const double* xs, int64_t n, int dim, double diag,
                            hipStream_t stream);

// Galerkin boundary-element entries on flat triangles (piecewise constants):
// layer 0 the single layer 1/(4 pi |x - y|), layer 1 half the mass matrix
// plus the double layer <y - x, n_y> / (4 pi |x - y|^3).  tri: per triangle
// in cluster order, BEM_TRI_DOUBLES doubles made by bem_triangle_table.
constexpr int BEM_TRI_DOUBLES = 40;
void bem_triangle_table(const double* tri9, const int32_t* perm, int64_t n, double* out);
hipError_t launch_bem_eval(const KEvalTile* tiles, int64_t ntiles, const double* tri, int layer, hipStream_t stream);

// Device descriptors of hm_trunc_batch_device to truncation items (dt[count],
// dp[2 count]); invalid items become no-ops and set ST_BAD_DESC in *status.
hipError_t launch_lower_trunc_descs(const hm_trunc_desc* in, int count, int max_rows, int max_stack, DTrunc* dt,
                                    DTruncPart* dp, int* status, hipStream_t stream);

}  // namespace hm
