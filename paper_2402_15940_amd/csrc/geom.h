// Device helpers for the trilinear geometry of a structured hexahedral mesh.
#pragma once

#include "internal.h"

namespace pafem {

// Position X and Jacobian J[r][m] = d x_r / d xi_m of the trilinear map of the
// element with corners v[i + 2 j + 4 k] at reference point (s, tt, u).
static __device__ __forceinline__ void trilinear_at(const double (&v)[8][3], double s, double tt,
                                             double u, double X[3], double J[3][3]) {
  const double fs[2] = {1.0 - s, s}, ft[2] = {1.0 - tt, tt}, fu[2] = {1.0 - u, u};
  const double ds[2] = {-1.0, 1.0};
  for (int i = 0; i < 3; ++i) {
    X[i] = 0.0;
    J[i][0] = J[i][1] = J[i][2] = 0.0;
  }
#pragma unroll
  for (int k = 0; k < 2; ++k)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int c = i + 2 * j + 4 * k;
        const double n0 = fs[i] * ft[j] * fu[k];
        const double d0 = ds[i] * ft[j] * fu[k];
        const double d1 = fs[i] * ds[j] * fu[k];
        const double d2 = fs[i] * ft[j] * ds[k];
#pragma unroll
        for (int r = 0; r < 3; ++r) {
          X[r] += n0 * v[c][r];
          J[r][0] += d0 * v[c][r];
          J[r][1] += d1 * v[c][r];
          J[r][2] += d2 * v[c][r];
        }
      }
}

static __device__ __forceinline__ void load_corners(const GeomArgs& g, int64_t e, double (&v)[8][3]) {
  const int ex = (int)(e % g.nx);
  const int ey = (int)((e / g.nx) % g.ny);
  const int ez = (int)(e / ((int64_t)g.nx * g.ny));
  const int64_t sx = 1, sy = g.nx + 1, sz = (int64_t)(g.nx + 1) * (g.ny + 1);
#pragma unroll
  for (int k = 0; k < 2; ++k)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int64_t vi = (ex + i) * sx + (ey + j) * sy + (ez + k) * sz;
#pragma unroll
        for (int r = 0; r < 3; ++r) v[i + 2 * j + 4 * k][r] = g.verts[vi * 3 + r];
      }
}

static __device__ __forceinline__ double det3(const double J[3][3]) {
  return J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
         J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
         J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
}

}  // namespace pafem
