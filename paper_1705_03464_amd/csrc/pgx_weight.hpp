// The paper's Gaussian-sigmoid weighting function, shared by the host bin
// tables and the device bin kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>

namespace pgx {

// Gaussian-sigmoid weighting function of the paper (Section "weighting",
// equation weighting) at a lattice offset with xy = i'^2 + j'^2 (across the
// line of sight) and kk = k'^2 (along it), up to its normalisation constant:
// sigmoid(s0 (r_perp - r_s)) exp(-(r_perp^2 + r_par^2) / (2 sigma^2)).
// g = {cell size, s0, r_s, 1 / (2 sigma^2)}; the cuts are applied by the
// classification.
__host__ __device__ inline double gsw_value(int xy, int kk, const double* g) {
  const double d2 = g[0] * g[0];
  const double rperp = g[0] * sqrt((double)xy);
  return 1.0 / (1.0 + exp(-g[1] * (rperp - g[2]))) * exp(-((double)xy + (double)kk) * d2 * g[3]);
}

}  // namespace pgx
