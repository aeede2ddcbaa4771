// Real spherical harmonics of even degree l <= 4, for the multipoles of the
// pair-galaxy correlation in the angle between the pair axis and the
// pair-to-galaxy direction.  The Legendre polynomial of that angle factorises
// by the addition theorem, P_l(a . b) = 4 pi / (2l + 1) sum_m Y_lm(a) Y_lm(b),
// so the pair fields carry Y_lm(pair axis) and the bin kernels Y_lm(r^).
//
// Harmonic index h runs over the even degrees in order: h = 0 is (0, 0);
// h = 1..5 are (2, m = -2..2); h = 6..14 are (4, m = -4..4).  The Cartesian
// polynomial forms are used, with r^2 kept in the terms where a unit vector
// would give 1, so a zero vector yields 0 for l > 0.
#pragma once

namespace pgx {

constexpr int kMaxHarm = 15;  // harmonics of the even degrees up to 4

__host__ __device__ constexpr int harm_count(int lmax) {
  return lmax >= 4 ? 15 : (lmax >= 2 ? 6 : 1);
}
// degree of harmonic h
__host__ __device__ constexpr int harm_degree(int h) { return h == 0 ? 0 : (h < 6 ? 2 : 4); }

// Y_h(x, y, z) for a unit vector (or the zero vector).
__host__ __device__ inline double real_ylm(int h, double x, double y, double z) {
  constexpr double PI = 3.14159265358979323846;
  const double x2 = x * x, y2 = y * y, z2 = z * z, r2 = x2 + y2 + z2;
  switch (h) {
    case 0: return 0.5 * sqrt(1.0 / PI);
    // l = 2
    case 1: return 0.5 * sqrt(15.0 / PI) * x * y;
    case 2: return 0.5 * sqrt(15.0 / PI) * y * z;
    case 3: return 0.25 * sqrt(5.0 / PI) * (2.0 * z2 - x2 - y2);
    case 4: return 0.5 * sqrt(15.0 / PI) * x * z;
    case 5: return 0.25 * sqrt(15.0 / PI) * (x2 - y2);
    // l = 4
    case 6: return 0.75 * sqrt(35.0 / PI) * x * y * (x2 - y2);
    case 7: return 0.75 * sqrt(35.0 / (2.0 * PI)) * (3.0 * x2 - y2) * y * z;
    case 8: return 0.75 * sqrt(5.0 / PI) * x * y * (7.0 * z2 - r2);
    case 9: return 0.75 * sqrt(5.0 / (2.0 * PI)) * y * z * (7.0 * z2 - 3.0 * r2);
    case 10: return 3.0 / 16.0 * sqrt(1.0 / PI) * (35.0 * z2 * z2 - 30.0 * z2 * r2 + 3.0 * r2 * r2);
    case 11: return 0.75 * sqrt(5.0 / (2.0 * PI)) * x * z * (7.0 * z2 - 3.0 * r2);
    case 12: return 3.0 / 8.0 * sqrt(5.0 / PI) * (x2 - y2) * (7.0 * z2 - r2);
    case 13: return 0.75 * sqrt(35.0 / (2.0 * PI)) * (x2 - 3.0 * y2) * x * z;
    case 14: return 3.0 / 16.0 * sqrt(35.0 / PI) * (x2 * (x2 - 3.0 * y2) - y2 * (3.0 * x2 - y2));
    default: return 0.0;
  }
}

// Y_h of the direction of (a, b, c) (zero for the zero vector when l > 0).
__host__ __device__ inline double real_ylm_dir(int h, double a, double b, double c) {
  const double n = sqrt(a * a + b * b + c * c);
  if (n == 0.0) return h == 0 ? real_ylm(0, 0.0, 0.0, 0.0) : 0.0;
  return real_ylm(h, a / n, b / n, c / n);
}

}  // namespace pgx
