// The acceptance test of the multipole acceptance criterion (Sec. III, eq. mac) as one device
// function, shared by the walk that builds the lists (mac.hip) and the M2L kernel that applies it to
// the children of the split cell pairs (m2l.hip): both take every decision with the same float64
// operations, each rounded on its own (no fused multiply-adds), so they decide alike.
#pragma once

#include "kernels.hpp"
#include "morton.hpp"

namespace pfmm {

__device__ inline void mac_coords(uint64_t key, int c[3]) {
  c[0] = compact3(key >> 2);
  c[1] = compact3(key >> 1);
  c[2] = compact3(key);
}

// sqrt((x x + y y) + z z), correctly rounded square root
__device__ inline double mac_length3(double x, double y, double z) {
  return __dsqrt_rn(__dadd_rn(__dadd_rn(__dmul_rn(x, x), __dmul_rn(y, y)), __dmul_rn(z, z)));
}

// Target B and source A of one level, coordinate offset d = B - A, cell edge w: accepted for M2L when
// they are two cells, not adjacent (Chebyshev distance >= 2), hold at least ndirect particles
// together, and theta |d| w > r_B + r_A.  Leaf pairs under the leaf-direct rule are the caller's test.
__device__ inline bool mac_accept(const TreeView& t, const double* renc, double theta, int ndirect, double w, int B,
                                  int A, int dx, int dy, int dz) {
  if (A == B || max(abs(dx), max(abs(dy), abs(dz))) < 2) return false;
  if (t.count[B] + t.count[A] < ndirect) return false;
  const double dist = mac_length3(__dmul_rn((double)dx, w), __dmul_rn((double)dy, w), __dmul_rn((double)dz, w));
  return __dmul_rn(theta, dist) > __dadd_rn(renc[B], renc[A]);
}

}  // namespace pfmm
