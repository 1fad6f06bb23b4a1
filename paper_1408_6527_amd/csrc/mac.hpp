// The acceptance test of the dual tree walk (the multipole acceptance criterion of Sec. III, eq. mac,
// or the well-separation rule) as one device function, shared by the walk that builds the lists
// (mac.hip) and the M2L kernel that applies it to the children of the split cell pairs (m2l.hip):
// both take every decision with the same float64 operations, each rounded on its own (no fused
// multiply-adds), so they decide alike.
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

// A cell is terminal when the walk may sum it directly: at level L, or, on the adaptive octree, when
// it is not split.
__device__ inline bool mac_terminal(const TreeView& t, const MacView& mv, int c) {
  return mv.nonleaf ? mv.nonleaf[c] == 0 : c >= t.off[t.L];
}

// Target B and source A of one level, coordinate offset d = B - A, cell edge w: accepted for M2L when
// they are two cells at Chebyshev distance >= minsep that hold at least ndirect particles together,
// are not two terminal cells under the leaf-direct rule, and, with the criterion, theta |d| w > r_B + r_A.
__device__ inline bool mac_accept(const TreeView& t, const MacView& mv, double w, int B, int A, int dx, int dy,
                                  int dz) {
  if (A == B || max(abs(dx), max(abs(dy), abs(dz))) < mv.minsep) return false;
  if (t.count[B] + t.count[A] < mv.ndirect) return false;
  if (mv.leaf_direct && mac_terminal(t, mv, B) && mac_terminal(t, mv, A)) return false;
  if (!mv.use_theta) return true;
  const double dist = mac_length3(__dmul_rn((double)dx, w), __dmul_rn((double)dy, w), __dmul_rn((double)dz, w));
  return __dmul_rn(mv.theta, dist) > __dadd_rn(mv.renc[B], mv.renc[A]);
}

}  // namespace pfmm
