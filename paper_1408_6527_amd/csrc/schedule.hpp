// Compile-time layout of the degree-blocked M2L contraction (shared by the host table packer and
// the MFMA kernels, so that both walk the blocks in the same order).
//
// Multi-indices n with |n| <= p are ordered by degree.  The M2L of Sec. II.B,
//   F_n = sum_{|m| <= p - |n|} M_m D_{n+m},
// is a matrix product F = K M with K[n][m] = D_{n+m} where |n| + |m| <= p and 0 elsewhere.
// Rows are cut into blocks of 16 (the MFMA tile height) and columns into steps of 4 (the MFMA
// reduction depth).  Row block rb starts at degree dmin(rb), so only its first
// count(p - dmin(rb)) columns can be non-zero: the staircase of the truncation is skipped at
// 16 x 4 granularity.  Blocks are visited step-major: for each step s, every row block that
// still has columns at s.
#pragma once

namespace pfmm {

// number of multi-indices of degree <= d in 3D: C(d + 3, 3)
__host__ __device__ constexpr int mi_count(int d) { return d < 0 ? 0 : (d + 1) * (d + 2) * (d + 3) / 6; }
__host__ __device__ constexpr int sched_nc(int p) { return mi_count(p); }
__host__ __device__ constexpr int sched_stride(int p) { return (mi_count(p) + 3) / 4 * 4; }
__host__ __device__ constexpr int sched_nrb(int p) { return (mi_count(p) + 15) / 16; }
__host__ __device__ constexpr int sched_deg_of(int row) {
  int d = 0;
  while (mi_count(d) <= row) ++d;
  return d;
}
__host__ __device__ constexpr int sched_nsteps(int p, int rb) {
  return (mi_count(p - sched_deg_of(16 * rb)) + 3) / 4;
}
__host__ __device__ constexpr int sched_maxsteps(int p) { return sched_nsteps(p, 0); }
__host__ __device__ constexpr int sched_nblocks(int p) {
  int t = 0;
  for (int rb = 0; rb < sched_nrb(p); ++rb) t += sched_nsteps(p, rb);
  return t;
}

}  // namespace pfmm
