// Compile-time layout of the degree-blocked M2L contraction (shared by the host table packer and
// the MFMA kernels, so that both walk the blocks in the same order).
//
// Multi-indices n with |n| <= p are ordered by degree.  The M2L of Sec. II.B,
//   F_n = sum_{|m| <= p - |n|} M_m D_{n+m},
// is a matrix product F = K M with K[n][m] = D_{n+m} where |n| + |m| <= p and 0 elsewhere.  K is
// a Hankel-type matrix: its entries are the C(p + 3, 3) values D_k, |k| <= p, so the kernels keep
// only that vector per offset and address it through a fixed table of indices k = n + m.
// Rows are cut into blocks of 16 (the MFMA tile height).  The reduction runs in steps of 4
// coefficients, one per lane quarter q = 0..3; step s reads coefficient
//   m(s, q) = 8 (s / 2) + 2 q + (s % 2),
// so that each lane's two consecutive steps are two adjacent coefficients (one 16-byte load) and
// the four quarters of a 16-target tile cover 8 adjacent coefficients of each source row.
// Row block rb starts at degree dmin(rb), so only its first count(p - dmin(rb)) coefficients can be
// non-zero: the blocks of the truncation staircase that are all zero are skipped.  Blocks are
// visited step-major: for each step s, every row block that still has coefficients at s.
#pragma once

namespace pfmm {

// number of multi-indices of degree <= d in 3D: C(d + 3, 3)
__host__ __device__ constexpr int mi_count(int d) { return d < 0 ? 0 : (d + 1) * (d + 2) * (d + 3) / 6; }
__host__ __device__ constexpr int sched_nc(int p) { return mi_count(p); }
__host__ __device__ constexpr int sched_stride(int p) { return (mi_count(p) + 7) / 8 * 8; }
// length of a stored derivative vector D_k(d): the C(p + 3, 3) values, then at least one zero (the
// entry that the index table names for the zero entries of K), rounded up to an even count
__host__ __device__ constexpr int sched_dpitch(int p) { return (mi_count(p) + 2) / 2 * 2; }
// coefficient read by lane quarter q at step s
__host__ __device__ constexpr int sched_coef(int s, int q) { return 8 * (s / 2) + 2 * q + (s % 2); }
__host__ __device__ constexpr int sched_nrb(int p) { return (mi_count(p) + 15) / 16; }
__host__ __device__ constexpr int sched_deg_of(int row) {
  int d = 0;
  while (mi_count(d) <= row) ++d;
  return d;
}
// steps s whose quarter-0 coefficient is still inside row block rb's non-zero columns
__host__ __device__ constexpr int sched_nsteps(int p, int rb) {
  int s = 0;
  while (sched_coef(s, 0) < mi_count(p - sched_deg_of(16 * rb))) ++s;
  return s;
}
__host__ __device__ constexpr int sched_maxsteps(int p) { return sched_nsteps(p, 0); }
__host__ __device__ constexpr int sched_nblocks(int p) {
  int t = 0;
  for (int rb = 0; rb < sched_nrb(p); ++rb) t += sched_nsteps(p, rb);
  return t;
}
// The K-entry index table holds one 16-bit index per block and lane, the 64 lanes of a block
// adjacent (one conflict-free 128-byte LDS read per block): position of (block, lane).
__host__ __device__ constexpr int sched_hpos(int blk, int lane) { return blk * 64 + lane; }

}  // namespace pfmm
