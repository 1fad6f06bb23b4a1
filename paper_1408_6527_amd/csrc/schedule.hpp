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
// position of n = (nx, ny, nz) in the degree-major order (descending nx, then descending ny)
__host__ __device__ constexpr int mi_index(int nx, int ny, int nz) {
  return mi_count(nx + ny + nz - 1) + (ny + nz) * (ny + nz + 1) / 2 + nz;
}
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
// steps s whose quarter-0 coefficient m(s, 0) is below count: ceil(count / 8) even steps
// (m = 8j) and ceil((count - 1) / 8) odd ones (m = 8j + 1)
__host__ __device__ constexpr int sched_steps_below(int count) { return count <= 0 ? 0 : (count + 7) / 8 + (count + 6) / 8; }
// steps s whose quarter-0 coefficient is still inside row block rb's non-zero columns
__host__ __device__ constexpr int sched_nsteps(int p, int rb) { return sched_steps_below(mi_count(p - sched_deg_of(16 * rb))); }
__host__ __device__ constexpr int sched_maxsteps(int p) { return sched_nsteps(p, 0); }
__host__ __device__ constexpr int sched_nblocks(int p) {
  int t = 0;
  for (int rb = 0; rb < sched_nrb(p); ++rb) t += sched_nsteps(p, rb);
  return t;
}
// Steps of row block rb that a truncation at order q <= p keeps (quarter-0 coefficient below
// count(q - lowest row degree)).
__host__ __device__ constexpr int sched_nsteps_q(int p, int q, int rb) {
  const int d0 = sched_deg_of(16 * rb);
  return d0 > q || q > p ? 0 : sched_steps_below(mi_count(q - d0));
}
// Two waves share the rows of one target: row block 0 is split by step pairs (half (s / 2) % 2),
// every other row block belongs to one half, assigned in index order to the half that keeps the
// larger of the two block counts smallest, summed over the truncation orders ceil(p/2) .. p.
// half[rb] (rb >= 1) is the half of row block rb, loc[rb] its accumulator slot within the half
// (row block 0 is slot 0 of both halves), nloc the slots of the larger half.
struct SchedHalves {
  int half[32];
  int loc[32];
  int nloc;
};
__host__ __device__ constexpr SchedHalves sched_halves(int p) {
  SchedHalves hs{};
  const int lo = (p + 1) / 2, nrb = sched_nrb(p);
  int ns[16][32] = {};  // steps kept per order q = lo .. p and row block
  for (int q = lo; q <= p; ++q)
    for (int rb = 0; rb < nrb; ++rb) ns[q - lo][rb] = sched_nsteps_q(p, q, rb);
  int load[2][16] = {};
  for (int q = lo; q <= p; ++q) {
    const int n0 = ns[q - lo][0];
    load[0][q - lo] = (n0 + 3) / 4 * 2 - (n0 % 4 == 1 ? 1 : 0);  // steps s < n0 with (s / 2) % 2 == 0
    load[1][q - lo] = n0 - load[0][q - lo];
  }
  int cnt[2] = {1, 1};
  hs.half[0] = 0;
  hs.loc[0] = 0;
  for (int r = 1; r < nrb; ++r) {
    int best = 0, best_cost = -1;
    for (int h = 0; h < 2; ++h) {
      int cost = 0;
      for (int q = lo; q <= p; ++q) {
        const int a = load[0][q - lo] + (h == 0 ? ns[q - lo][r] : 0);
        const int b = load[1][q - lo] + (h == 1 ? ns[q - lo][r] : 0);
        cost += a > b ? a : b;
      }
      if (best_cost < 0 || cost < best_cost) {
        best = h;
        best_cost = cost;
      }
    }
    for (int q = lo; q <= p; ++q) load[best][q - lo] += ns[q - lo][r];
    hs.half[r] = best;
    hs.loc[r] = cnt[best]++;
  }
  hs.nloc = cnt[0] > cnt[1] ? cnt[0] : cnt[1];
  return hs;
}
// evaluated once per order p
template <int P>
struct SchedHalvesOf {
  static constexpr SchedHalves value = sched_halves(P);
};
template <int P>
constexpr SchedHalves SchedHalvesOf<P>::value;

// The K-entry index table holds one 16-bit index per block and lane, the 64 lanes of a block
// adjacent (one conflict-free 128-byte LDS read per block): position of (block, lane).
__host__ __device__ constexpr int sched_hpos(int blk, int lane) { return blk * 64 + lane; }

}  // namespace pfmm
