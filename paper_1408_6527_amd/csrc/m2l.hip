// M2L on the matrix cores (Sec. II.B, local expansion from a multipole expansion):
//   F~_n(B) = sum_{|m| <= p - |n|} D_{n+m}(d) M~_m(A),   d = B - A in cells of the level.
//
// In level-scaled form the operator depends only on the integer offset d, and its matrix
// K_d[n][m] = D_{n+m}(d) is fixed by the vector of C(p + 3, 3) derivatives D_k(d), |k| <= p.
//
// Work unit: a tile of 16 parents on one level (the 16 columns of the MFMA tiles) and their
// children, in 8 waves: each wave computes the targets of one pair of child octants for one half of
// the row blocks of F~ (schedule.hpp, sched_halves).  A target B = 2 P + oB meets its sources
// A = 2 (P + e) + c, the children of P's colleagues P + e, at d = oB - c - 2 e whenever the
// Chebyshev norm of d exceeds ws.  For one colleague offset e and one source octant c (a slot), the
// 16 source expansions are the same rows for all eight target octants, so the workgroup stages them
// in LDS once (coalesced row loads) and every wave multiplies them by the K_d of its octants:
//   for e in the split's share of colleague offsets:
//     stage D(d) for the 27 offsets d = u - 2 e, u = oB - c in [-1, 1]^3
//     for c in octants: stage the 16 source rows; each wave runs, for each octant of its pair
//       with |d| > ws, its half of the degree-blocked MFMA schedule: A = K_d entries gathered from
//       the LDS copy of D(d) through the index table, B = source coefficients from LDS.
// With a per-offset truncation order q(d) <= p (m2l_order_slack >= 0, or a cap set by a relaxed
// dipole solve) a wave runs the unrolled schedule of that q: the blocks of the order-p schedule
// that hold entries of degree <= q, reading a copy of D(d) whose entries above degree q are zero.
// Accumulators stay in registers for the whole loop and each target's (partial) F~ is written once
// (the two halves' shares of row block 0 are added through LDS first): no atomics, deterministic.
//
// FP64 path: v_mfma_f64_16x16x4f64.  Mixed path: v_mfma_f32_16x16x4f32 with float32 operands and
// float32 accumulation, except for targets at levels <= fp64_max_level (both list kinds).
#include <algorithm>
#include <type_traits>
#include <utility>

#include "kernels.hpp"
#include "mac.hpp"
#include "schedule.hpp"

namespace pfmm {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int TPB = 512;  // 8 waves: 4 octant pairs x 2 row halves
constexpr int M2L_XCD_TILES = 2;  // tiles per XCD chunk (k_m2l)
constexpr int NU = 27;    // u = oB - c in [-1, 1]^3

// The blocks of the order-P schedule (schedule.hpp) that a truncation at order Q <= P needs (rows
// of degree <= Q, steps below count(Q - lowest row degree)) and that half H of the row split issues,
// in schedule order, as compile-time tables: step s, row block rb, and position bp in the full
// order-P block order (which locates their K-entry indices).
template <int P, int Q, int H>
struct BlockOrder {
  int n;
  int s[sched_nblocks(P)];
  int rb[sched_nblocks(P)];
  int bp[sched_nblocks(P)];
  int loc[sched_nblocks(P)];  // accumulator slot of the row block (sched_halves)
  constexpr BlockOrder() : n(0), s(), rb(), bp(), loc() {
    const SchedHalves& hs = SchedHalvesOf<P>::value;
    int b = 0;
    for (int st = 0; st < sched_maxsteps(P); ++st)
      for (int r = 0; r < sched_nrb(P); ++r)
        if (sched_nsteps(P, r) > st) {
          const int d0 = sched_deg_of(16 * r);
          const int owner = r == 0 ? (st / 2) % 2 : hs.half[r];
          if (d0 <= Q && sched_coef(st, 0) < mi_count(Q - d0) && owner == H) {
            s[n] = st;
            rb[n] = r;
            bp[n] = b;
            loc[n] = hs.loc[r];
            ++n;
          }
          ++b;
        }
  }
  // most step pairs (s / 2) met by w consecutive blocks (steps never decrease along the order)
  constexpr int pair_span(int w) const {
    int m = 1;
    for (int k = 0; k < n; ++k) {
      const int last = k + w - 1 < n ? k + w - 1 : n - 1;
      const int span = s[last] / 2 - s[k] / 2 + 1;
      m = span > m ? span : m;
    }
    return m;
  }
};

// Software pipeline of one slot, in blocks of the schedule: while block k is issued to the matrix
// core, the K-entry index of block k + DI is read from LDS and the K entry of block k + DG is
// gathered (with the source coefficients of its step pair), so that no MFMA waits on the
// two dependent LDS reads that feed it.
// 16-parent tiles per workgroup: every K_d entry gathered from LDS feeds NCB MFMAs.  Bounded by
// the accumulator registers (NCB x NRB tiles of 16 x 16) and the LDS of the staged sources.
template <int P, bool F32>
constexpr int m2l_ncb() { return (F32 ? P <= 10 : P <= 7) ? 2 : 1; }

// (a shorter distance where the float64 accumulators leave fewer registers)
template <int P, bool F32>
constexpr int m2l_dg() { return F32 ? (P >= 9 ? 3 : 6) : (P == 9 ? 2 : (P >= 10 || m2l_ncb<P, F32>() > 1 ? 3 : 4)); }

// One slot of one wave at truncation order Q: A = K_d entries gathered from the staged D(d) at Dv
// through the index table sH, B = the staged source coefficients at Bp.  The staged D(d) holds zeros
// above degree Q, so the blocks of the order-Q subset read the truncated operator unmasked.
template <int P, bool F32, int NCB, int Q, int H, bool MASK, typename kt, typename kt2, typename acc_t>
__device__ __forceinline__ void m2l_mfma(const kt* Dv, const kt* Bp, const unsigned short* sH, int lane,
                                         acc_t (&acc)[NCB][SchedHalvesOf<P>::value.nloc], const bool (&bm)[NCB]) {
  constexpr BlockOrder<P, Q, H> order{};
  constexpr int NB = order.n;
  constexpr int BP = sched_stride(P) + 2;
  // (one block less of look-ahead with column masks, whose test needs registers of its own)
  constexpr int DG = MASK ? (m2l_dg<P, F32>() > 2 ? m2l_dg<P, F32>() - 1 : m2l_dg<P, F32>()) : m2l_dg<P, F32>();
  constexpr int DI = 2 * DG;
  constexpr int RA = DG + 1, RI = DI - DG + 1;  // live K entries and indices
  constexpr int RB = order.pair_span(DG + 1);   // live step pairs of source coefficients
  unsigned ix[RI];
  kt a[RA];
  kt2 bb[RB][NCB];
#pragma unroll
  for (int k = -DI; k < NB; ++k) {
    const int ki = k + DI, kg = k + DG;
    if (ki >= 0 && ki < NB) ix[ki % RI] = sH[sched_hpos(order.bp[ki], lane)];
    if (kg >= 0 && kg < NB) {
      a[kg % RA] = Dv[ix[kg % RI]];
      const int sg = order.s[kg];
      if (kg == 0 || order.s[kg - 1] / 2 != sg / 2) {
        // steps 2j and 2j + 1 read coefficients m(2j, q) and m(2j, q) + 1 of the lane's column
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
          kt2 v = *reinterpret_cast<const kt2*>(Bp + cb * 16 * BP + 8 * (sg / 2));
          if constexpr (MASK) {
            if (!bm[cb]) v = kt2{(kt)0, (kt)0};  // the lane's column holds a pair that is not accepted
          }
          bb[(sg / 2) % RB][cb] = v;
        }
      }
    }
    if (k >= 0) {
      const int s = order.s[k], lc = order.loc[k];
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) {
        const kt b = (s & 1) ? bb[(s / 2) % RB][cb].y : bb[(s / 2) % RB][cb].x;
        if constexpr (F32)
          acc[cb][lc] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[k % RA], b, acc[cb][lc], 0, 0, 0);
        else
          acc[cb][lc] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[k % RA], b, acc[cb][lc], 0, 0, 0);
      }
    }
    // keep each block's reads in its own issue window: the scheduler would otherwise sink the
    // gathers down to their MFMAs to shorten register live ranges, which serialises the slot
    __builtin_amdgcn_sched_barrier(0);
  }
}

// Run the slot of half H at a runtime order q <= P (one unrolled schedule per order).  MASK: the
// source coefficients of column cb are taken as 0 where bm[cb] is false.
template <int P, bool F32, int NCB, int H, bool MASK, typename kt, typename kt2, typename acc_t, int... Qs>
__device__ __forceinline__ void m2l_mfma_order(int q, std::integer_sequence<int, Qs...>, const kt* Dv,
                                               const kt* Bp, const unsigned short* sH, int lane,
                                               acc_t (&acc)[NCB][SchedHalvesOf<P>::value.nloc], const bool (&bm)[NCB]) {
  (void)((q == Qs ? (m2l_mfma<P, F32, NCB, Qs, H, MASK, kt, kt2, acc_t>(Dv, Bp, sH, lane, acc, bm), true) : false) ||
         ...);
}
template <int P, bool F32, int NCB, int H, bool MASK, typename kt, typename kt2, typename acc_t>
__device__ __forceinline__ void m2l_slot(int q, const kt* Dv, const kt* Bp, const unsigned short* sH, int lane,
                                         acc_t (&acc)[NCB][SchedHalvesOf<P>::value.nloc], const bool (&bm)[NCB]) {
  if (q >= P)
    m2l_mfma<P, F32, NCB, P, H, MASK, kt, kt2, acc_t>(Dv, Bp, sH, lane, acc, bm);
  else
    m2l_mfma_order<P, F32, NCB, H, MASK, kt, kt2, acc_t>(q, std::make_integer_sequence<int, P>{}, Dv, Bp, sH, lane,
                                                         acc, bm);
}

// registers per lane: 2 waves per SIMD, one workgroup per CU
template <int P, bool F32>
constexpr int m2l_waves_per_eu() { return 2; }

// MAC: the lists of the dual tree walk (the acceptance criterion, or the ws rule on the adaptive
// octree).  The split partners of each parent (mv.split, at offsets e in [-Rp, Rp]^3) take the place
// of its colleagues, the operator rows come from mv.dvec, and every (target, source) column of a slot
// is tested with the walk's acceptance rule (mac.hpp); the columns of pairs that are not accepted
// multiply zero source coefficients.  Every M2L at order P or the cap.
template <int P, bool F32, bool MAC>
__global__ __launch_bounds__(TPB) __attribute__((amdgpu_waves_per_eu(m2l_waves_per_eu<P, F32>()))) void k_m2l(TreeView t, OpTables op, MacView mv, int lp_lo, int lp_hi, int nsplit, int nwork,
                                             const double* __restrict__ M, const float* __restrict__ M32,
                                             double* __restrict__ F,
                                             int64_t split_stride, const int* done, const int* qcap) {
  if (done && *done) return;
  const int qc = qcap ? *qcap : P;  // order cap of a relaxed evaluation
  using kt = typename std::conditional<F32, float, double>::type;
  using kt2 = typename std::conditional<F32, float2, double2>::type;
  using acc_t = typename std::conditional<F32, f4, d4>::type;
  // (one column block with the criterion: its masks leave no registers for a second)
  constexpr int NCB = MAC ? 1 : m2l_ncb<P, F32>();
  constexpr int NRB = sched_nrb(P);
  constexpr int NC = mi_count(P);
  constexpr int STRIDE = sched_stride(P);
  constexpr int DP = sched_dpitch(P);
  // LDS row pitch of the staged sources: STRIDE + 2 puts the 16 rows of one column read on
  // distinct banks (STRIDE is a multiple of 8)
  constexpr int BP = STRIDE + 2;
  constexpr int HALF = STRIDE / 2;  // 16-byte pieces of one source row
  constexpr int NBLK = sched_nblocks(P);
  constexpr int ROWS = 16 * NCB;
  constexpr int PF = (ROWS * HALF + TPB - 1) / TPB;  // 16-byte source pieces per thread and slot
  constexpr int QUART = STRIDE / 4;                   // 16-byte pieces of a float32 source row
  constexpr int PF4 = (ROWS * QUART + TPB - 1) / TPB;
  __shared__ uint4 sHv[NBLK * 8];  // K-entry index table, 64 16-bit indices per block
  __shared__ kt sD[NU * DP];
  __shared__ int sQ[NU];  // truncation order of the 27 staged offsets
  // source rows of two slots: the rows of the next slot are stored while the current one is read
  __shared__ __attribute__((aligned(16))) kt sB[2][ROWS * BP];
  __shared__ int sSrc[8][ROWS];
  __shared__ unsigned char sMask[MAC ? 8 : 1][MAC ? ROWS : 1];  // MAC: accepted source octants per target
  constexpr int NXCH = 2 * 4 * NCB * 64;  // row-block-0 partial sums handed between the halves
  constexpr bool XCH_IN_SB = NXCH * sizeof(acc_t) <= 2 * ROWS * BP * sizeof(kt);
  __shared__ acc_t sX[XCH_IN_SB ? 1 : NXCH];

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // Each wave computes the targets of an octant pair for one half of the row blocks (sched_half).
  // The pairs (0,3) (5,6) | (1,2) (4,7) form the octant sets {0,3,5,6} and {1,2,4,7}, whose
  // per-offset orders at any slot nearly balance; waves w and w + 4 share a SIMD, and the SIMD
  // takes half 0 of one pair and half 1 of the other pair of the same set, so that each SIMD
  // carries half of one set's work.
  const int simd = wave & 3, half = wave >> 2;
  const int pair = half == 0 ? simd : (simd ^ 1);
  constexpr int PAIRS[4][2] = {{0, 3}, {5, 6}, {1, 2}, {4, 7}};
  const int oc[2] = {PAIRS[pair][0], PAIRS[pair][1]};
  // XCD-aware order: the dispatcher hands workgroup b to XCD b % 8, so chunks of M2L_XCD_TILES
  // consecutive tiles (Morton-adjacent parents, which share most of their source rows) go to one XCD
  // in turn and meet in its L2; the chunks still run in tile order across the chip
  const int chunk = M2L_XCD_TILES * nsplit;
  const int wg = (((int)(blockIdx.x >> 3) / chunk) * 8 + (int)(blockIdx.x & 7)) * chunk + (int)(blockIdx.x >> 3) % chunk;
  if (wg >= nwork) return;  // padding of the last chunks: whole workgroup, before any barrier
  const int split = wg % nsplit;
  // finest level first: the coarse levels' tiles, fewer and lighter (their colleagues often fall
  // outside the occupied region), fill the end of the launch
  int tile = wg / nsplit, lp = lp_hi;
  for (; lp >= lp_lo; --lp) {
    const int nt = (t.off[lp + 1] - t.off[lp] + ROWS - 1) / ROWS;
    if (tile < nt) break;
    tile -= nt;
  }
  if (lp < lp_lo) return;  // whole workgroup, before any barrier
  const int pbeg = t.off[lp] + ROWS * tile;
  const int pend = min(pbeg + ROWS, t.off[lp + 1]);
  const int col = lane & 15, kq = lane >> 4;
  // targets of the two octants (A: octant j, B: octant 7 - j) in the lane's columns
  int tgtA[NCB], tgtB[NCB];
  bool anyA = false, anyB = false;
#pragma unroll
  for (int cb = 0; cb < NCB; ++cb) {
    const int P_ = pbeg + 16 * cb + col;
    tgtA[cb] = P_ < pend ? t.child8[8 * P_ + oc[0]] : -1;
    tgtB[cb] = P_ < pend ? t.child8[8 * P_ + oc[1]] : -1;
    anyA |= tgtA[cb] >= 0;
    anyB |= tgtB[cb] >= 0;
  }
  const bool activeA = __ballot(anyA) != 0, activeB = __ballot(anyB) != 0;
  for (int e = threadIdx.x; e < NBLK * 8; e += TPB) sHv[e] = reinterpret_cast<const uint4*>(op.hidx)[e];
  const unsigned short* sH = reinterpret_cast<const unsigned short*>(sHv);

  // ws lists: colleagues within ws; MAC: split partners within Rp.  Offsets d = u - 2 e of a slot
  // then lie within R = 2 ws + 1 (or 2 Rp + 1), the radius of the operator table.
  const int ws = MAC ? mv.Rp : t.ws, side = 2 * ws + 1, nn = MAC ? side * side * side : t.nnear;
  const int near_r = MAC ? mv.minsep - 1 : ws;  // offsets within this Chebyshev distance never interact
  const int* colls = MAC ? mv.split : t.coll;
  const int R = 2 * ws + 1, cube = 2 * R + 1;
  const kt* dtab;
  if constexpr (F32) dtab = MAC ? mv.dvec32 : op.dvec32; else dtab = MAC ? mv.dvec : op.dvec;
  const double wt = ldexp(t.w, t.L - (lp + 1));  // cell edge of the targets (MAC)

  constexpr const SchedHalves& HS = SchedHalvesOf<P>::value;
  constexpr int NLOC = HS.nloc;
  acc_t accA[NCB][NLOC], accB[NCB][NLOC];
#pragma unroll
  for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
    for (int l = 0; l < NLOC; ++l) {
      accA[cb][l] = acc_t{0, 0, 0, 0};
      accB[cb][l] = acc_t{0, 0, 0, 0};
    }

  // source rows pass through registers: loaded from global memory one slot before they are stored
  // to LDS, and stored one slot before they are read.  The float32 path reads the float32 copy of
  // the multipoles (half the registers and bytes of the float64 rows).
  double2 pre[F32 ? 1 : PF];
  float4 pre4[F32 ? PF4 : 1];
  // The schedule of order q reads the coefficients below count(q), rounded up to whole step pairs
  // (8), so a slot loads only those pieces of each source row, for the highest order among its
  // target octants (op.slotq, with the ws lists' per-offset orders) and at most the cap; the rest
  // of the staged row is never read.
  // (the float32 tiles, two column blocks, have no registers to spare for the per-slot bound: they
  // take the cap's alone)
  __shared__ int sNread[8];  // coefficients to load per source octant of the current offset
  const int nread_cap = (mi_count(min(P, qc)) + 7) / 8 * 8;
  auto prefetch = [&](int r) {
    const int nread = F32 ? nread_cap : sNread[r];
    if constexpr (F32) {
#pragma unroll
      for (int i = 0; i < PF4; ++i) {
        const int e = threadIdx.x + i * TPB;
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (e < ROWS * QUART) {
          const int row = e / QUART, h = e - row * QUART;
          const int src = sSrc[r][row];
          if (src >= 0 && 4 * h < nread) v = reinterpret_cast<const float4*>(M32 + (int64_t)src * STRIDE)[h];
        }
        pre4[i] = v;
      }
    } else {
#pragma unroll
      for (int i = 0; i < PF; ++i) {
        const int e = threadIdx.x + i * TPB;
        double2 v = make_double2(0.0, 0.0);
        if (e < ROWS * HALF) {
          const int row = e / HALF, h = e - row * HALF;
          const int src = sSrc[r][row];
          if (src >= 0 && 2 * h < nread) v = reinterpret_cast<const double2*>(M + (int64_t)src * STRIDE)[h];
        }
        pre[i] = v;
      }
    }
  };
  auto commit = [&](kt* dst) {
    if constexpr (F32) {
      // rows start at 8-byte multiples (pitch STRIDE + 2 floats): two 8-byte stores per piece
#pragma unroll
      for (int i = 0; i < PF4; ++i) {
        const int e = threadIdx.x + i * TPB;
        if (e < ROWS * QUART) {
          const int row = e / QUART, h = e - row * QUART;
          float2* d = reinterpret_cast<float2*>(dst + row * BP + 4 * h);
          d[0] = make_float2(pre4[i].x, pre4[i].y);
          d[1] = make_float2(pre4[i].z, pre4[i].w);
        }
      }
    } else {
#pragma unroll
      for (int i = 0; i < PF; ++i) {
        const int e = threadIdx.x + i * TPB;
        if (e < ROWS * HALF) {
          const int row = e / HALF, h = e - row * HALF;
          *reinterpret_cast<kt2*>(dst + row * BP + 2 * h) = kt2{(kt)pre[i].x, (kt)pre[i].y};
        }
      }
    }
  };
  // next live source octant after r, or -1
  auto next_live = [](unsigned live, int r) {
    const unsigned rest = live & ~((2u << r) - 1u);
    return rest ? __ffs(rest) - 1 : -1;
  };

  // split s takes the colleague offsets ci = s, s + nsplit, ...: every split then mixes the inner
  // offsets (mostly near-field, little M2L) with the outer ones, so the splits weigh alike
  for (int ci = split; ci < nn; ci += nsplit) {
    const int e0 = ci / (side * side) - ws, e1 = (ci / side) % side - ws, e2 = ci % side - ws;
    if (e0 == 0 && e1 == 0 && e2 == 0) continue;  // the parent's own children are all near
    __syncthreads();  // every wave is done with sSrc, sD and sB of the previous offset
    for (int e = threadIdx.x; e < 8 * ROWS; e += TPB) {
      const int c = e % ROWS, r = e / ROWS;
      int src = -1;
      if (pbeg + c < pend) {
        const int S = colls[(int64_t)(pbeg + c) * nn + ci];
        if (S >= 0) src = t.child8[8 * S + r];
      }
      sSrc[r][c] = src;
    }
    if (!F32 && threadIdx.x < 8) {
      const int qs = MAC && mv.use_theta ? min(P, qc) : min((int)op.slotq[ci * 8 + threadIdx.x], qc);
      sNread[threadIdx.x] = (mi_count(qs) + 7) / 8 * 8;
    }
    __syncthreads();
    unsigned live = 0;  // source octants with at least one source (same value in every thread)
    for (int r = 0; r < 8; ++r) {
      int any = 0;
      for (int c = 0; c < ROWS; ++c) any |= sSrc[r][c] >= 0;
      live |= (unsigned)any << r;
    }
    if (!live) continue;
    if constexpr (MAC) {
      // the criterion for every (target octant, column): bit r set when the pair with the column's
      // source of octant r is accepted (read after the barrier that opens the first slot)
      for (int e = threadIdx.x; e < 8 * ROWS; e += TPB) {
        const int o = e / ROWS, c = e - o * ROWS;
        const int tg = pbeg + c < pend ? t.child8[8 * (pbeg + c) + o] : -1;
        unsigned bits = 0u;
        if (tg >= 0) {
          for (int rr = 0; rr < 8; ++rr) {
            const int src = sSrc[rr][c];
            if (src < 0) continue;
            const int d0 = ((o >> 2) & 1) - ((rr >> 2) & 1) - 2 * e0, d1 = ((o >> 1) & 1) - ((rr >> 1) & 1) - 2 * e1,
                      d2 = (o & 1) - (rr & 1) - 2 * e2;
            if (mac_accept(t, mv, wt, tg, src, d0, d1, d2)) bits |= 1u << rr;
          }
        }
        sMask[o][c] = (unsigned char)bits;
      }
    }
    int r = __ffs(live) - 1;
    prefetch(r);
    for (int e = threadIdx.x; e < NU * DP; e += TPB) {
      const int v = e / DP, k = e - v * DP;
      const int d0 = v / 9 - 1 - 2 * e0, d1 = (v / 3) % 3 - 1 - 2 * e1, d2 = v % 3 - 1 - 2 * e2;
      if (max(abs(d0), max(abs(d1), abs(d2))) > near_r) {
        // D_k(d) for |k| <= q(d), zero above: the M2L truncated at order q(d)
        const int slot = ((d0 + R) * cube + (d1 + R)) * cube + (d2 + R);
        // (the ws rule of the adaptive octree keeps the ws lists' per-offset orders)
        const int q = MAC && mv.use_theta ? min(P, qc) : min((int)op.dorder[slot], qc);
        sD[e] = k < mi_count(q) ? dtab[(int64_t)slot * DP + k] : (kt)0;
        if (k == 0) sQ[v] = q;
      }
    }
    commit(sB[0]);
    int rn = next_live(live, r);
    if (rn >= 0) prefetch(rn);
    int buf = 0;
    while (true) {
      // the rows of slot r (and, on the first slot, sD) are visible, and every wave is done with
      // the slot before r, whose buffer now receives the rows of slot rn
      __syncthreads();
      int rnn = -1;
      if (rn >= 0) {
        commit(sB[buf ^ 1]);
        rnn = next_live(live, rn);
        if (rnn >= 0) prefetch(rnn);
      }
      // one octant of the pair at this slot (its accumulators are always named statically)
      auto octant_slot = [&](acc_t(&acc)[NCB][NLOC], int o, bool act) {
        const int u0 = ((o >> 2) & 1) - ((r >> 2) & 1), u1 = ((o >> 1) & 1) - ((r >> 1) & 1), u2 = (o & 1) - (r & 1);
        const int d0 = u0 - 2 * e0, d1 = u1 - 2 * e1, d2 = u2 - 2 * e2;
        if (act && max(abs(d0), max(abs(d1), abs(d2))) > near_r) {  // wave-uniform
          bool bm[NCB];
          bool run = true;
          if constexpr (MAC) {
            bool any = false;
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) {
              bm[cb] = (sMask[o][16 * cb + col] >> r) & 1u;
              any |= bm[cb];
            }
            run = __ballot(any) != 0;
          } else {
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) bm[cb] = true;
          }
          if (run) {
            const int v = (u0 + 1) * 9 + (u1 + 1) * 3 + (u2 + 1);
            const kt* Dv = sD + v * DP;
            const kt* Bp = sB[buf] + col * BP + 2 * kq;
            const int q = sQ[v];
            if (half == 0)
              m2l_slot<P, F32, NCB, 0, MAC, kt, kt2, acc_t>(q, Dv, Bp, sH, lane, acc, bm);
            else
              m2l_slot<P, F32, NCB, 1, MAC, kt, kt2, acc_t>(q, Dv, Bp, sH, lane, acc, bm);
          }
        }
      };
      octant_slot(accA, oc[0], activeA);
      octant_slot(accB, oc[1], activeB);
      if (rn < 0) break;
      r = rn;
      rn = rnn;
      buf ^= 1;
    }
  }
  // row block 0 is split between the halves: half 1 hands its partial sums to half 0 through LDS
  // (in the source buffers, free once every wave has passed this barrier, where they are large
  // enough)
  acc_t* xch = XCH_IN_SB ? reinterpret_cast<acc_t*>(&sB[0][0]) : sX;
  __syncthreads();
  if (half == 1) {
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
      xch[((0 * 4 + pair) * NCB + cb) * 64 + lane] = accA[cb][0];
      xch[((1 * 4 + pair) * NCB + cb) * 64 + lane] = accB[cb][0];
    }
  }
  __syncthreads();
  if (half == 0) {
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
      accA[cb][0] += xch[((0 * 4 + pair) * NCB + cb) * 64 + lane];
      accB[cb][0] += xch[((1 * 4 + pair) * NCB + cb) * 64 + lane];
    }
  }
  // each half writes the rows of its row blocks (row block 0: half 0, which holds the sum)
  auto write_rows = [&](const acc_t(&acc)[NCB][NLOC], const int(&tg)[NCB], auto hc) {
    constexpr int H = decltype(hc)::value;
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
      if (tg[cb] < 0) continue;
      double* Fr = F + (int64_t)split * split_stride + (int64_t)tg[cb] * STRIDE;
#pragma unroll
      for (int rb = 0; rb < NRB; ++rb) {
        if (SchedHalvesOf<P>::value.half[rb] != H) continue;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          // f64 16x16x4: lane l, register q holds row 4 q + l/16; f32 16x16x4: row 4 (l/16) + q
          const int row = 16 * rb + (F32 ? (4 * kq + q) : (4 * q + kq));
          if (row < NC) Fr[row] = (double)acc[cb][SchedHalvesOf<P>::value.loc[rb]][q];
        }
      }
    }
  };
  if (half == 0) {
    write_rows(accA, tgtA, std::integral_constant<int, 0>{});
    write_rows(accB, tgtB, std::integral_constant<int, 0>{});
  } else {
    write_rows(accA, tgtA, std::integral_constant<int, 1>{});
    write_rows(accB, tgtB, std::integral_constant<int, 1>{});
  }
}

// workgroups of a launch of nt tiles: whole chunks of M2L_XCD_TILES tiles on each of the 8 XCDs
int m2l_grid(int nt, int nsplit) {
  const int per = 8 * M2L_XCD_TILES * nsplit;
  return (nt * nsplit + per - 1) / per * per;
}

template <int P>
void m2l_dispatch(const TreeView& t, const OpTables& op, int nsplit, const double* M, const float* M32,
                  double* F, int64_t split_stride, bool fp32, int fp64_max_level, const int* done,
                  const int* qcap, hipStream_t s, const MacView* mac) {
  if (mac) {
    // parents of levels [1, L - 1] (L - 2 when leaf pairs are direct); on the mixed path float32
    // tiles below fp64_max_level, as for the ws lists.  At order 10 the accumulators of a tile leave
    // no registers for the rule's masks.
    if constexpr (P <= MAX_P_MAC) {
      const int lo = 1, hi = t.L - 1 - (mac->leaf_direct ? 1 : 0);
      const int hi64 = fp32 ? std::min(hi, fp64_max_level - 1) : hi;
      if (hi64 >= lo) {
        const int nt = m2l_tiles(t, lo, hi64, 1);
        if (nt > 0)
          hipLaunchKernelGGL((k_m2l<P, false, true>), dim3(m2l_grid(nt, nsplit)), dim3(TPB), 0, s, t, op, *mac, lo, hi64, nsplit, nt * nsplit, M, M32, F, split_stride, done, qcap);
      }
      const int lo32 = std::max(lo, hi64 + 1);
      if (fp32 && hi >= lo32) {
        const int nt = m2l_tiles(t, lo32, hi, 1);
        if (nt > 0)
          hipLaunchKernelGGL((k_m2l<P, true, true>), dim3(m2l_grid(nt, nsplit)), dim3(TPB), 0, s, t, op, *mac, lo32, hi, nsplit, nt * nsplit, M, M32, F, split_stride, done, qcap);
      }
    } else {
      throw Error(PFMM_ERR_INVALID_ARG, "the dual-walk lists (mac_theta, adaptive_leaf_max) support order_p up to 9");
    }
    return;
  }
  // parents of levels [1, L - 1]; float64 for targets at levels <= fp64_max_level on the mixed path
  const int lo = 1, hi = t.L - 1;
  const int hi64 = fp32 ? std::min(hi, fp64_max_level - 1) : hi;
  if (hi64 >= lo) {
    const int nt = m2l_tiles(t, lo, hi64, m2l_ncb<P, false>());
    if (nt > 0)
      hipLaunchKernelGGL((k_m2l<P, false, false>), dim3(m2l_grid(nt, nsplit)), dim3(TPB), 0, s, t, op, MacView(), lo, hi64, nsplit, nt * nsplit, M, M32, F, split_stride, done, qcap);
  }
  if (fp32) {
    const int lo32 = std::max(lo, hi64 + 1);
    if (hi >= lo32) {
      const int nt = m2l_tiles(t, lo32, hi, m2l_ncb<P, true>());
      if (nt > 0)
        hipLaunchKernelGGL((k_m2l<P, true, false>), dim3(m2l_grid(nt, nsplit)), dim3(TPB), 0, s, t, op, MacView(), lo32, hi, nsplit, nt * nsplit, M, M32, F, split_stride, done, qcap);
    }
  }
}

// Orders above the matrix-core kernel's (MAX_P_MFMA < p <= MAX_P): the same contraction on the
// vector units in float64, one workgroup per target cell B of levels 2..L.  For each source A, a
// child of a colleague of B's parent farther than ws from B, the workgroup stages the source row and
// the operator row D(d), d = B - A, truncated at the offset's order q(d) (or the cap), in LDS, and
// each thread accumulates its rows n of
//   F~_n(B) = sum_{|m| <= q - |n|} D_{n+m}(d) M~_m(A)
// in the sources' fixed order; F~(B) is written once (no offset splits).  Float64 on both precision
// paths.
constexpr int VTPB = 256;

template <int PM>
__global__ __launch_bounds__(VTPB) void k_m2l_vector(TreeView t, OpTables op, const double* __restrict__ M,
                                                     double* __restrict__ F, const int* done, const int* qcap) {
  if (done && *done) return;
  constexpr int NCM = mi_count(PM), DPM = sched_dpitch(PM);
  constexpr int RPT = (NCM + VTPB - 1) / VTPB;  // rows per thread
  __shared__ double sM[NCM];
  __shared__ double sD[DPM];
  __shared__ int sE[NCM];  // exponents of m packed nx | ny << 8 | nz << 16
  const int B = t.off[2] + blockIdx.x;
  const int nc = op.nc, p = op.p;
  const int qc = qcap ? min(*qcap, p) : p;
  const int ws = t.ws, R = 2 * ws + 1, cube = 2 * R + 1;
  for (int k = threadIdx.x; k < nc; k += VTPB) sE[k] = op.mi[3 * k] | (op.mi[3 * k + 1] << 8) | (op.mi[3 * k + 2] << 16);
  int cb[3];
  {
    const uint64_t k = t.key[B];
    cb[0] = compact3(k >> 2); cb[1] = compact3(k >> 1); cb[2] = compact3(k);
  }
  int rn[RPT], rdeg[RPT];
  double acc[RPT];
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    rn[r] = threadIdx.x + r * VTPB;
    rdeg[r] = rn[r] < nc ? op.mi[3 * rn[r]] + op.mi[3 * rn[r] + 1] + op.mi[3 * rn[r] + 2] : PM + 1;
    acc[r] = 0.0;
  }
  const int P_ = t.parent[B];
  for (int k = 0; k < t.nnear; ++k) {
    const int S = t.coll[(int64_t)P_ * t.nnear + k];
    if (S < 0) continue;
    for (int c = 0; c < 8; ++c) {
      const int A = t.child8[8 * S + c];
      if (A < 0) continue;
      const uint64_t ka = t.key[A];
      const int d0 = cb[0] - compact3(ka >> 2), d1 = cb[1] - compact3(ka >> 1), d2 = cb[2] - compact3(ka);
      if (max(abs(d0), max(abs(d1), abs(d2))) <= ws) continue;  // uniform over the workgroup
      const int slot = ((d0 + R) * cube + (d1 + R)) * cube + (d2 + R);
      const int q = min((int)op.dorder[slot], qc);
      const int nq = mi_count(q);
      __syncthreads();  // the previous source's rows are no longer read
      for (int j = threadIdx.x; j < nq; j += VTPB) {
        sM[j] = M[(int64_t)A * op.stride + j];
        sD[j] = op.dvec[(int64_t)slot * sched_dpitch(p) + j];
      }
      __syncthreads();
#pragma unroll
      for (int r = 0; r < RPT; ++r) {
        const int dn = rdeg[r];
        if (dn > q) continue;
        const int n = rn[r];
        const int nx = op.mi[3 * n], ny = op.mi[3 * n + 1], nz = op.mi[3 * n + 2];
        const int cnt = mi_count(q - dn);
        double a = 0.0;
        for (int m = 0; m < cnt; ++m) {
          const int e = sE[m];
          a = fma(sD[mi_index(nx + (e & 0xff), ny + ((e >> 8) & 0xff), nz + (e >> 16))], sM[m], a);
        }
        acc[r] += a;
      }
    }
  }
#pragma unroll
  for (int r = 0; r < RPT; ++r)
    if (rn[r] < op.stride) F[(int64_t)B * op.stride + rn[r]] = rn[r] < nc ? acc[r] : 0.0;
  for (int k = NCM + threadIdx.x; k < op.stride; k += VTPB) F[(int64_t)B * op.stride + k] = 0.0;
}

}  // namespace

__global__ __launch_bounds__(256) void k_to_float(const double* __restrict__ in, float* __restrict__ out,
                                                   int64_t count, const int* done) {
  if (done && *done) return;
  for (int64_t k = blockIdx.x * 256 + threadIdx.x; k < count; k += (int64_t)gridDim.x * 256) out[k] = (float)in[k];
}

void launch_to_float(const double* in, float* out, int64_t count, const int* done, hipStream_t s) {
  if (count <= 0) return;
  const int64_t blocks = std::min<int64_t>((count + 255) / 256, 16384);
  hipLaunchKernelGGL(k_to_float, dim3((unsigned)blocks), dim3(256), 0, s, in, out, count, done);
  PFMM_LAUNCH_CHECK();
}

int m2l_tile_ncb(int p, bool fp32) {
  switch (p) {
#define PFMM_NCB_CASE(PP) \
  case PP:                \
    return fp32 ? m2l_ncb<PP, true>() : m2l_ncb<PP, false>();
    PFMM_NCB_CASE(1) PFMM_NCB_CASE(2) PFMM_NCB_CASE(3) PFMM_NCB_CASE(4) PFMM_NCB_CASE(5)
    PFMM_NCB_CASE(6) PFMM_NCB_CASE(7) PFMM_NCB_CASE(8) PFMM_NCB_CASE(9) PFMM_NCB_CASE(10)
#undef PFMM_NCB_CASE
    default: return 1;  // the vector M2L of the higher orders
  }
}

int m2l_tiles(const TreeView& t, int lp_lo, int lp_hi, int ncb) {
  int n = 0;
  for (int lp = std::max(lp_lo, 0); lp <= lp_hi && lp < t.L; ++lp)
    n += (t.off[lp + 1] - t.off[lp] + 16 * ncb - 1) / (16 * ncb);
  return n;
}

void launch_m2l(const TreeView& t, const OpTables& op, int nsplit, const double* M, const float* M32,
                double* F, int64_t split_stride, bool fp32, int fp64_max_level, const int* done,
                const int* qcap, hipStream_t s, const MacView* mac) {
  if (t.L < 2) return;
  const int side = mac ? 2 * mac->Rp + 1 : 0;
  if (nsplit < 1 || nsplit > (mac ? side * side * side : t.nnear))
    throw Error(PFMM_ERR_INVALID_ARG, "internal: M2L split out of range");
  if (mac && (!mac->split || !mac->dvec || (mac->use_theta && !mac->renc) || mac->Rp < 1 || mac->minsep < 2 ||
              (mac->nonleaf && (!mac->lfirst || !mac->lcount))))
    throw Error(PFMM_ERR_INVALID_ARG, "internal: dual-walk M2L inputs missing");
  if (op.p > MAX_P_MFMA) {
    if (mac || nsplit != 1 || op.p > MAX_P) throw Error(PFMM_ERR_INVALID_ARG, "internal: vector M2L configuration");
    const int nt = t.ncell - t.off[2];  // target cells of levels 2..L
    if (nt > 0)
      hipLaunchKernelGGL(k_m2l_vector<MAX_P>, dim3(nt), dim3(VTPB), 0, s, t, op, M, F, done, qcap);
    PFMM_LAUNCH_CHECK();
    return;
  }
  if (fp32 && (!(mac ? mac->dvec32 : op.dvec32) || !M32))
    throw Error(PFMM_ERR_INVALID_ARG, "internal: float32 M2L inputs missing");
  switch (op.p) {
#define PFMM_M2L_CASE(PP)                                                                               \
  case PP:                                                                                              \
    m2l_dispatch<PP>(t, op, nsplit, M, M32, F, split_stride, fp32, fp64_max_level, done, qcap, s, mac); \
    break;
    PFMM_M2L_CASE(1) PFMM_M2L_CASE(2) PFMM_M2L_CASE(3) PFMM_M2L_CASE(4) PFMM_M2L_CASE(5)
    PFMM_M2L_CASE(6) PFMM_M2L_CASE(7) PFMM_M2L_CASE(8) PFMM_M2L_CASE(9) PFMM_M2L_CASE(10)
#undef PFMM_M2L_CASE
    default: throw Error(PFMM_ERR_INVALID_ARG, "order_p out of range");
  }
  PFMM_LAUNCH_CHECK();
}

}  // namespace pfmm
