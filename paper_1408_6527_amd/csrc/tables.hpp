// Constant operator tables of the Cartesian FMM (Sec. II.B), built on the host once per (p, ws)
// and uploaded to the device.  Every expansion on the device is stored in level-scaled form:
//   M~_n = M_n / w^|n|,   F~_n = F_n * w^(|n|+1),
// where w is the edge of the cell's level.  With this scaling the M2L kernel for an offset of
// d cells is D_{n+m}(d) at unit cell width on every level (homogeneity of 1/r).
#pragma once

#include <cstdint>
#include <vector>

#include "common.hpp"

namespace pfmm {

struct HostTables {
  int p = 0, ws = 0, nc = 0, stride = 0;
  int nnear = 0;        // (2 ws + 1)^3 colleagues per cell
  int noff = 0;         // M2L offsets per target octant: (4 ws + 2)^3 - (2 ws + 1)^3
  int R = 0;            // offsets span [-R, R]^3 with R = 2 ws + 1
  int nslot = 0;        // (2R + 1)^3 offset slots
  int nblocks = 0;      // MFMA blocks per offset (schedule.hpp)

  std::vector<int> mi;          // nc x 3 exponents
  std::vector<double> inv_fact; // nc
  std::vector<double> p2m_coef; // nc: (-1)^|n| / n!
  std::vector<int> idx_e;       // nc x 3: index of n + e_c, or -1 (needs |n| <= p - 1)
  std::vector<int> idx_ee;      // nc x 6: index of n + e_a + e_b for (xx, yy, zz, xy, xz, yz), or -1
  std::vector<int> l2p_tab;     // nc x 16: nx, ny, nz, |n|, idx_e (3), idx_ee (6), 0 0 0
  // M2L: for each target octant, noff entries packed as
  //   slot | (colleague index of the source's parent) << 12 | (source octant) << 20
  std::vector<int> m2l_code;    // 8 x noff
  int dpitch = 0;                // sched_dpitch(p)
  std::vector<double> dvec;      // nslot x dpitch: D_k(d) of every offset slot, zero-padded
  std::vector<unsigned short> hidx;  // index of K[n][m] in a dvec row per block and lane (sched_hpos)

  // truncation order of the M2L per offset slot (0 for the near slots), see offset_order()
  std::vector<unsigned char> dorder;
  // per colleague offset e (index ((e + ws) (2 ws + 1) + ...)) and source octant c: the highest order
  // over the eight target octants o of the offsets d = o - c - 2 e that interact (0 if none)
  std::vector<unsigned char> slotq;

  void build(int p, int ws, int order_slack);
};

// Truncation order of the M2L at the integer cell offset d: with slack < 0 the fixed order p;
// otherwise the smallest q whose bound on the relative truncation error at this offset,
// (sqrt(3)/|d|)^(q+1) (two unit cells of radius sqrt(3)/2, centres |d| apart), does not exceed the
// bound of the nearest offsets at order p, (sqrt(3)/(ws+1))^(p+1), plus slack, capped at p.
// Decided exactly in integers: 3^(q+1) (ws+1)^(2(p+1)) <= 3^(p+1) |d|^(2(q+1)).
int offset_order(const int d[3], int p, int ws, int slack);

// D_n(d) = d^n (1/|d|) for |n| <= p at an integer offset d, by the Taylor-coefficient recurrence
// |n| r^2 a_n = -(2|n| - 1) sum_i d_i a_{n - e_i} - (|n| - 1) sum_i a_{n - 2 e_i},  D_n = n! a_n.
void derivative_tensor_unit(int p, const int* mi, int nc, const int d[3], double* out);

// The operators of the acceptance-criterion lists: D_k(d), |k| <= p, at unit cell width for every
// offset d in [-R, R]^3 of Chebyshev norm >= 2, one row per slot ((dx + R)(2R + 1) + dy + R)(2R + 1)
// + dz + R at the pitch dpitch of dvec, zero-padded (zero rows for the other slots).
std::vector<double> mac_operator_rows(const HostTables& t, int R);

}  // namespace pfmm
