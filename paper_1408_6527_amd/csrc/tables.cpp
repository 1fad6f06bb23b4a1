// Host construction of the FMM operator tables (Sec. II.B; multi-index notation of App. D).
#include "tables.hpp"

#include <cmath>

#include "schedule.hpp"

namespace pfmm {

namespace {

long double fact_ld(int k) {
  long double f = 1;
  for (int i = 2; i <= k; ++i) f *= i;
  return f;
}

long double ipow(long double x, int k) {
  long double r = 1;
  for (int i = 0; i < k; ++i) r *= x;
  return r;
}

// Multi-indices of degree <= p, ordered by degree, then by descending n_x, then descending n_y.
struct MIndex {
  int p;
  std::vector<int> e;    // nc x 3
  std::vector<int> lut;  // (p+1)^3 -> index or -1
  explicit MIndex(int p_) : p(p_), lut((p_ + 1) * (p_ + 1) * (p_ + 1), -1) {
    for (int d = 0; d <= p; ++d)
      for (int nx = d; nx >= 0; --nx)
        for (int ny = d - nx; ny >= 0; --ny) {
          int nz = d - nx - ny;
          lut[(nx * (p + 1) + ny) * (p + 1) + nz] = (int)(e.size() / 3);
          e.push_back(nx);
          e.push_back(ny);
          e.push_back(nz);
        }
  }
  int nc() const { return (int)e.size() / 3; }
  int at(int x, int y, int z) const {
    if (x < 0 || y < 0 || z < 0 || x + y + z > p) return -1;
    return lut[(x * (p + 1) + y) * (p + 1) + z];
  }
  int deg(int k) const { return e[3 * k] + e[3 * k + 1] + e[3 * k + 2]; }
  long double fact(int k) const { return fact_ld(e[3 * k]) * fact_ld(e[3 * k + 1]) * fact_ld(e[3 * k + 2]); }
};

}  // namespace

void derivative_tensor_unit(int p, const int* mi, int nc, const int d[3], double* out) {
  MIndex ix(p);
  std::vector<long double> a(nc, 0.0L);
  const long double R[3] = {(long double)d[0], (long double)d[1], (long double)d[2]};
  const long double r2 = R[0] * R[0] + R[1] * R[1] + R[2] * R[2];
  // a is indexed in the caller's order `mi`; map through exponents
  std::vector<int> pos(nc);
  for (int k = 0; k < nc; ++k) pos[ix.at(mi[3 * k], mi[3 * k + 1], mi[3 * k + 2])] = k;
  auto A = [&](int x, int y, int z) -> long double& { return a[pos[ix.at(x, y, z)]]; };
  A(0, 0, 0) = 1.0L / std::sqrt(r2);
  for (int k = 1; k < nc; ++k) {  // ix order = increasing degree, so dependencies come first
    const int n[3] = {ix.e[3 * k], ix.e[3 * k + 1], ix.e[3 * k + 2]};
    const int dg = n[0] + n[1] + n[2];
    long double acc = 0;
    for (int i = 0; i < 3; ++i) {
      if (n[i] >= 1) {
        int m[3] = {n[0], n[1], n[2]};
        m[i] -= 1;
        acc -= (2 * dg - 1) * R[i] * A(m[0], m[1], m[2]);
      }
      if (n[i] >= 2) {
        int m[3] = {n[0], n[1], n[2]};
        m[i] -= 2;
        acc -= (dg - 1) * A(m[0], m[1], m[2]);
      }
    }
    A(n[0], n[1], n[2]) = acc / (dg * r2);
  }
  for (int k = 0; k < nc; ++k)
    out[k] = (double)(a[k] * fact_ld(mi[3 * k]) * fact_ld(mi[3 * k + 1]) * fact_ld(mi[3 * k + 2]));
}

int offset_order(const int d[3], int p, int ws, int slack) {
  if (slack < 0) return p;
  typedef unsigned __int128 u128;
  const u128 r2 = (u128)(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  u128 base = 1;
  for (int k = 0; k < 2 * (p + 1); ++k) base *= (u128)(ws + 1);
  u128 three_p1 = 1;
  for (int k = 0; k < p + 1; ++k) three_p1 *= 3;
  int q = 0;
  u128 three_q1 = 3, r2_q1 = r2;  // 3^(q+1), r2^(q+1)
  while (q < p && three_q1 * base > three_p1 * r2_q1) {
    ++q;
    three_q1 *= 3;
    r2_q1 *= r2;
  }
  return std::min(p, q + slack);
}

void HostTables::build(int p_, int ws_, int order_slack) {
  p = p_;
  ws = ws_;
  MIndex ix(p);
  nc = ix.nc();
  stride = sched_stride(p);
  const int side = 2 * ws + 1;
  nnear = side * side * side;
  R = 2 * ws + 1;
  const int cube = 2 * R + 1;
  nslot = cube * cube * cube;
  noff = (4 * ws + 2) * (4 * ws + 2) * (4 * ws + 2) - nnear;
  nblocks = sched_nblocks(p);

  mi = ix.e;
  inv_fact.resize(nc);
  p2m_coef.resize(nc);
  idx_e.assign(3 * nc, -1);
  idx_ee.assign(6 * nc, -1);
  for (int k = 0; k < nc; ++k) {
    const int x = mi[3 * k], y = mi[3 * k + 1], z = mi[3 * k + 2];
    inv_fact[k] = (double)(1.0L / ix.fact(k));
    p2m_coef[k] = (double)(((x + y + z) % 2 ? -1.0L : 1.0L) / ix.fact(k));
    idx_e[3 * k + 0] = ix.at(x + 1, y, z);
    idx_e[3 * k + 1] = ix.at(x, y + 1, z);
    idx_e[3 * k + 2] = ix.at(x, y, z + 1);
    idx_ee[6 * k + 0] = ix.at(x + 2, y, z);
    idx_ee[6 * k + 1] = ix.at(x, y + 2, z);
    idx_ee[6 * k + 2] = ix.at(x, y, z + 2);
    idx_ee[6 * k + 3] = ix.at(x + 1, y + 1, z);
    idx_ee[6 * k + 4] = ix.at(x + 1, y, z + 1);
    idx_ee[6 * k + 5] = ix.at(x, y + 1, z + 1);
  }

  l2p_tab.assign(16 * nc, 0);
  for (int k = 0; k < nc; ++k) {
    for (int a = 0; a < 3; ++a) l2p_tab[16 * k + a] = mi[3 * k + a];
    l2p_tab[16 * k + 3] = ix.deg(k);
    for (int a = 0; a < 3; ++a) l2p_tab[16 * k + 4 + a] = std::max(idx_e[3 * k + a], 0);
    for (int a = 0; a < 6; ++a) l2p_tab[16 * k + 7 + a] = std::max(idx_ee[6 * k + a], 0);
  }

  // M2L offsets per target octant.  A target B in octant oB of its parent P sees, through the
  // children of P's colleagues, the cells A = 2 (P + e) + c, e in [-ws, ws]^3, c in {0,1}^3, and
  // interacts by M2L with those that are not its own colleagues: d = B - A = oB - c - 2 e with
  // Chebyshev |d| > ws.
  m2l_code.assign(8 * noff, 0);
  for (int o = 0; o < 8; ++o) {
    const int ob[3] = {(o >> 2) & 1, (o >> 1) & 1, o & 1};
    int cnt = 0;
    for (int tx = -2 * ws; tx <= 2 * ws + 1; ++tx)
      for (int ty = -2 * ws; ty <= 2 * ws + 1; ++ty)
        for (int tz = -2 * ws; tz <= 2 * ws + 1; ++tz) {
          const int t[3] = {tx, ty, tz};  // t = oB - d = c + 2 e
          int d[3], e[3], c[3];
          int cheb = 0;
          for (int a = 0; a < 3; ++a) {
            d[a] = ob[a] - t[a];
            c[a] = ((t[a] % 2) + 2) % 2;
            e[a] = (t[a] - c[a]) / 2;
            cheb = std::max(cheb, std::abs(d[a]));
          }
          if (cheb <= ws) continue;
          const int slot = ((d[0] + R) * cube + (d[1] + R)) * cube + (d[2] + R);
          const int coll = ((e[0] + ws) * side + (e[1] + ws)) * side + (e[2] + ws);
          const int oct = (c[0] << 2) | (c[1] << 1) | c[2];
          m2l_code[o * noff + cnt] = slot | (coll << 12) | (oct << 20);
          ++cnt;
        }
    if (cnt != noff) throw Error(PFMM_ERR_INVALID_ARG, "internal: M2L offset count mismatch");
  }

  // D_k(d) for every offset slot (zeros for the near slots, which no M2L reads), each row followed
  // by zeros up to the pitch; and the index of K[n][m] = D_{n+m} for every MFMA block (rb, s) and
  // lane l, n = 16 rb + (l & 15), m = m(s, l >> 4) (schedule.hpp), pointing at the zero entry nc
  // where |n| + |m| > p or n, m fall in the padding.
  dpitch = sched_dpitch(p);
  dvec.assign((size_t)nslot * dpitch, 0.0);
  dorder.assign((size_t)nslot, 0);
  std::vector<double> Dn(nc);
  for (int dx = -R; dx <= R; ++dx)
    for (int dy = -R; dy <= R; ++dy)
      for (int dz = -R; dz <= R; ++dz) {
        if (std::max(std::abs(dx), std::max(std::abs(dy), std::abs(dz))) <= ws) continue;
        const int slot = ((dx + R) * cube + (dy + R)) * cube + (dz + R);
        const int d[3] = {dx, dy, dz};
        derivative_tensor_unit(p, mi.data(), nc, d, Dn.data());
        std::copy(Dn.begin(), Dn.end(), dvec.begin() + (size_t)slot * dpitch);
        dorder[slot] = (unsigned char)offset_order(d, p, ws, order_slack);
      }
  {
    const int side = 2 * ws + 1, nn = side * side * side;
    slotq.assign((size_t)nn * 8, 0);
    for (int ci = 0; ci < nn; ++ci) {
      const int e[3] = {ci / (side * side) - ws, (ci / side) % side - ws, ci % side - ws};
      for (int c = 0; c < 8; ++c) {
        int qm = 0;
        for (int o = 0; o < 8; ++o) {
          int d[3], cheb = 0;
          for (int a = 0; a < 3; ++a) {
            d[a] = ((o >> (2 - a)) & 1) - ((c >> (2 - a)) & 1) - 2 * e[a];
            cheb = std::max(cheb, std::abs(d[a]));
          }
          if (cheb <= ws) continue;
          qm = std::max(qm, (int)dorder[((d[0] + R) * cube + (d[1] + R)) * cube + (d[2] + R)]);
        }
        slotq[(size_t)ci * 8 + c] = (unsigned char)qm;
      }
    }
  }
  std::vector<int> degv(nc);
  for (int k = 0; k < nc; ++k) degv[k] = ix.deg(k);
  const int nrb = sched_nrb(p);
  hidx.assign((size_t)nblocks * 64, (unsigned short)nc);
  int blk = 0;
  for (int s = 0; s < sched_maxsteps(p); ++s)
    for (int rb = 0; rb < nrb; ++rb) {
      if (sched_nsteps(p, rb) <= s) continue;
      for (int l = 0; l < 64; ++l) {
        const int row = 16 * rb + (l & 15), col = sched_coef(s, l >> 4);
        if (row < nc && col < nc && degv[row] + degv[col] <= p)
          hidx[sched_hpos(blk, l)] = (unsigned short)ix.at(
              mi[3 * row] + mi[3 * col], mi[3 * row + 1] + mi[3 * col + 1], mi[3 * row + 2] + mi[3 * col + 2]);
      }
      ++blk;
    }
  if (blk != nblocks) throw Error(PFMM_ERR_INVALID_ARG, "internal: M2L block count mismatch");
}

std::vector<double> mac_operator_rows(const HostTables& t, int R) {
  const int cube = 2 * R + 1, nc = t.nc, dp = t.dpitch;
  std::vector<double> rows((size_t)cube * cube * cube * dp, 0.0);
  for (int dx = -R; dx <= R; ++dx)
    for (int dy = -R; dy <= R; ++dy)
      for (int dz = -R; dz <= R; ++dz) {
        if (std::max(std::abs(dx), std::max(std::abs(dy), std::abs(dz))) < 2) continue;
        const int slot = ((dx + R) * cube + (dy + R)) * cube + (dz + R);
        const int d[3] = {dx, dy, dz};
        derivative_tensor_unit(t.p, t.mi.data(), nc, d, rows.data() + (size_t)slot * dp);
      }
  return rows;
}

}  // namespace pfmm
