"""The host side of the operator tables (csrc/tables.cpp) and the M2L schedule (csrc/schedule.hpp),
built with g++ under AddressSanitizer and UndefinedBehaviorSanitizer, for every order p = 1..12, both
separations and several order slacks, with every index the kernels read from the tables checked
against the range of what it indexes:

* multi-index tables: exponents sum to the degree, n + e_c and n + e_a + e_b indices in range (or
  -1 exactly when the degree would exceed p), L2P table entries in [0, nc);
* M2L codes: offset slot, colleague index and source octant in range, the slot's offset equal to
  oB - c - 2 e and farther than ws (Chebyshev), every far offset of the cube listed once per octant;
* derivative rows: finite, zero beyond nc in every pitch, zero at the near slots;
* K-entry index table: each (block, lane) points at n + m inside the staircase |n| + |m| <= p and at
  the zero entry nc everywhere else, and stays inside one row pitch;
* truncation orders within [0, p] and non-increasing with the offset's length;
* row halves of the schedule: every row block owned once, accumulator slots below nloc <= 32.
No GPU call is made; the device code is not built here.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1408_6527_amd", "csrc")

DRIVER = r'''
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>
#include "tables.hpp"
#include "schedule.hpp"
using namespace pfmm;
static int fails = 0;
#define CHECK(c) do { if (!(c)) { std::printf("FAIL p=%d ws=%d slack=%d: %s (line %d)\n", p, ws, slack, #c, __LINE__); if (++fails > 20) std::exit(1); } } while (0)
int main() {
  for (int p = 1; p <= 12; ++p)
    for (int ws = 1; ws <= 2; ++ws)
      for (int slack = -1; slack <= 3; ++slack) {
        HostTables t;
        t.build(p, ws, slack);
        const int nc = t.nc;
        CHECK(nc == sched_nc(p) && t.stride == sched_stride(p) && t.stride >= nc && t.stride % 8 == 0);
        CHECK((int)t.mi.size() == 3 * nc && (int)t.l2p_tab.size() == 16 * nc);
        std::vector<int> deg(nc);
        for (int k = 0; k < nc; ++k) deg[k] = t.mi[3 * k] + t.mi[3 * k + 1] + t.mi[3 * k + 2];
        for (int k = 0; k < nc; ++k) {
          CHECK(deg[k] <= p && (k == 0 || deg[k] >= deg[k - 1]));
          CHECK(t.l2p_tab[16 * k + 3] == deg[k]);
          for (int a = 0; a < 3; ++a) {
            const int i = t.idx_e[3 * k + a];
            CHECK(i >= -1 && i < nc && ((i < 0) == (deg[k] + 1 > p)));
            if (i >= 0) CHECK(deg[i] == deg[k] + 1 && t.mi[3 * i + a] == t.mi[3 * k + a] + 1);
            CHECK(t.l2p_tab[16 * k + 4 + a] >= 0 && t.l2p_tab[16 * k + 4 + a] < nc);
          }
          for (int a = 0; a < 6; ++a) {
            const int i = t.idx_ee[6 * k + a];
            CHECK(i >= -1 && i < nc && ((i < 0) == (deg[k] + 2 > p)));
            if (i >= 0) CHECK(deg[i] == deg[k] + 2);
            CHECK(t.l2p_tab[16 * k + 7 + a] >= 0 && t.l2p_tab[16 * k + 7 + a] < nc);
          }
          CHECK(std::isfinite(t.inv_fact[k]) && t.inv_fact[k] > 0 && std::fabs(t.p2m_coef[k]) == t.inv_fact[k]);
        }
        // M2L codes
        const int side = 2 * ws + 1, R = 2 * ws + 1, cube = 2 * R + 1;
        CHECK(t.nnear == side * side * side && t.nslot == cube * cube * cube);
        CHECK((int)t.m2l_code.size() == 8 * t.noff);
        for (int o = 0; o < 8; ++o) {
          std::vector<int> seen(t.nslot, 0);
          for (int k = 0; k < t.noff; ++k) {
            const int code = t.m2l_code[o * t.noff + k];
            const int slot = code & 0xfff, coll = (code >> 12) & 0xff, oct = (code >> 20) & 0xf;
            CHECK(slot >= 0 && slot < t.nslot && coll >= 0 && coll < t.nnear && oct >= 0 && oct < 8);
            const int d[3] = {slot / (cube * cube) - R, (slot / cube) % cube - R, slot % cube - R};
            const int e[3] = {coll / (side * side) - ws, (coll / side) % side - ws, coll % side - ws};
            const int c[3] = {(oct >> 2) & 1, (oct >> 1) & 1, oct & 1};
            const int ob[3] = {(o >> 2) & 1, (o >> 1) & 1, o & 1};
            int cheb = 0;
            for (int a = 0; a < 3; ++a) {
              CHECK(d[a] == ob[a] - c[a] - 2 * e[a]);
              cheb = std::max(cheb, std::abs(d[a]));
            }
            CHECK(cheb > ws && cheb <= R);
            seen[slot] += 1;
          }
          int listed = 0;
          for (int s = 0; s < t.nslot; ++s) { CHECK(seen[s] <= 1); listed += seen[s]; }
          CHECK(listed == t.noff);
        }
        // derivative rows, orders
        const int dp = t.dpitch;
        CHECK(dp == sched_dpitch(p) && dp > nc && (int)t.dvec.size() == t.nslot * dp);
        for (int s = 0; s < t.nslot; ++s) {
          const int d[3] = {s / (cube * cube) - R, (s / cube) % cube - R, s % cube - R};
          const int cheb = std::max(std::abs(d[0]), std::max(std::abs(d[1]), std::abs(d[2])));
          for (int k = 0; k < dp; ++k) {
            const double v = t.dvec[(size_t)s * dp + k];
            CHECK(std::isfinite(v));
            if (k >= nc || cheb <= ws) CHECK(v == 0.0);
          }
          const int q = t.dorder[s];
          CHECK(q >= 0 && q <= p);
          if (cheb > ws) CHECK(q == offset_order(d, p, ws, slack));
          if (slack < 0 && cheb > ws) CHECK(q == p);
        }
        for (int s = 0; s < t.nslot; ++s)
          for (int u = 0; u < t.nslot; ++u) {
            const int a[3] = {s / (cube * cube) - R, (s / cube) % cube - R, s % cube - R};
            const int b[3] = {u / (cube * cube) - R, (u / cube) % cube - R, u % cube - R};
            const int ca = std::max(std::abs(a[0]), std::max(std::abs(a[1]), std::abs(a[2])));
            const int cb = std::max(std::abs(b[0]), std::max(std::abs(b[1]), std::abs(b[2])));
            if (ca <= ws || cb <= ws) continue;
            const int ra = a[0] * a[0] + a[1] * a[1] + a[2] * a[2], rb = b[0] * b[0] + b[1] * b[1] + b[2] * b[2];
            if (ra < rb) CHECK(t.dorder[s] >= t.dorder[u]);
          }
        // K-entry indices
        CHECK(t.nblocks == sched_nblocks(p) && (int)t.hidx.size() == 64 * t.nblocks);
        int blk = 0;
        for (int st = 0; st < sched_maxsteps(p); ++st)
          for (int rb = 0; rb < sched_nrb(p); ++rb) {
            if (sched_nsteps(p, rb) <= st) continue;
            for (int l = 0; l < 64; ++l) {
              const int h = t.hidx[sched_hpos(blk, l)];
              CHECK(h >= 0 && h < dp);
              const int row = 16 * rb + (l & 15), col = sched_coef(st, l >> 4);
              if (row < nc && col < nc && deg[row] + deg[col] <= p) {
                CHECK(h < nc && deg[h] == deg[row] + deg[col]);
                for (int a = 0; a < 3; ++a) CHECK(t.mi[3 * h + a] == t.mi[3 * row + a] + t.mi[3 * col + a]);
              } else {
                CHECK(h == nc);
              }
            }
            ++blk;
          }
        CHECK(blk == t.nblocks);
        // row halves of the schedule
        const SchedHalves hs = sched_halves(p);
        CHECK(hs.nloc >= 1 && hs.nloc <= 32 && sched_nrb(p) <= 32);
        int cnt[2] = {1, 1};
        for (int rb = 1; rb < sched_nrb(p); ++rb) {
          CHECK(hs.half[rb] == 0 || hs.half[rb] == 1);
          CHECK(hs.loc[rb] == cnt[hs.half[rb]]);
          cnt[hs.half[rb]] += 1;
          CHECK(hs.loc[rb] < hs.nloc);
        }
      }
  std::printf(fails ? "FAILED\n" : "OK\n");
  return fails ? 1 : 0;
}
'''


@pytest.mark.slow
def test_tables_and_schedule_under_address_and_ub_sanitizers(tmp_path):
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("no g++")
    src = tmp_path / "driver.cpp"
    src.write_text(DRIVER)
    exe = tmp_path / "driver"
    cmd = [cxx, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-fno-omit-frame-pointer", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", f"-I{CSRC}",
           os.path.join(CSRC, "tables.cpp"), str(src), "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    # the sanitizer runtime need not be the first library of the process
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0", UBSAN_OPTIONS="print_stacktrace=1")
    out = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=600)
    assert out.returncode == 0 and out.stdout.strip().endswith("OK"), (out.stdout[-4000:], out.stderr[-4000:])
