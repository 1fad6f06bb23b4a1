"""Host logic of the M2L schedule (paper_1408_6527_amd/csrc/schedule.hpp), compiled with the host C++
compiler: the degree-blocked block counts against a brute-force count of the MFMA blocks that the
truncation |n| + |m| <= q needs, and the split of the row blocks between the two waves of a SIMD
(every row block owned once, static accumulator slots, balanced work at the orders it is built
for).  No GPU call is made here."""
import os
import shutil
import subprocess
from math import comb

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SCHED = os.path.join(ROOT, "paper_1408_6527_amd", "csrc", "schedule.hpp")


def mi_count(d):
    return 0 if d < 0 else comb(d + 3, 3)


def deg_of(row):
    d = 0
    while mi_count(d) <= row:
        d += 1
    return d


def coef(s, q):
    return 8 * (s // 2) + 2 * q + (s % 2)


@pytest.fixture(scope="module")
def tables(tmp_path_factory):
    cxx = shutil.which("g++") or shutil.which("c++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    d = tmp_path_factory.mktemp("sched")
    src = d / "dump.cpp"
    src.write_text(r'''
#define __host__
#define __device__
#include <cstdio>
#include "SCHED"
using namespace pfmm;
int main() {
  for (int c = 0; c <= 300; ++c) printf("below %d %d\n", c, sched_steps_below(c));
  for (int p = 1; p <= 10; ++p) {
    const SchedHalves hs = sched_halves(p);
    printf("p %d %d %d %d %d\n", p, sched_nblocks(p), sched_nrb(p), sched_maxsteps(p), hs.nloc);
    for (int rb = 0; rb < sched_nrb(p); ++rb)
      printf("rb %d %d %d %d %d\n", p, rb, sched_nsteps(p, rb), hs.half[rb], hs.loc[rb]);
  }
  return 0;
}
'''.replace("SCHED", SCHED))
    exe = d / "dump"
    subprocess.run([cxx, "-std=c++17", "-O1", str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    below, head, rbs = {}, {}, {}
    for line in out:
        f = line.split()
        if not f:
            continue
        if f[0] == "below":
            below[int(f[1])] = int(f[2])
        elif f[0] == "p":
            head[int(f[1])] = tuple(map(int, f[2:]))
        else:
            rbs[(int(f[1]), int(f[2]))] = tuple(map(int, f[3:]))
    return below, head, rbs


def test_steps_below_counts_quarter0_coefficients(tables):
    below, _, _ = tables
    for c in range(301):
        assert below[c] == sum(1 for s in range(200) if coef(s, 0) < c)


def test_blocks_cover_the_truncated_staircase(tables):
    """Every non-zero entry K[n][m] (|n| + |m| <= p) lies in exactly one scheduled block, and every
    scheduled block holds at least one (no all-zero block is issued)."""
    _, head, rbs = tables
    for p in range(1, 11):
        nblocks, nrb, maxsteps, _ = head[p]
        nc = mi_count(p)
        assert nrb == (nc + 15) // 16
        assert nblocks == sum(rbs[(p, rb)][0] for rb in range(nrb))
        assert maxsteps == rbs[(p, 0)][0]
        covered = set()
        for rb in range(nrb):
            for s in range(rbs[(p, rb)][0]):
                cells = {(16 * rb + r, coef(s, q)) for r in range(16) for q in range(4)}
                nonzero = {(n, m) for n, m in cells if n < nc and m < nc and deg_of(n) + deg_of(m) <= p}
                assert nonzero, (p, rb, s)
                assert not (covered & nonzero)
                covered |= nonzero
        need = {(n, m) for n in range(nc) for m in range(nc) if deg_of(n) + deg_of(m) <= p}
        assert covered == need


def test_row_halves_are_complete_static_and_balanced(tables):
    _, head, rbs = tables
    for p in range(1, 11):
        nblocks, nrb, _, nloc = head[p]
        slots = {0: {0}, 1: {0}}
        for rb in range(1, nrb):
            _, half, loc = rbs[(p, rb)]
            assert half in (0, 1) and loc >= 1 and loc not in slots[half]
            slots[half].add(loc)
        assert rbs[(p, 0)][2] == 0
        assert nloc == max(len(slots[0]), len(slots[1]))
        assert all(max(v) < nloc for v in slots.values())
        # blocks issued by each half at the orders the split is balanced for
        for q in range((p + 1) // 2, p + 1):
            load = [0, 0]
            for rb in range(nrb):
                d0 = deg_of(16 * rb)
                if d0 > q:
                    continue
                n = sum(1 for s in range(rbs[(p, rb)][0]) if coef(s, 0) < mi_count(q - d0))
                for s in range(n):
                    load[(s // 2) % 2 if rb == 0 else rbs[(p, rb)][1]] += 1
            if p >= 6:
                assert max(load) <= 0.55 * sum(load) + 1, (p, q, load)
