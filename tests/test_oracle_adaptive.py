"""Pins of the oracle's adaptive octree (oracle.fmm.Octree.refined_cells and walk_lists with
leaf_max; the octree form of the paper's adaptive tree, whose recursion stops at N_bucket particles,
Sec. III) and of its FMM on those lists, against what the mathematics fixes:

* every ordered pair of distinct particles is covered exactly once (brute force over the pairs), by
  one accepted M2L of ancestor cells or by the direct sum of two terminal cells, for the
  well-separation rule (ws = 1, 2) and the acceptance criterion;
* the tree obeys its definition: leaves above the finest level hold at most leaf_max particles,
  touching leaves differ by at most one level, and every split cell is over-full or touches a split
  cell one level finer (nothing is split without a reason);
* when no cell above the finest level is a leaf, the lists are the uniform tree's (the separately
  written m2l_pairs / near_pairs, and the acceptance-criterion walk);
* a root that is a leaf makes everything direct: the FMM is the direct sum (closed form);
* Newton's third law: the total force of an evaluation vanishes to rounding (symmetric lists, one
  truncation order);
* the error against the direct sum falls with p, and stays at the uniform tree's level.
"""
import numpy as np
import pytest

from oracle import direct as D
from oracle import fmm as FM


def _clumped(n, seed, side=24.0, core=4.0, frac=0.6):
    """A dense core of frac * n particles in a cube of edge core, the rest spread over a cube of edge
    side: cells of very different occupancy on every level."""
    rng = np.random.default_rng(seed)
    nc = int(frac * n)
    X = np.vstack([rng.uniform(0, core, (nc, 3)) + (side - core) / 2, rng.uniform(0, side, (n - nc, 3))])
    q = rng.normal(0, 0.6, n)
    q -= q.mean()
    mu = rng.normal(0, 0.3, (n, 3))
    a = rng.uniform(0.5, 1.5, n)
    return X, q, mu, a


def _leaves(tree, R):
    """Top-most terminal cells (level, coordinates) of the adaptive tree."""
    out = []
    for l in range(tree.L + 1):
        for c in tree.cells[l]:
            parent_split = l == 0 or (c[0] >> 1, c[1] >> 1, c[2] >> 1) in R[l - 1]
            if parent_split and (l == tree.L or c not in R[l]):
                out.append((l, c))
    return out


def _touch(la, A, lb, B):
    """Closed boxes of cell A (level la) and cell B (level lb) intersect."""
    lf = max(la, lb)
    sa, sb = 1 << (lf - la), 1 << (lf - lb)
    return all(A[k] * sa <= (B[k] + 1) * sb and B[k] * sb <= (A[k] + 1) * sa for k in range(3))


@pytest.mark.parametrize("ws,theta,lmax,nd,ld", [(1, None, 8, 0, False), (2, None, 12, 0, False),
                                                 (1, 0.6, 10, 0, False), (1, 0.7, 10, 20, True),
                                                 (1, 0.99, 4, 0, True)])
def test_walk_covers_every_pair_once(ws, theta, lmax, nd, ld):
    X, _, _, _ = _clumped(220, 1)
    tree = FM.Octree(X, 1.2, ws)
    m2l, near = tree.walk_lists(X, theta, nd, ld, leaf_max=lmax)
    n = len(X)
    C = np.zeros((n, n), np.int64)
    for l in range(tree.L + 1):
        for B, A in m2l[l]:
            C[np.ix_(tree.members(l, B), tree.members(l, A))] += 1
    for l, B, A in near:
        C[np.ix_(tree.members(l, B), tree.members(l, A))] += 1
    np.fill_diagonal(C, C.diagonal() - 1)  # each particle meets itself once, in its own cell pair
    off = ~np.eye(n, dtype=bool)
    assert C[off].min() == 1 and C[off].max() == 1
    assert np.all(C.diagonal() == 0)
    assert sum(len(x) for x in m2l) > 0
    # direct pairs above the finest level: the adaptive leaves are in use
    assert any(l < tree.L for l, _, _ in near)
    # the lists are symmetric
    for l in range(tree.L + 1):
        assert sorted(m2l[l]) == sorted((A, B) for B, A in m2l[l])
    assert sorted(near) == sorted((l, A, B) for l, B, A in near)


@pytest.mark.parametrize("lmax", [1, 6, 20])
def test_refined_cells_obey_the_definition(lmax):
    X, _, _, _ = _clumped(400, 2)
    tree = FM.Octree(X, 0.9, 1)
    R = tree.refined_cells(lmax)
    leaves = _leaves(tree, R)
    # the leaves partition the particles
    assert sorted(i for l, c in leaves for i in tree.members(l, c)) == list(range(len(X)))
    for l, c in leaves:
        assert l == tree.L or len(tree.members(l, c)) <= lmax
    # 2:1 balance of touching leaves
    by_level = {}
    for l, c in leaves:
        by_level.setdefault(l, []).append(c)
    for la in by_level:
        for lb in by_level:
            if lb < la + 2:
                continue
            for A in by_level[la]:
                for B in by_level[lb]:
                    assert not _touch(la, A, lb, B)
    # every split cell has a reason, and its parent is split
    for l in range(tree.L):
        for c in R[l]:
            over = len(tree.members(l, c)) > lmax
            pushed = any(_touch(l, c, l + 1, f) for f in R[l + 1])
            assert over or pushed
            if l > 0:
                assert (c[0] >> 1, c[1] >> 1, c[2] >> 1) in R[l - 1]
    assert len({l for l, _ in leaves}) >= 3


def test_no_leaf_above_the_finest_level_gives_the_uniform_lists():
    """Two jittered particles in every leaf of a 6 x 6 x 6 block: every cell above the finest level
    holds at least two, so leaf_max = 1 splits them all."""
    rng = np.random.default_rng(3)
    w = 1.5
    g = np.array([(i, j, k) for i in range(6) for j in range(6) for k in range(6)], np.float64)
    X = np.vstack([(g + rng.uniform(0.1, 0.9, g.shape)) * w, (g + rng.uniform(0.1, 0.9, g.shape)) * w])
    for ws in (1, 2):
        tree = FM.Octree(X, w, ws)
        assert all(len(tree.members(l, c)) >= 2 for l in range(tree.L) for c in tree.cells[l])
        m2l, near = tree.walk_lists(X, None, leaf_max=1)
        for l in range(tree.L + 1):
            assert m2l[l] == sorted(tree.m2l_pairs(l))
        assert near == sorted((tree.L, B, A) for B, A in tree.near_pairs())
    tree = FM.Octree(X, w, 1)
    m2l, near = tree.walk_lists(X, 0.6, 10, True, leaf_max=1)
    m2l_u, near_u = tree.mac_lists(X, 0.6, 10, True)
    assert m2l == m2l_u and [(B, A) for _, B, A in near] == near_u


def test_root_leaf_is_the_direct_sum():
    X, q, mu, a = _clumped(150, 4)
    ref = FM.fmm_fields(X, q, mu, a, 2.0, 4, 1.2, 1, leaf_max=len(X))
    tree = ref["tree"]
    m2l, near = tree.walk_lists(X, None, leaf_max=len(X))
    assert tree.L >= 3 and sum(len(x) for x in m2l) == 0 and near == [(0, (0, 0, 0), (0, 0, 0))]
    pq, Eq, Gq = D.charge_fields(X, q)
    pm, Eu, Ed, Gd = D.dipole_fields(X, mu, a, 2.0)
    for got, want in ((ref["phi"], pq + pm), (ref["E_u"], Eq + Eu), (ref["E_d"], Eq + Ed), (ref["G_d"], Gq + Gd)):
        assert np.abs(got - want).max() < 1e-12 * np.abs(want).max()


@pytest.mark.parametrize("ws,theta,ld", [(1, None, False), (2, None, False), (1, 0.6, True)])
def test_total_force_vanishes(ws, theta, ld):
    """F_i = q_i E_i + (mu_i . grad) E_i with undamped fields sums to zero to rounding."""
    X, q, mu, a = _clumped(240, 5)
    r = FM.fmm_fields(X, q, mu, a, 0.0, 5, 1.2, ws, theta=theta, leaf_direct=ld, leaf_max=10)
    m2l, near = r["tree"].walk_lists(X, theta, 0, ld, leaf_max=10)
    assert sum(len(x) for x in m2l) > 0 and any(l < r["tree"].L for l, _, _ in near)
    F = q[:, None] * r["E_u"] + np.einsum("ia,iab->ib", mu, r["G_d"])
    assert np.abs(F.sum(axis=0)).max() < 1e-13 * np.abs(F).sum()


def test_error_falls_with_order_and_matches_the_uniform_tree():
    X, q, mu, a = _clumped(360, 6, side=30.0)
    pq, Eq, _ = D.charge_fields(X, q)
    pm, Eu, _, _ = D.dipole_fields(X, mu, a, 2.0)
    E = Eq + Eu

    def err(p, lmax):
        r = FM.fmm_fields(X, q, mu, a, 2.0, p, 1.2, 1, want_grad=False, leaf_max=lmax)
        return float(np.median(np.linalg.norm(r["E_u"] - E, axis=1) / np.linalg.norm(E, axis=1)))

    ad = [err(p, 12) for p in (2, 4, 6)]
    un = err(6, 0)
    assert ad[0] > 2.5 * ad[1] > 6 * ad[2]
    assert ad[2] < 3 * un
    tree = FM.Octree(X, 1.2, 1)
    n_ad = sum(len(x) for x in tree.walk_lists(X, None, leaf_max=12)[0])
    n_un = sum(len(tree.m2l_pairs(l)) for l in range(tree.L + 1))
    assert n_ad < n_un
