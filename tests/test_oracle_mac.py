"""Pins of the oracle's acceptance-criterion walk (oracle.fmm.Octree.mac_lists, Sec. III eq. mac)
and of its FMM on those lists, against what the mathematics fixes:

* every ordered pair of distinct particles is covered exactly once (brute force over the pairs):
  by the M2L of one accepted pair of ancestor cells, or by the near field of their leaves;
* theta = 0 accepts nothing, so the FMM is the direct sum (closed form of the pair fields);
* what is accepted obeys the rules: not adjacent, at least ndirect particles together, no leaf pair
  with leaf_direct, and the criterion itself with the radii found by brute force;
* Newton's third law: the total force of an FMM evaluation vanishes to rounding (the lists are
  symmetric and every M2L has the same truncation |n| + |m| <= p), for charges and dipoles;
* the error against the direct sum falls with p at fixed theta and with theta at fixed p.
"""
import numpy as np
import pytest

from oracle import direct as D
from oracle import fmm as FM


def _cluster(n, seed, side=18.0):
    rng = np.random.default_rng(seed)
    X = rng.uniform(0, side, (n, 3))
    # a denser clump in one corner, so cells of very different occupancy meet
    X[: n // 3] = rng.uniform(0, side / 4, (n // 3, 3))
    q = rng.normal(0, 0.6, n)
    q -= q.mean()
    mu = rng.normal(0, 0.3, (n, 3))
    a = rng.uniform(0.5, 1.5, n)
    return X, q, mu, a


def _members(tree, l, c):
    sh = tree.L - l
    return [i for i, cc in enumerate(map(tuple, tree.leaf_coord)) if (cc[0] >> sh, cc[1] >> sh, cc[2] >> sh) == c]


@pytest.mark.parametrize("theta,nd,ld", [(0.3, 0, False), (0.5, 0, False), (0.99, 0, False), (0.5, 24, True),
                                         (0.7, 20, False)])
def test_walk_covers_every_pair_once(theta, nd, ld):
    X, _, _, _ = _cluster(140, 1)
    tree = FM.Octree(X, 2.0, 1)
    m2l, near = tree.mac_lists(X, theta, nd, ld)
    n = len(X)
    C = np.zeros((n, n), np.int64)
    for l in range(tree.L + 1):
        for B, A in m2l[l]:
            C[np.ix_(_members(tree, l, B), _members(tree, l, A))] += 1
    for B, A in near:
        C[np.ix_(tree.leaves[B], tree.leaves[A])] += 1
    np.fill_diagonal(C, C.diagonal() - 1)  # each particle meets itself once, in its own leaf pair
    off = ~np.eye(n, dtype=bool)
    assert C[off].min() == 1 and C[off].max() == 1
    assert np.all(C.diagonal() == 0)
    assert sum(len(x) for x in m2l) > 0


@pytest.mark.parametrize("theta,nd,ld", [(0.5, 0, False), (0.7, 30, True), (0.99, 0, True)])
def test_accepted_pairs_obey_the_rules(theta, nd, ld):
    X, _, _, _ = _cluster(160, 2)
    tree = FM.Octree(X, 2.0, 1)
    m2l, near = tree.mac_lists(X, theta, nd, ld)
    for l in range(tree.L + 1):
        for B, A in m2l[l]:
            ib, ia = _members(tree, l, B), _members(tree, l, A)
            assert A != B and tree.cheb(A, B) >= 2 and len(ib) + len(ia) >= nd
            assert not (ld and l == tree.L)
            zb, za = tree.centre(l, B), tree.centre(l, A)
            rb = max(np.sqrt(np.sum((X[i] - zb) ** 2)) for i in ib)
            ra = max(np.sqrt(np.sum((X[i] - za) ** 2)) for i in ia)
            assert theta * np.sqrt(np.sum((zb - za) ** 2)) > rb + ra - 1e-9
    for B, A in near:
        assert B in tree.leaves and A in tree.leaves
    # the lists are symmetric
    for l in range(tree.L + 1):
        assert sorted(m2l[l]) == sorted((A, B) for B, A in m2l[l])
    assert sorted(near) == sorted((A, B) for B, A in near)


def test_theta_zero_is_the_direct_sum():
    X, q, mu, a = _cluster(120, 3)
    ref = FM.fmm_fields(X, q, mu, a, 2.0, 4, 2.6, 1, theta=0.0)
    tree = ref["tree"]
    assert tree.L >= 2 and sum(len(x) for x in tree.mac_lists(X, 0.0)[0]) == 0
    pq, Eq, Gq = D.charge_fields(X, q)
    pm, Eu, Ed, Gd = D.dipole_fields(X, mu, a, 2.0)
    for got, want in ((ref["phi"], pq + pm), (ref["E_u"], Eq + Eu), (ref["E_d"], Eq + Ed), (ref["G_d"], Gq + Gd)):
        assert np.abs(got - want).max() < 1e-12 * np.abs(want).max()


@pytest.mark.parametrize("theta,nd,ld", [(None, 0, False), (0.5, 0, False), (0.7, 24, True)])
def test_total_force_vanishes(theta, nd, ld):
    """F_i = q_i E_i + (mu_i . grad) E_i with undamped fields: the sum over all particles is zero to
    rounding, far field included."""
    X, q, mu, a = _cluster(200, 4)
    r = FM.fmm_fields(X, q, mu, a, 0.0, 5, 2.0, 1, theta=theta, ndirect=nd, leaf_direct=ld)
    if theta is not None:
        assert sum(len(x) for x in r["tree"].mac_lists(X, theta, nd, ld)[0]) > 0
    F = q[:, None] * r["E_u"] + np.einsum("ia,iab->ib", mu, r["G_d"])
    assert np.abs(F.sum(axis=0)).max() < 1e-13 * np.abs(F).sum()


def test_error_falls_with_order_and_theta():
    X, q, mu, a = _cluster(300, 5, side=24.0)
    pq, Eq, _ = D.charge_fields(X, q)
    pm, Eu, _, _ = D.dipole_fields(X, mu, a, 2.0)
    E = Eq + Eu

    def err(theta, p):
        r = FM.fmm_fields(X, q, mu, a, 2.0, p, 2.6, 1, want_grad=False, theta=theta)
        return float(np.median(np.linalg.norm(r["E_u"] - E, axis=1) / np.linalg.norm(E, axis=1)))

    by_p = [err(0.6, p) for p in (2, 4, 6)]
    by_theta = [err(t, 4) for t in (0.9, 0.6, 0.4)]
    assert by_p[0] > 3 * by_p[1] > 9 * by_p[2]
    assert by_theta[0] > by_theta[1] > by_theta[2]
