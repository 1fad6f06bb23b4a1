"""Plain FP64 reference of the Cartesian fast multipole method of Coles & Masella (arXiv:1408.6527),
Sec. II.B-II.C, on a uniform-depth octree.

TEST INFRASTRUCTURE ONLY: nothing in the product path imports this module.  It shares no code
with the HIP library; the two meet only in the definition of the tree geometry, which is stated
once in prose here and implemented independently on each side.

The FMM is an approximation, so this module follows the method's steps in the paper's order and
notation, one operator at a time and with no blocking or fusion:

  P2M  M_n(z_A) = sum_a q_a (-1)^|n| r_a^n / n!                 (Sec. II.B, multipole equation)
       plus, for a point dipole mu_a (the delta-l -> 0 limit of the +/- q^mu pair, Sec. II.C),
       M_n += (-1)^|n| / n! * mu_a . grad(r^n) at r_a; or, on request, the pair itself: charges
       +/- |mu_a| / (2 dl) at r_a +/- dl mu_a / |mu_a|
  M2M  M_n(z + x) = sum_{k <= n} x^k / k! M_{n-k}(z)             (Sec. II.B, shifting operator)
  M2L  F_n(z_B) = sum_{|m| <= p-|n|} M_m(z_A) D_{n+m}(z_B - z_A)  (Sec. II.B, local expansion)
  L2L  F_n(z + x) = sum_{|k| <= p-|n|} x^k / k! F_{n+k}(z)        (Sec. II.B, field-tensor shift)
  L2P  d^kappa Phi(x_b) = sum_{|n| <= p-|kappa|} (x_b - z_B)^n / n! F_{n+kappa}(z_B)
       (Sec. II.B, evaluation at particles; the stray q_b of the printed formula is dropped and k
       is read as a derivative multi-index kappa)
  D_n(R) = d^n (1/|R|): the Taylor coefficients a_n = D_n / n! obey
       |n| R^2 a_n = -(2|n| - 1) sum_i R_i a_{n-e_i} - (|n| - 1) sum_i a_{n-2e_i},  a_0 = 1/|R|.

Near-field pairs are summed directly with true point dipoles and Thole damping of the
dipole-dipole tensor (Sec. III, direct component).

Tree geometry (the same rule is implemented by the library):
  * lo, hi = per-axis min and max of the positions; c = (lo + hi) * 0.5; extent = max(hi - lo).
  * L = the smallest L >= 0 with w * 2^L >= extent * (1 + 2^-20) (w = leaf width); side = w * 2^L.
  * origin o = c - side * 0.5 (per axis).  Leaf coordinate i_a = floor((x_a - o_a) / w), clamped to
    [0, 2^L - 1].  A cell at level l has coordinates (leaf coordinate) >> (L - l), width
    w_l = w * 2^(L-l) and centre o + (i + 1/2) w_l.  Only non-empty cells exist.
  * Near field: leaves A, B with Chebyshev distance max_a |i_a(A) - i_a(B)| <= ws.
  * M2L from A to B at level l >= 1: the parents of A and B are within Chebyshev distance ws at
    level l - 1 and A, B themselves are farther apart than ws.
These lists reproduce the classical well-separation criterion of Greengard and Rokhlin (Sec. III
mentions it beside the paper's own MAC); every particle pair is counted exactly once, either in
the near field or in exactly one M2L.  Octree.walk_lists gives the lists of a dual tree walk instead:
the paper's acceptance criterion, and the adaptive octree, whose leaves stop splitting at leaf_max
particles (Sec. III) and whose walk sums the particles of two terminal cells directly.
"""
from __future__ import annotations

from functools import lru_cache
from math import factorial

import numpy as np

from . import direct


# ----------------------------------------------------------------------------------------------
# Multi-index machinery (App. D).
# ----------------------------------------------------------------------------------------------

class MultiIndex:
    """All n = (nx, ny, nz) with |n| <= P, ordered by degree then lexicographically (descending nx)."""

    def __init__(self, P: int):
        self.P = P
        self.items = []
        for d in range(P + 1):
            for nx in range(d, -1, -1):
                for ny in range(d - nx, -1, -1):
                    self.items.append((nx, ny, d - nx - ny))
        self.index = {n: k for k, n in enumerate(self.items)}
        self.arr = np.array(self.items, dtype=np.int64)
        self.deg = self.arr.sum(axis=1)
        self.fact = np.array([factorial(a) * factorial(b) * factorial(c) for a, b, c in self.items], np.float64)

    def __len__(self):
        return len(self.items)

    def powers(self, r: np.ndarray) -> np.ndarray:
        """r^n for every row of r (shape (m, 3)); returns (m, len)."""
        r = np.atleast_2d(np.asarray(r, np.float64))
        out = np.ones((r.shape[0], len(self)))
        for k, (a, b, c) in enumerate(self.items):
            out[:, k] = r[:, 0] ** a * r[:, 1] ** b * r[:, 2] ** c
        return out


@lru_cache(maxsize=None)
def _mi(P: int) -> MultiIndex:
    return MultiIndex(P)


def ncoef(p: int) -> int:
    return (p + 1) * (p + 2) * (p + 3) // 6


def derivative_tensor(R: np.ndarray, P: int) -> np.ndarray:
    """D_n(R) = d^n (1/|R|) for all |n| <= P, for each row of R; returns (m, ncoef(P))."""
    mi = _mi(P)
    R = np.atleast_2d(np.asarray(R, np.float64))
    r2 = np.sum(R * R, axis=1)
    a = np.zeros((R.shape[0], len(mi)))
    a[:, 0] = 1.0 / np.sqrt(r2)
    for k, n in enumerate(mi.items):
        d = sum(n)
        if d == 0:
            continue
        acc = np.zeros(R.shape[0])
        for i in range(3):
            if n[i] >= 1:
                m1 = list(n); m1[i] -= 1
                acc -= (2 * d - 1) * R[:, i] * a[:, mi.index[tuple(m1)]]
            if n[i] >= 2:
                m2 = list(n); m2[i] -= 2
                acc -= (d - 1) * a[:, mi.index[tuple(m2)]]
        a[:, k] = acc / (d * r2)
    return a * mi.fact[None, :]


# ----------------------------------------------------------------------------------------------
# The five operators.
# ----------------------------------------------------------------------------------------------

def p2m(p, centre, X, q=None, mu=None):
    """Multipole expansion about `centre` of charges q and point dipoles mu located at X."""
    mi = _mi(p)
    r = np.atleast_2d(X) - centre[None, :]
    sign = (-1.0) ** mi.deg
    M = np.zeros(len(mi))
    if q is not None:
        M += sign / mi.fact * (np.asarray(q)[:, None] * mi.powers(r)).sum(axis=0)
    if mu is not None:
        mu = np.atleast_2d(mu)
        for k, n in enumerate(mi.items):
            acc = 0.0
            for j in range(3):
                if n[j] >= 1:
                    m = list(n); m[j] -= 1
                    e = tuple(m)
                    acc += n[j] * np.sum(mu[:, j] * r[:, 0] ** e[0] * r[:, 1] ** e[1] * r[:, 2] ** e[2])
            M[k] += sign[k] / mi.fact[k] * acc
    return M


def p2m_pair(p, centre, X, mu, dl):
    """Multipole expansion about `centre` of point dipoles mu at X, each taken as the pair of
    charges +/- q^mu at X +/- delta-l of Sec. II.C: mu = 2 |q^mu| delta-l with |delta-l| = dl along
    mu, so q^mu = |mu| / (2 dl) at X + dl mu/|mu| and -q^mu at X - dl mu/|mu|.  A zero dipole has no
    pair and adds nothing."""
    X = np.atleast_2d(np.asarray(X, np.float64))
    mu = np.atleast_2d(np.asarray(mu, np.float64))
    norm = np.linalg.norm(mu, axis=1)
    keep = norm > 0
    if not np.any(keep):
        return np.zeros(ncoef(p))
    u = mu[keep] / norm[keep, None]
    qmu = norm[keep] / (2.0 * dl)
    Xpm = np.concatenate([X[keep] + dl * u, X[keep] - dl * u])
    return p2m(p, centre, Xpm, np.concatenate([qmu, -qmu]))


@lru_cache(maxsize=None)
def _shift_tables(p: int):
    """Index triples for the two shifts: M2M uses (n, k, n-k) with k <= n componentwise; L2L uses
    (n, k, n+k) with |n| + |k| <= p."""
    mi = _mi(p)
    up, down = [], []
    for a, n in enumerate(mi.items):
        for b, k in enumerate(mi.items):
            if k[0] <= n[0] and k[1] <= n[1] and k[2] <= n[2]:
                up.append((a, b, mi.index[(n[0] - k[0], n[1] - k[1], n[2] - k[2])]))
            if sum(n) + sum(k) <= p:
                down.append((a, b, mi.index[(n[0] + k[0], n[1] + k[1], n[2] + k[2])]))
    return np.array(up, np.int64), np.array(down, np.int64)


def m2m(p, M_child, x):
    """M_n(z + x) = sum_{k <= n} x^k / k! M_{n-k}(z); x = new centre - old centre."""
    mi = _mi(p)
    xp = mi.powers(x)[0] / mi.fact
    up, _ = _shift_tables(p)
    out = np.zeros(len(mi))
    np.add.at(out, up[:, 0], xp[up[:, 1]] * M_child[up[:, 2]])
    return out


def m2l_matrix(p: int):
    """Gather table nm[n, m] = index of n + m in the order-2p set, or -1 when |n| + |m| > p."""
    mi = _mi(p)
    mi2 = _mi(2 * p)
    nm = -np.ones((len(mi), len(mi)), dtype=np.int64)
    for a, n in enumerate(mi.items):
        for b, m in enumerate(mi.items):
            if sum(n) + sum(m) <= p:
                nm[a, b] = mi2.index[(n[0] + m[0], n[1] + m[1], n[2] + m[2])]
    return nm


def m2l(p, M_src, R, nm=None, orders=None):
    """F_n(z_B) = sum_{|m| <= q - |n|} M_m(z_A) D_{n+m}(z_B - z_A) for a batch of pairs, with the
    truncation order q = p, or q = orders[k] for pair k when given (q <= p; F_n = 0 for |n| > q).

    M_src: (k, ncoef) source multipoles; R: (k, 3) = z_B - z_A.  Returns (k, ncoef).
    """
    if nm is None:
        nm = m2l_matrix(p)
    D = derivative_tensor(R, p)  # only |n + m| <= p is ever used
    mask = nm >= 0
    idx = np.where(mask, nm, 0)
    # restrict the order-2p index to order p: indices of degree <= p coincide in both orderings
    K = np.where(mask[None], D[:, idx], 0.0)
    if orders is not None:
        deg = np.array([sum(t) for t in _mi(p).items])
        keep = (deg[None, :, None] + deg[None, None, :]) <= np.asarray(orders)[:, None, None]
        K = np.where(keep, K, 0.0)
    return np.einsum("knm,km->kn", K, M_src)


def offset_order(d, p, ws, slack):
    """Truncation order of the M2L at the integer cell offset d (an extension of the fixed-order
    scheme, not in the paper): the smallest q whose bound on the relative truncation error at this
    offset, (rho_d)^(q+1) with rho_d = sqrt(3) / |d| (two cells of unit edge, radius sqrt(3)/2 each,
    centres |d| apart), does not exceed that of the nearest offsets at order p, (sqrt(3)/(ws+1))^(p+1);
    then raised by slack and capped at p.  Compared exactly in integers:
        3^(q+1) (ws+1)^(2(p+1)) <= 3^(p+1) |d|^(2(q+1)).
    slack < 0 means the fixed order p."""
    if slack < 0:
        return p
    r2 = int(d[0]) ** 2 + int(d[1]) ** 2 + int(d[2]) ** 2
    lhs_base = (ws + 1) ** (2 * (p + 1))
    q = 0
    while q < p and 3 ** (q + 1) * lhs_base > 3 ** (p + 1) * r2 ** (q + 1):
        q += 1
    return min(p, q + slack)


def l2l(p, F_parent, x):
    """F_n(z + x) = sum_{|k| <= p - |n|} x^k / k! F_{n+k}(z); x = child centre - parent centre."""
    mi = _mi(p)
    xp = mi.powers(x)[0] / mi.fact
    _, down = _shift_tables(p)
    out = np.zeros(len(mi))
    np.add.at(out, down[:, 0], xp[down[:, 1]] * F_parent[down[:, 2]])
    return out


def l2p(p, F, centre, X):
    """Potential, field and field gradient at X from the local expansion F about centre.

    phi = sum_n r^n/n! F_n;  E_c = -sum_{|n| <= p-1} r^n/n! F_{n+e_c};
    G[a, b] = d_a E_b = -sum_{|n| <= p-2} r^n/n! F_{n+e_a+e_b}.
    """
    mi = _mi(p)
    r = np.atleast_2d(X) - centre[None, :]
    w = mi.powers(r) / mi.fact[None, :]
    phi = w @ F
    E = np.zeros((r.shape[0], 3))
    G = np.zeros((r.shape[0], 3, 3))
    for k, n in enumerate(mi.items):
        d = sum(n)
        for c in range(3):
            if d <= p - 1:
                nc = list(n); nc[c] += 1
                E[:, c] -= w[:, k] * F[mi.index[tuple(nc)]]
            for c2 in range(3):
                if d <= p - 2:
                    nc = list(n); nc[c] += 1; nc[c2] += 1
                    G[:, c, c2] -= w[:, k] * F[mi.index[tuple(nc)]]
    return phi, E, G


# ----------------------------------------------------------------------------------------------
# Tree geometry and interaction lists.
# ----------------------------------------------------------------------------------------------

class Octree:
    def __init__(self, X: np.ndarray, leaf_width: float, ws: int = 1):
        X = np.asarray(X, np.float64)
        self.ws = ws
        self.w = float(leaf_width)
        lo = X.min(axis=0); hi = X.max(axis=0)
        c = (lo + hi) * 0.5
        extent = float(np.max(hi - lo))
        L = 0
        while self.w * 2.0**L < extent * (1.0 + 2.0**-20):
            L += 1
        self.L = L
        self.side = self.w * 2.0**L
        self.origin = c - self.side * 0.5
        coords = np.floor((X - self.origin[None, :]) / self.w).astype(np.int64)
        self.leaf_coord = np.clip(coords, 0, 2**L - 1)
        self.leaves = {}
        for i, cc in enumerate(map(tuple, self.leaf_coord)):
            self.leaves.setdefault(cc, []).append(i)
        self.cells = []  # per level: sorted list of coordinate tuples
        for l in range(L + 1):
            sh = L - l
            self.cells.append(sorted({(a >> sh, b >> sh, d >> sh) for (a, b, d) in self.leaves}))
        # particles of every cell of every level (the leaves' lists at level L)
        self._mem = [dict() for _ in range(L + 1)]
        self._mem[L] = self.leaves
        for cc, idx in self.leaves.items():
            for l in range(L):
                sh = L - l
                self._mem[l].setdefault((cc[0] >> sh, cc[1] >> sh, cc[2] >> sh), []).extend(idx)

    def members(self, l, c):
        """Indices of the particles in cell c of level l."""
        return self._mem[l][c]

    def width(self, l):
        return self.w * 2.0 ** (self.L - l)

    def centre(self, l, cc):
        return self.origin + (np.asarray(cc, np.float64) + 0.5) * self.width(l)

    @staticmethod
    def cheb(a, b):
        return max(abs(a[0] - b[0]), abs(a[1] - b[1]), abs(a[2] - b[2]))

    def m2l_pairs(self, l):
        """(target B, source A) pairs at level l."""
        out = []
        if l == 0:
            return out
        cells = self.cells[l]
        for B in cells:
            pB = (B[0] >> 1, B[1] >> 1, B[2] >> 1)
            for A in cells:
                pA = (A[0] >> 1, A[1] >> 1, A[2] >> 1)
                if self.cheb(pA, pB) <= self.ws and self.cheb(A, B) > self.ws:
                    out.append((B, A))
        return out

    def near_pairs(self):
        leaves = self.cells[self.L]
        return [(B, A) for B in leaves for A in leaves if self.cheb(A, B) <= self.ws]

    @staticmethod
    def _length(d):
        """|d| of the rows of d, summed in the order x, y, z in float64 (np.sqrt is correctly
        rounded): the acceptance decisions below are integer results decided in floating point, so
        the arithmetic is spelled out."""
        d = np.atleast_2d(np.asarray(d, np.float64))
        return np.sqrt(d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1] + d[:, 2] * d[:, 2])

    def enclosing_radii(self, X):
        """r_enc of every cell: the largest distance from the cell's centre (its expansion centre) to
        one of its particles (Sec. III, the cell record's enclosing radius)."""
        X = np.asarray(X, np.float64)
        renc = [dict() for _ in range(self.L + 1)]
        for cc, idx in self.leaves.items():
            for l in range(self.L + 1):
                sh = self.L - l
                c = (cc[0] >> sh, cc[1] >> sh, cc[2] >> sh)
                r = float(np.max(self._length(X[idx] - self.centre(l, c)[None, :])))
                renc[l][c] = max(renc[l].get(c, 0.0), r)
        return renc

    def refined_cells(self, leaf_max):
        """The split cells of the adaptive octree, per level: the octree form of the paper's adaptive
        tree, whose recursion stops once a cell holds no more than N_bucket particles (Sec. III).

        A cell of a level below L is split when it holds more than leaf_max particles.  The tree is
        then 2:1 balanced over the full octree, empty cells included (a reading: the paper's kd-tree
        needs no balance): a cell of level l whose closed box touches the box of a split cell of
        level l + 1 is split as well, until nothing changes, so two leaves that touch differ by at
        most one level.  A cell that is not split, and every cell below it, is terminal; the top-most
        terminal cells are the adaptive leaves."""
        R = [set() for _ in range(self.L + 1)]
        for l in range(self.L):
            for c in self.cells[l]:
                if len(self._mem[l][c]) > leaf_max:
                    R[l].add(c)
        changed = True
        while changed:
            changed = False
            for l in range(self.L - 1, -1, -1):
                if not R[l + 1]:
                    continue
                fine = np.array(sorted(R[l + 1]), np.int64)
                for B in self.cells[l]:
                    if B in R[l]:
                        continue
                    # B spans [2 B, 2 B + 2] in units of the finer level, a cell c spans [c, c + 1]
                    lo = 2 * np.asarray(B, np.int64)
                    if np.any(np.all((fine + 1 >= lo) & (fine <= lo + 2), axis=1)):
                        R[l].add(B)
                        changed = True
        return R

    def walk_lists(self, X, theta=None, ndirect=0, leaf_direct=False, leaf_max=0):
        """Interaction lists of a dual tree walk over pairs of cells of one level (Sec. III), from the
        root paired with itself, so that every ordered pair of particles is counted once.

        Acceptance for M2L, of a pair of distinct cells that hold at least ndirect particles together
        (and, with leaf_direct, are not both terminal: the paper's direct interaction of leaf pairs):
          * theta None: the cells are farther apart than ws (Chebyshev distance of their coordinates
            > ws), the well-separation rule;
          * theta: the paper's multipole acceptance criterion (eq:mac), theta |z_A - z_B| > r_A + r_B
            with z the cell centres and r the enclosing radii, for cells that are not adjacent
            (Chebyshev distance >= 2: Thole-damped pairs, closer than a leaf edge, stay direct).
        A pair that is not accepted goes to the direct part when both cells are terminal, else it is
        split into the pairs of the two cells' children.  Terminal cells: the leaf level L; with
        leaf_max > 0 also every cell that the adaptive rule (refined_cells) does not split, and the
        cells below it.  Below ndirect particles the children hold fewer still, so all of a pair's
        descendants are direct.
        Returns (m2l, near): m2l[l] the (B, A) pairs accepted at level l; near the (l, B, A) pairs of
        cells whose particles are summed directly."""
        renc = self.enclosing_radii(X) if theta is not None else None
        R = self.refined_cells(leaf_max) if leaf_max > 0 else None

        def terminal(l, c):
            return l == self.L or (R is not None and c not in R[l])

        kids = [dict() for _ in range(self.L + 1)]
        for l in range(1, self.L + 1):
            for c in self.cells[l]:
                kids[l - 1].setdefault((c[0] >> 1, c[1] >> 1, c[2] >> 1), []).append(c)
        m2l = [[] for _ in range(self.L + 1)]
        near = []
        stack = [(0, (0, 0, 0), (0, 0, 0))]
        while stack:
            l, B, A = stack.pop()
            tB, tA = terminal(l, B), terminal(l, A)
            accept = False
            if (A != B and len(self._mem[l][B]) + len(self._mem[l][A]) >= ndirect
                    and not (leaf_direct and tB and tA)):
                if theta is None:
                    accept = self.cheb(A, B) > self.ws
                elif self.cheb(A, B) >= 2:
                    dist = float(self._length((np.asarray(B, np.float64) - np.asarray(A, np.float64)) * self.width(l))[0])
                    accept = theta * dist > renc[l][B] + renc[l][A]
            if accept:
                m2l[l].append((B, A))
            elif tB and tA:
                near.append((l, B, A))
            else:
                for b in kids[l][B]:
                    for a in kids[l][A]:
                        stack.append((l + 1, b, a))
        for lst in m2l:
            lst.sort()
        near.sort()
        return m2l, near

    def mac_lists(self, X, theta, ndirect=0, leaf_direct=False):
        """The lists of the paper's multipole acceptance criterion on this uniform-depth octree
        (walk_lists with theta): (m2l, near) with near the (B, A) leaf pairs summed directly."""
        m2l, near = self.walk_lists(X, theta, ndirect, leaf_direct)
        return m2l, sorted((B, A) for _, B, A in near)


# ----------------------------------------------------------------------------------------------
# Field evaluation.
# ----------------------------------------------------------------------------------------------

def fmm_fields(X, q, mu, alpha, thole_a, p, leaf_width, ws=1, want_grad=True, order_slack=-1,
               pair_dl=0.0, excl=None, theta=None, ndirect=0, leaf_direct=False, leaf_max=0):
    """FMM fields of charges q and point dipoles mu at every particle.

    pair_dl > 0 builds the multipoles of the dipoles from their +/- q^mu pairs (Sec. II.C, p2m_pair)
    instead of the point-dipole limit; the near field keeps the point dipoles.
    excl: excluded pairs (direct.exclusion_matrix); the exact terms of each excluded pair are taken
    off the result, wherever the pair was counted (near field, or M2L to within its truncation).
    theta: the interaction lists of the paper's dual tree walk with its acceptance criterion
    (Octree.walk_lists, with ndirect and leaf_direct) instead of the well-separation lists; the M2L
    then runs at order p.
    leaf_max > 0: the adaptive octree (Octree.refined_cells): the walk stops at pairs of terminal
    cells, whose particles are summed directly, with the well-separation rule of ws (theta None) or
    the acceptance criterion; every M2L at order p.  The expansions of the cells below an adaptive
    leaf (P2M at the leaf level, M2M, L2L and L2P there) are the exact translations of the leaf's
    own, so they serve the interactions with finer neighbours at the finer levels.

    Returns a dict with
      phi  total potential (undamped),
      E_u  total field with undamped dipole part (what acts on charges),
      E_d  total field with Thole-damped dipole part (what acts on dipoles),
      G_d  d_a (E_d)_b,
    and the tree used.  q or mu may be None.  Far field is undamped; damping lives in the near
    field (requires the damping radius not to exceed the near-field range).
    """
    X = np.asarray(X, np.float64)
    n = X.shape[0]
    alpha = np.asarray(alpha, np.float64)
    tree = Octree(X, leaf_width, ws)
    L = tree.L
    nc = ncoef(p)
    qq = np.zeros(n) if q is None else np.asarray(q, np.float64)
    mm = np.zeros((n, 3)) if mu is None else np.asarray(mu, np.float64)

    # upward pass
    M = [dict() for _ in range(L + 1)]
    for cc, idx in tree.leaves.items():
        if pair_dl > 0:
            M[L][cc] = p2m(p, tree.centre(L, cc), X[idx], qq[idx]) + p2m_pair(p, tree.centre(L, cc), X[idx],
                                                                                 mm[idx], pair_dl)
        else:
            M[L][cc] = p2m(p, tree.centre(L, cc), X[idx], qq[idx], mm[idx])
    for l in range(L, 0, -1):
        for cc, Mc in M[l].items():
            par = (cc[0] >> 1, cc[1] >> 1, cc[2] >> 1)
            x = tree.centre(l - 1, par) - tree.centre(l, cc)
            M[l - 1][par] = M[l - 1].get(par, np.zeros(nc)) + m2m(p, Mc, x)

    # transfer
    nm = m2l_matrix(p)
    F = [dict() for _ in range(L + 1)]
    walk = None
    if theta is not None or leaf_max > 0:
        walk = tree.walk_lists(X, theta, ndirect, leaf_direct, leaf_max)
    for l in range(1, L + 1):
        pairs = walk[0][l] if walk is not None else tree.m2l_pairs(l)
        for s in range(0, len(pairs), 256):
            chunk = pairs[s:s + 256]
            R = np.array([tree.centre(l, B) - tree.centre(l, A) for B, A in chunk])
            Ms = np.array([M[l][A] for B, A in chunk])
            orders = None
            if order_slack >= 0:
                orders = [offset_order((B[0] - A[0], B[1] - A[1], B[2] - A[2]), p, ws, order_slack)
                          for B, A in chunk]
            Fk = m2l(p, Ms, R, nm, orders)
            for (B, A), f in zip(chunk, Fk):
                F[l][B] = F[l].get(B, np.zeros(nc)) + f

    # downward pass
    for l in range(1, L + 1):
        for cc in tree.cells[l]:
            par = (cc[0] >> 1, cc[1] >> 1, cc[2] >> 1)
            if par in F[l - 1]:
                x = tree.centre(l, cc) - tree.centre(l - 1, par)
                F[l][cc] = F[l].get(cc, np.zeros(nc)) + l2l(p, F[l - 1][par], x)

    phi = np.zeros(n); E_far = np.zeros((n, 3)); G_far = np.zeros((n, 3, 3))
    for cc, idx in tree.leaves.items():
        if cc in F[L]:
            ph, E, G = l2p(p, F[L][cc], tree.centre(L, cc), X[idx])
            phi[idx] += ph; E_far[idx] += E; G_far[idx] += G

    # near field, direct with point dipoles
    E_u = E_far.copy(); E_d = E_far.copy(); G_d = G_far.copy()
    for l, B, A in (walk[1] if walk is not None else [(L, B, A) for B, A in tree.near_pairs()]):
        ib = tree.members(l, B); ia = tree.members(l, A)
        for i in ib:
            src = [j for j in ia if j != i]
            if not src:
                continue
            src = np.array(src)
            rv = X[i] - X[src]
            g, grad, H, T3 = direct.hessian_and_third(rv)
            s = direct.thole_radius(alpha[i], alpha[src], thole_a)
            _, _, Hd, T3d = direct.hessian_and_third(rv, s)
            # charges: phi = q g, E = -q grad g, d_a E_b = -q H_ab
            phi[i] += np.sum(qq[src] * g)
            Eq = -np.sum(qq[src][:, None] * grad, axis=0)
            Gq = -np.sum(qq[src][:, None, None] * H, axis=0)
            # dipoles: phi = -mu.grad g, E = H mu (damped for dipole targets), d_a E_b = T3_abc mu_c
            phi[i] -= np.sum(mm[src] * grad)
            E_u[i] += Eq + np.einsum("jab,jb->a", H, mm[src])
            E_d[i] += Eq + np.einsum("jab,jb->a", Hd, mm[src])
            if want_grad:
                G_d[i] += Gq + np.einsum("jabc,jc->ab", T3d, mm[src])
    if excl is not None and len(excl):
        e = np.asarray(excl, np.int64).reshape(-1, 2)
        for i, j in np.concatenate([e, e[:, ::-1]]):
            rv = (X[i] - X[j])[None, :]
            g, grad, H, T3 = direct.hessian_and_third(rv)
            s = direct.thole_radius(alpha[i], alpha[j:j + 1], thole_a)
            _, _, Hd, T3d = direct.hessian_and_third(rv, s)
            phi[i] -= qq[j] * g[0] - grad[0] @ mm[j]
            Eq = -qq[j] * grad[0]
            E_u[i] -= Eq + H[0] @ mm[j]
            E_d[i] -= Eq + Hd[0] @ mm[j]
            if want_grad:
                G_d[i] -= -qq[j] * H[0] + T3d[0] @ mm[j]
    return dict(phi=phi, E_u=E_u, E_d=E_d, G_d=G_d, tree=tree)
