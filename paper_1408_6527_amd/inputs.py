"""Seeded synthetic particle sets (positions, charges, polarisabilities).

This module only draws inputs: it holds none of the electrostatics.  The same generators feed the
HIP path, the CPU oracle, the tests and the benchmark.

The workloads stand in for the paper's protein systems (Sec. IV.B-IV.C: a protein complex and
subsets of the HIV-1 capsid, which are not available here) by shape, size and density:

* ``uniform_cube``   1,000 particles in a 20 Angstrom cube, charges +1/-1 alternating,
                     alpha ~ U[0.5, 2.0] Angstrom^3.
* ``globular``       clumped particles (clumps of 20 drawn from N(c, 3^2 I)) in a ball at
                     0.1 particles/Angstrom^3, charges N(0, 0.4) shifted to net zero,
                     alpha ~ U[0.2, 2.0]: a globular protein.
* ``hexamer_shell``  six rotated copies of a 20,000-particle globular blob (radius 35) on a ring
                     of radius 45 plus 40,000 uncharged solvent sites (alpha = 1.5) uniform in a
                     spherical shell at 0.03 per Angstrom^3: a capsid hexamer in solvent.
* ``scaling``        half uniform in a cube and half globular at 0.1 per Angstrom^3.
* ``sphere``         the paper's own random sphere (Sec. IV.A): 4,096 points in a 45 Angstrom ball,
                     minimum separation 2 Angstrom, +/-1 e in equal numbers, independent +/-1 e field
                     charges qE, one alpha for all.

Every protein-like set keeps a minimum separation r_min = 1.0 Angstrom (rejection on a cell grid);
the paper's 2 Angstrom, used by its sphere test, cannot be packed at protein density.
Seeds: numpy ``SeedSequence([14086527, k])`` for workload k, spawned into independent streams for
positions, charges and polarisabilities.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

R_MIN = 1.0
SEED_BASE = 14086527


@dataclass
class ParticleSet:
    name: str
    pos: np.ndarray      # (n, 3) float64, Angstrom
    q: np.ndarray        # (n,)   float64, e
    alpha: np.ndarray    # (n,)   float64, Angstrom^3
    qE: np.ndarray | None = None  # (n,) charges of the polarising field where they differ from q

    @property
    def n(self) -> int:
        return self.pos.shape[0]


def _streams(k: int, extra: int = 0):
    ss = np.random.SeedSequence([SEED_BASE, k, extra])
    return [np.random.default_rng(s) for s in ss.spawn(3)]


class _Exclusion:
    """Accepted points on a dense grid whose cell diagonal is below r_min (one point per cell)."""

    def __init__(self, lo, hi, r_min=R_MIN):
        self.r2 = r_min * r_min
        self.a = r_min / math.sqrt(3.0) * (1.0 - 1e-9)
        self.pad = 3
        self.lo = np.asarray(lo, np.float64)
        dims = np.ceil((np.asarray(hi, np.float64) - self.lo) / self.a).astype(np.int64) + 2 * self.pad + 1
        self.dims = dims
        self.grid = np.full(int(np.prod(dims)), -1, dtype=np.int32)
        self.pts = np.zeros((0, 3))
        self._buf = []
        self.count = 0
        off = np.arange(-2, 3)
        ox, oy, oz = np.meshgrid(off, off, off, indexing="ij")
        self.offsets = (ox.ravel() * dims[1] * dims[2] + oy.ravel() * dims[2] + oz.ravel())

    def _cells(self, x):
        c = np.floor((x - self.lo) / self.a).astype(np.int64) + self.pad
        return (c[:, 0] * self.dims[1] + c[:, 1]) * self.dims[2] + c[:, 2]

    def _points(self):
        if self._buf:
            self.pts = np.concatenate([self.pts] + self._buf)
            self._buf = []
        return self.pts

    def try_add(self, x):
        """Accept the rows of x that keep r_min to all accepted points and to earlier rows."""
        from scipy.spatial import cKDTree

        x = np.asarray(x, np.float64)
        if x.shape[0] == 0:
            return np.zeros(0, bool)
        cells = self._cells(x)
        nb = self.grid[cells[:, None] + self.offsets[None, :]]
        ok = np.ones(x.shape[0], bool)
        has = nb >= 0
        if np.any(has):
            pts = self._points()
            rows, cols = np.nonzero(has)
            d = x[rows] - pts[nb[rows, cols]]
            bad = np.sum(d * d, axis=1) < self.r2
            ok[rows[bad]] = False
        idx = np.nonzero(ok)[0]
        if idx.size > 1:
            pairs = cKDTree(x[idx]).query_pairs(math.sqrt(self.r2) * (1 - 1e-12), output_type="ndarray")
            if pairs.size:
                later = np.maximum(pairs[:, 0], pairs[:, 1])
                ok[idx[np.unique(later)]] = False
        acc = np.nonzero(ok)[0]
        self.grid[cells[acc]] = np.arange(self.count, self.count + acc.size, dtype=np.int32)
        self._buf.append(x[acc])
        self.count += acc.size
        return ok


def _uniform_ball(rng, n, R):
    v = rng.normal(size=(n, 3))
    v /= np.linalg.norm(v, axis=1)[:, None]
    return v * (R * np.cbrt(rng.uniform(size=n)))[:, None]


def _fill(excl, n, draw, batch=8192):
    """Draw batches from draw(m) -> (points, tag), keep the accepted ones, until n are kept."""
    out, tags = [], []
    have = 0
    while have < n:
        m = min(batch, n - have)
        x, t = draw(m)
        ok = excl.try_add(x)
        out.append(x[ok]); tags.append(t[ok])
        have += int(ok.sum())
    return np.concatenate(out)[:n], np.concatenate(tags)[:n]


def _clumped(excl, rng, n, R, centre, rot=None, sigma=3.0, per_clump=20, clump_centres=None):
    """Clumps of ~per_clump particles from N(c, sigma^2 I) with c uniform in a ball of radius R;
    draws outside the ball or within r_min of an accepted particle are drawn again."""
    if clump_centres is None:
        clump_centres = _uniform_ball(rng, math.ceil(n / per_clump), R)
    nc = clump_centres.shape[0]
    rot = np.eye(3) if rot is None else rot
    cc = clump_centres @ rot.T + centre[None, :]
    # first pass: per_clump draws per clump, in clump order
    owner = np.repeat(np.arange(nc), per_clump)[:n]
    pts = np.empty((0, 3)); tag = np.empty(0, np.int64)
    pending = owner
    out_pts, out_tag = [], []
    need = n
    while need > 0:
        c = pending[:need] if pending.size >= need else np.concatenate(
            [pending, rng.integers(0, nc, need - pending.size)])
        x = cc[c] + rng.normal(scale=sigma, size=(c.size, 3))
        inside = np.linalg.norm(x - centre[None, :], axis=1) <= R
        okx = np.zeros(c.size, bool)
        sel = np.nonzero(inside)[0]
        for s in range(0, sel.size, 8192):
            part = sel[s:s + 8192]
            okx[part] = excl.try_add(x[part])
        out_pts.append(x[okx]); out_tag.append(c[okx])
        need -= int(okx.sum())
        pending = c[~okx]  # redraw the rejected ones from their own clump
    return np.concatenate(out_pts), np.concatenate(out_tag), clump_centres


def _net_zero_normal(rng, n, sd=0.4):
    q = rng.normal(0.0, sd, n)
    return q - q.mean()


def uniform_cube(n: int = 1000, side: float = 20.0, k: int = 1) -> ParticleSet:
    rp, rq, ra = _streams(k)
    excl = _Exclusion([0, 0, 0], [side] * 3)
    pos, _ = _fill(excl, n, lambda m: (rp.uniform(0.0, side, (m, 3)), np.zeros(m, np.int64)))
    q = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
    alpha = ra.uniform(0.5, 2.0, n)
    return ParticleSet("uniform_cube", pos, q, alpha)


def globular(n: int = 50_000, density: float = 0.1, k: int = 2, radius: float | None = None) -> ParticleSet:
    rp, rq, ra = _streams(k)
    R = radius if radius is not None else (3.0 * n / (4.0 * math.pi * density)) ** (1.0 / 3.0)
    excl = _Exclusion([-R] * 3, [R] * 3)
    pos, _, _ = _clumped(excl, rp, n, R, np.zeros(3))
    return ParticleSet("globular", pos, _net_zero_normal(rq, n), ra.uniform(0.2, 2.0, n))


def _rot_z(t):
    c, s = math.cos(t), math.sin(t)
    return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])


def hexamer_shell(blob: int = 20_000, copies: int = 6, blob_radius: float = 35.0, ring: float = 45.0,
                  solvent: int = 40_000, r_in: float = 83.0, r_out: float = 96.2, k: int = 3) -> ParticleSet:
    rp, rq, ra = _streams(k)
    excl = _Exclusion([-r_out] * 3, [r_out] * 3)
    centres = _uniform_ball(rp, math.ceil(blob / 20), blob_radius)
    parts = []
    for c in range(copies):
        t = c * 2.0 * math.pi / copies
        ctr = ring * np.array([math.cos(t), math.sin(t), 0.0])
        x, _, _ = _clumped(excl, rp, blob, blob_radius, ctr, rot=_rot_z(t), clump_centres=centres)
        parts.append(x)

    def shell(m):
        v = rp.normal(size=(m, 3)); v /= np.linalg.norm(v, axis=1)[:, None]
        r = np.cbrt(rp.uniform(r_in**3, r_out**3, m))
        return v * r[:, None], np.zeros(m, np.int64)

    sol, _ = _fill(excl, solvent, shell)
    pos = np.concatenate(parts + [sol])
    nb = blob * copies
    q = np.concatenate([_net_zero_normal(rq, nb), np.zeros(solvent)])
    alpha = np.concatenate([ra.uniform(0.2, 2.0, nb), np.full(solvent, 1.5)])
    return ParticleSet("hexamer_shell", pos, q, alpha)


def scaling(n: int = 1_000_000, density: float = 0.1, k: int = 5) -> ParticleSet:
    rp, rq, ra = _streams(k, n)
    nu = n // 2
    ncl = n - nu
    L = (nu / density) ** (1.0 / 3.0)
    R = (3.0 * ncl / (4.0 * math.pi * density)) ** (1.0 / 3.0)
    ex1 = _Exclusion([0, 0, 0], [L] * 3)
    cube, _ = _fill(ex1, nu, lambda m: (rp.uniform(0.0, L, (m, 3)), np.zeros(m, np.int64)), batch=65536)
    del ex1
    centre = np.array([L + 10.0 + R, L / 2.0, L / 2.0])
    ex2 = _Exclusion(centre - R, centre + R)
    ball, _, _ = _clumped(ex2, rp, ncl, R, centre)
    del ex2
    pos = np.concatenate([cube, ball])
    return ParticleSet("scaling", pos, _net_zero_normal(rq, n), ra.uniform(0.2, 2.0, n))


def sphere(n: int = 4096, radius: float = 45.0, r_min: float = 2.0, alpha: float = 0.0, k: int = 6) -> ParticleSet:
    """The random sphere of the paper's accuracy tests (Sec. IV.A): n points uniform in a ball of
    the given radius with minimum separation r_min, n/2 charges +1 e and n/2 charges -1 e in random
    order (neutral), independently drawn field charges qE = +/-1 e (also neutral), the same
    polarisability alpha for every atom."""
    rp, rq, re = _streams(k)
    excl = _Exclusion([-radius] * 3, [radius] * 3, r_min=r_min)
    pos, _ = _fill(excl, n, lambda m: (_uniform_ball(rp, m, radius), np.zeros(m, np.int64)))
    q = np.where(rq.permutation(n) < n // 2, 1.0, -1.0)
    qE = np.where(re.permutation(n) < n // 2, 1.0, -1.0)
    if n % 2:
        q[-1] = 0.0
        qE[-1] = 0.0
    return ParticleSet("sphere", pos, q, np.full(n, float(alpha)), qE)


def small_globular(n: int = 2000, k: int = 4) -> ParticleSet:
    """The 2,000-particle clumped ball at 0.1 per Angstrom^3 (radius 16.8) used for gradient checks."""
    ps = globular(n, density=0.1, k=k, radius=16.8)
    ps.name = "small_globular"
    return ps


WORKLOADS = {
    "uniform_cube_1k": lambda: uniform_cube(1000),
    "globular_50k": lambda: globular(50_000),
    "hexamer_shell_160k": lambda: hexamer_shell(),
    "small_globular_2k": lambda: small_globular(2000),
    "scaling_250k": lambda: scaling(250_000),
    "scaling_1m": lambda: scaling(1_000_000),
    "scaling_4m": lambda: scaling(4_000_000),
    "sphere_4096": lambda: sphere(4096),
}


def make(name: str) -> ParticleSet:
    return WORKLOADS[name]()
