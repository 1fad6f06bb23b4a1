"""The adaptive octree on the GPU (adaptive_leaf_max: cells split only above leaf_max particles, 2:1
balanced; the octree form of the paper's adaptive tree, Sec. III) against the oracle's adaptive walk
(oracle.fmm.Octree.walk_lists with leaf_max) and its FMM on those lists:

* list sizes are integer work: the M2L cell pairs and the ordered direct particle pairs of a solve
  equal the oracle's counts exactly, with the ws rule (ws = 1, 2) and with the acceptance criterion
  (with and without the paper's direct rules), up to order 9 and with a root that is a leaf;
* fields of fixed charges and dipoles: 1e-11 against the oracle's FMM on the same lists;
* Newton's third law: the total force of a solve vanishes to rounding;
* the dipole solve: the oracle's FMM fields of the library's dipoles satisfy the stopping rule, and
  the energy, forces and potentials are the oracle's evaluation at those dipoles (1e-10);
* the 160,000-particle hexamer in its solvent shell against the direct-sum oracle's exact solution,
  beside the uniform tree.
"""
import time

import numpy as np
import pytest

from oracle import direct as D
from oracle import fmm as FM

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    import torch
    from paper_1408_6527_amd import api as A
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return A


def T(x):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def N(t):
    return t.detach().cpu().numpy()


def relmax(a, b):
    a = np.asarray(a); b = np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _clumped(n_core, n_sparse, seed, core=10.0, side=40.0, r_min=1.2):
    """A dense core of n_core particles in a cube of edge core at the centre of a sparse cloud of
    n_sparse in a cube of edge side, no two closer than r_min (sequential rejection)."""
    rng = np.random.default_rng(seed)
    pts = []

    def add(n, lo, hi):
        k = 0
        while k < n:
            p = rng.uniform(lo, hi, 3)
            if not pts or np.min(np.sum((np.asarray(pts) - p) ** 2, axis=1)) >= r_min ** 2:
                pts.append(p)
                k += 1

    add(n_core, (side - core) / 2, (side + core) / 2)
    add(n_sparse, 0.0, side)
    X = np.asarray(pts)
    n = len(X)
    q = rng.normal(0, 0.5, n)
    q -= q.mean()
    a = rng.uniform(0.5, 1.0, n)
    mu = rng.normal(0, 0.2, (n, 3))
    return X, q, a, mu


def _dirty_device_memory():
    """Hand NaN-filled memory back to the HIP allocator, so that workspace the library allocates next
    is likely to start out as garbage rather than zeros."""
    import torch
    junk = torch.full((64 << 20,), float("nan"), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    del junk
    torch.cuda.empty_cache()


def _oracle_counts(X, lw, ws, theta, nd, ld, lmax):
    tree = FM.Octree(X, lw, ws)
    m2l, near = tree.walk_lists(X, theta, nd, bool(ld), leaf_max=lmax)
    nm = sum(len(x) for x in m2l)
    npairs = 0
    for l, B, A in near:
        nb, na = len(tree.members(l, B)), len(tree.members(l, A))
        npairs += nb * na - (nb if A == B else 0)
    return tree, nm, npairs, near


LW, THOLE = 2.6, 2.0
# ws, theta, leaf_max, p, ndirect, leaf_direct
CASES = [
    (1, None, 8, 5, 0, 0),
    (2, None, 12, 4, 0, 0),
    (1, 0.6, 8, 5, 0, 0),
    (1, 0.7, 8, 6, 20, 1),
    (1, None, 6, 9, 0, 0),
    (1, None, 10**6, 4, 0, 0),
]


@pytest.mark.parametrize("ws,theta,lmax,p,nd,ld", CASES)
def test_adaptive_fields_and_lists_match_oracle(api, ws, theta, lmax, p, nd, ld):
    print(f"[case] adaptive fields ws={ws} theta={theta} leaf_max={lmax} p={p} ndirect={nd} leaf_direct={ld}",
          flush=True)
    X, q, a, mu = _clumped(220, 330, 2)
    kw = dict(order_p=p, ws=ws, leaf_width=LW, thole_a=THOLE, adaptive_leaf_max=lmax,
              mac_theta=theta or 0.0, mac_ndirect=nd, mac_leaf_direct=ld)
    _dirty_device_memory()
    s = api.Solver(scf_tol=1e-10, **kw)
    # a first evaluation of other sources on the same handle: nothing of it may leak into the next
    s.field(T(X), T(3.0 * q[::-1].copy()), T(-2.0 * mu), T(a))
    phi, E, Ed, G = s.field(T(X), T(q), T(mu), T(a))
    ref = FM.fmm_fields(X, q, mu, a, THOLE, p, LW, ws, theta=theta, ndirect=nd, leaf_direct=bool(ld),
                        leaf_max=lmax)
    tree, nm, npairs, near = _oracle_counts(X, LW, ws, theta, nd, ld, lmax)
    assert tree.L >= 4 and any(l < tree.L for l, _, _ in near)
    if lmax < len(X):
        assert nm > 0
    errs = [relmax(N(phi), ref["phi"]), relmax(N(E), ref["E_u"]), relmax(N(Ed), ref["E_d"]),
            relmax(N(G), ref["G_d"])]
    r = s.solve(T(X), T(q), T(a))
    print(f"adaptive fields ws={ws} theta={theta} leaf_max={lmax}: M2L pairs {r.stats['n_m2l']} (oracle {nm}), "
          f"direct pairs {r.stats['n_p2p']} (oracle {npairs}), direct cell pairs above the finest level "
          f"{sum(1 for l, _, _ in near if l < tree.L)} of {len(near)}, field errors {max(errs):.1e}", flush=True)
    assert max(errs) < 1e-11
    assert r.stats["n_m2l"] == nm and r.stats["n_p2p"] == npairs


@pytest.mark.parametrize("ws,theta", [(2, None), (1, 0.5)])
def test_total_force_vanishes(api, ws, theta):
    print(f"[case] adaptive momentum ws={ws} theta={theta}", flush=True)
    X, q, a, _ = _clumped(300, 500, 5)
    kw = dict(order_p=6, ws=ws, leaf_width=LW, scf_tol=1e-8, adaptive_leaf_max=10)
    if theta is not None:
        kw.update(mac_theta=theta, mac_ndirect=0, mac_leaf_direct=0)
    r = api.Solver(**kw).solve(T(X), T(q), T(a))
    F = N(r.forces)
    rel = float(np.abs(F.sum(axis=0)).max() / np.abs(F).sum())
    print(f"adaptive momentum ws={ws} theta={theta}: |sum F| / sum |F| = {rel:.1e}, M2L pairs {r.stats['n_m2l']}",
          flush=True)
    assert r.stats["n_m2l"] > 0 and rel < 1e-12


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_adaptive_solve_matches_oracle_fmm(api, precision):
    """The dipole solve on the adaptive lists: the oracle's FMM of the library's dipoles (same lists)
    gives the residual within the tolerance, and its evaluation at those dipoles the library's energy,
    forces and potentials."""
    print(f"[case] adaptive solve {precision}", flush=True)
    X, q, a, _ = _clumped(220, 330, 3)
    p, lmax = 5, 8
    tol = 1e-10 if precision == "fp64" else 1e-7
    s = api.Solver(order_p=p, ws=1, leaf_width=LW, scf_tol=tol, adaptive_leaf_max=lmax, precision=precision,
                   precond_cutoff=2.6 if precision == "mixed" else 0.0)
    r = s.solve(T(X), T(q), T(a))
    mu = N(r.mu)
    st1 = FM.fmm_fields(X, q, None, a, THOLE, p, LW, 1, leaf_max=lmax)
    st2 = FM.fmm_fields(X, None, mu, a, THOLE, p, LW, 1, leaf_max=lmax)
    res = np.linalg.norm(a[:, None] * (st1["E_d"] + st2["E_d"]) - mu) / np.linalg.norm(a[:, None] * st1["E_d"])
    print(f"adaptive solve {precision}: oracle residual {res:.2e}, library {r.residual:.2e}, iters {r.iters}",
          flush=True)
    assert res < (2e-10 if precision == "fp64" else 3e-6)
    if precision == "fp64":
        ev = D.evaluate(X, q, a, mu, THOLE, D.COULOMB_K, charge=(st1["phi"], st1["E_d"], st1["G_d"]),
                        dip=(st2["phi"], st2["E_u"], st2["E_d"], st2["G_d"]), want_grad_alpha=False)
        assert abs(r.U - ev["U"]) < 1e-10 * abs(ev["U"])
        assert relmax(N(r.forces), ev["F"]) < 1e-10
        assert relmax(N(r.phi), ev["phi"]) < 1e-10
    # against the dense oracle: the FMM's own error, at the uniform tree's level (ws = 1 and p = 5 leave
    # about 1e-2 on this clump)
    ref = D.solve(X, q, a, thole_a=THOLE)
    u = api.Solver(order_p=p, ws=1, leaf_width=LW, scf_tol=tol, precision=precision,
                   precond_cutoff=2.6 if precision == "mixed" else 0.0).solve(T(X), T(q), T(a))
    fe = np.linalg.norm(N(r.forces) - ref["F"]) / np.linalg.norm(ref["F"])
    fu = np.linalg.norm(N(u.forces) - ref["F"]) / np.linalg.norm(ref["F"])
    print(f"adaptive solve {precision}: force error against the dense oracle {fe:.2e} (uniform tree {fu:.2e})",
          flush=True)
    assert fe < 1.5 * fu


@pytest.mark.parametrize("ws,p,slack", [(2, 6, 1), (1, 8, 0)])
def test_adaptive_offset_orders_match_oracle(api, ws, p, slack):
    """The ws lists' per-offset truncation orders (m2l_order_slack) on the adaptive octree: the same
    orders as the oracle's offset_order for every accepted pair, so the fields agree to rounding."""
    print(f"[case] adaptive offset orders ws={ws} p={p} slack={slack}", flush=True)
    X, q, a, mu = _clumped(220, 330, 4)
    s = api.Solver(order_p=p, ws=ws, leaf_width=LW, thole_a=THOLE, adaptive_leaf_max=10, m2l_order_slack=slack)
    phi, E, Ed, G = s.field(T(X), T(q), T(mu), T(a))
    ref = FM.fmm_fields(X, q, mu, a, THOLE, p, LW, ws, order_slack=slack, leaf_max=10)
    plain = FM.fmm_fields(X, q, mu, a, THOLE, p, LW, ws, leaf_max=10)
    assert relmax(ref["E_d"], plain["E_d"]) > 1e-9  # the truncation really differs
    errs = [relmax(N(phi), ref["phi"]), relmax(N(E), ref["E_u"]), relmax(N(Ed), ref["E_d"]),
            relmax(N(G), ref["G_d"])]
    print(f"adaptive offset orders ws={ws} p={p} slack={slack}: field errors {max(errs):.1e}", flush=True)
    assert max(errs) < 1e-11
    sm = api.Solver(order_p=p, ws=ws, leaf_width=LW, thole_a=THOLE, adaptive_leaf_max=10, m2l_order_slack=slack,
                    precision="mixed")
    assert relmax(N(sm.field(T(X), T(q), T(mu), T(a))[2]), ref["E_d"]) < 1e-5


def test_adaptive_edge_cases(api):
    """Sizes 0, 1 and 2; every particle in one cell; leaf_max = 1 (the deepest tree the balance
    allows); two clusters far apart with nothing between them: the library against the oracle."""
    print("[case] adaptive edge cases", flush=True)
    import torch
    s = api.Solver(order_p=4, ws=1, leaf_width=LW, adaptive_leaf_max=8)
    z = torch.zeros((0, 3), dtype=torch.float64, device="cuda")
    r = s.solve(z, torch.zeros(0, dtype=torch.float64, device="cuda"), torch.zeros(0, dtype=torch.float64, device="cuda"))
    assert r.U == 0.0 and r.mu.shape == (0, 3)
    r = s.solve(T([[1.0, 2.0, 3.0]]), T([0.7]), T([1.2]))
    assert r.U == 0.0 and np.all(N(r.mu) == 0) and np.all(N(r.forces) == 0)
    X2 = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 3.1]])
    r = api.Solver(order_p=4, ws=1, scf_tol=1e-14, thole_a=0.0, adaptive_leaf_max=1).solve(
        T(X2), T([0.7, -0.4]), T([1.3, 0.9]))
    ref = D.solve(X2, np.array([0.7, -0.4]), np.array([1.3, 0.9]), thole_a=0.0)
    assert relmax(N(r.mu), ref["mu"]) < 1e-13
    rng = np.random.default_rng(11)
    # every particle in one finest cell
    Xc = rng.uniform(0.0, 2.0, (40, 3))
    qc, ac, mc = rng.normal(0, 0.5, 40), rng.uniform(0.1, 0.3, 40), rng.normal(0, 0.2, (40, 3))
    fc = api.Solver(order_p=4, ws=1, leaf_width=LW, thole_a=0.0, adaptive_leaf_max=4).field(T(Xc), T(qc), T(mc), T(ac))
    pq, Eq, _ = D.charge_fields(Xc, qc)
    pm, Eu, _, _ = D.dipole_fields(Xc, mc, ac, 0.0)
    assert relmax(N(fc[1]), Eq + Eu) < 1e-12
    # leaf_max = 1, and two clusters 150 A apart
    X, q, a, mu = _clumped(150, 150, 12)
    Xf = np.vstack([X[:150], X[150:] + np.array([150.0, 0.0, 0.0])])
    for Xs, lmax in ((X, 1), (Xf, 10)):
        f = api.Solver(order_p=4, ws=1, leaf_width=LW, thole_a=THOLE, adaptive_leaf_max=lmax).field(
            T(Xs), T(q), T(mu), T(a))
        ref = FM.fmm_fields(Xs, q, mu, a, THOLE, 4, LW, 1, leaf_max=lmax)
        err = max(relmax(N(f[0]), ref["phi"]), relmax(N(f[1]), ref["E_u"]), relmax(N(f[2]), ref["E_d"]),
                  relmax(N(f[3]), ref["G_d"]))
        print(f"adaptive edge leaf_max={lmax} levels {ref['tree'].L}: field errors {err:.1e}", flush=True)
        assert err < 1e-11


def test_adaptive_with_exclusions_and_site_tree(api):
    """The adaptive lists with excluded pairs (1-2 and 1-3 pairs of a chain through the particle
    order and two far pairs) against the oracle's FMM with the same exclusions; and the dipole solve
    on a tree of the polarisable sites (a third of the particles), also adaptive, against the single
    adaptive tree."""
    print("[case] adaptive exclusions and site tree", flush=True)
    X, q, a, mu = _clumped(220, 330, 6)
    n = len(X)
    excl = [(i, i + 1) for i in range(n - 1)] + [(i, i + 2) for i in range(n - 2)] + [(3, 500), (10, 540)]
    s = api.Solver(order_p=5, ws=1, leaf_width=LW, thole_a=THOLE, adaptive_leaf_max=8)
    s.set_exclusions(n, excl)
    f = s.field(T(X), T(q), T(mu), T(a))
    ref = FM.fmm_fields(X, q, mu, a, THOLE, 5, LW, 1, excl=excl, leaf_max=8)
    err = max(relmax(N(f[0]), ref["phi"]), relmax(N(f[1]), ref["E_u"]), relmax(N(f[2]), ref["E_d"]),
              relmax(N(f[3]), ref["G_d"]))
    print(f"adaptive exclusions: field errors {err:.1e}", flush=True)
    assert err < 1e-11
    a3 = a.copy()
    a3[np.random.default_rng(7).permutation(n) >= n // 3] = 0.0
    kw = dict(order_p=6, ws=2, leaf_width=LW, scf_tol=1e-9, adaptive_leaf_max=10)
    r1 = api.Solver(**kw).solve(T(X), T(q), T(a3))
    r2 = api.Solver(dipole_tree=1, **kw).solve(T(X), T(q), T(a3))
    d = float(np.linalg.norm(N(r2.forces) - N(r1.forces)) / np.linalg.norm(N(r1.forces)))
    print(f"adaptive site tree: {r2.stats['n_sites']} sites, force difference from the single tree {d:.2e}",
          flush=True)
    assert r2.stats["n_sites"] == int(np.sum(a3 > 0)) and d < 1e-3


def test_config_rules(api):
    with pytest.raises(api.PFMMError, match="INVALID_ARG"):
        api.Solver(order_p=10, adaptive_leaf_max=8)
    with pytest.raises(api.PFMMError, match="INVALID_ARG"):
        api.Solver(order_p=6, adaptive_leaf_max=8, mac_theta=0.5, m2l_order_slack=1)
    with pytest.raises(api.PFMMError, match="INVALID_ARG"):
        api.Solver(order_p=6, adaptive_leaf_max=-1)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_hexamer_shell_160k_adaptive_vs_full_oracle(api, precision):
    """Six 20k blobs at 0.1 per A^3 in a shell of 40k solvent sites at 0.03 per A^3 (p = 8, ws = 2,
    5 A finest leaves, order slack 2): the adaptive octree (cells split above 32 particles) against
    the exact solution of the direct-sum oracle, beside the uniform tree at the same settings."""
    print(f"[case] adaptive hexamer shell 160k {precision}", flush=True)
    import os
    import torch
    from paper_1408_6527_amd import inputs
    ps = inputs.make("hexamer_shell_160k")
    ref = np.load(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "hexamer_shell_160k_oracle.npz"))
    out = {}
    for lmax in (0, 32):
        s = api.Solver(order_p=8, ws=2, leaf_width=5.0, scf_tol=1e-6, precond_cutoff=4.0, precision=precision,
                       m2l_order_slack=2, adaptive_leaf_max=lmax)
        s.solve(T(ps.pos), T(ps.q), T(ps.alpha))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = s.solve(T(ps.pos), T(ps.q), T(ps.alpha))
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        F = N(r.forces)
        e = float(np.linalg.norm(F - ref["F"]) / np.linalg.norm(ref["F"]))
        eu = abs(r.U - float(ref["U"])) / abs(float(ref["U"]))
        out[lmax] = e
        print(f"hexamer 160k {precision} leaf_max={lmax}: force error {e:.2e}, energy error {eu:.2e}, "
              f"{dt * 1e3:.1f} ms per solve, iters {r.iters}, M2L pairs {r.stats['n_m2l']}, "
              f"direct pairs {r.stats['n_p2p']}", flush=True)
        assert e < 1e-4 and eu < 1e-4
    assert out[32] < 3 * out[0]
