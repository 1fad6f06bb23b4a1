"""The dipole solve on a tree of the polarisable sites alone (dipole_tree = 1; T^mu of Sec. III)
against the oracle.  Only a third of the particles are polarisable, as in the paper's systems.

* one leaf on both trees (everything direct): the dense oracle's solution, 1e-11;
* through the FMM: the oracle's FMM of the charges on all particles plus its FMM of the dipoles on
  the sites alone (its own tree of the subset, built by the same rule) gives the library's residual,
  and its FMM of the final dipoles on all particles gives the library's energy, forces and
  potentials (1e-10); against the dense oracle the error is the method's;
* the adjoint (pfmm_backward_mu) runs on the same site tree: one leaf against the oracle's adjoint;
* all or no polarisable sites: the single tree is used (n_sites = n).
"""
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


def relnorm(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def _third_polarisable(ps, seed):
    """Every third particle (seeded choice) keeps its alpha; the others are not polarisable."""
    a = ps.alpha.copy()
    keep = np.random.default_rng(seed).permutation(ps.n) < ps.n // 3
    a[~keep] = 0.0
    return a


def test_sites_one_leaf_equals_dense_oracle(api):
    print("[case] sites one leaf", flush=True)
    from paper_1408_6527_amd import inputs
    ps = inputs.small_globular(2000)
    sel = np.arange(300)
    X, q = ps.pos[sel], ps.q[sel]
    a = ps.alpha[sel].copy()
    a[np.random.default_rng(3).permutation(300) >= 100] = 0.0
    ref = D.solve(X, q, a, thole_a=2.0)
    s = api.Solver(order_p=4, ws=1, leaf_width=100.0, scf_tol=1e-13, scf_max_iter=300, dipole_tree=1)
    r = s.solve(T(X), T(q), T(a))
    assert r.stats["n_sites"] == 100 and r.stats["levels"] == 0
    assert relmax(N(r.mu), ref["mu"]) < 1e-11
    assert abs(r.U - ref["U"]) < 1e-11 * abs(ref["U"])
    assert relmax(N(r.forces), ref["F"]) < 1e-11
    assert relmax(N(r.phi), ref["phi"]) < 1e-11
    gp, gq, ga = s.backward(1.0)
    assert relmax(-N(gp), ref["F"]) < 1e-11 and relmax(N(ga), ref["grad_alpha"]) < 1e-10
    G = np.random.default_rng(4).normal(0, 1, (300, 3))
    adj = D.dipole_adjoint(X, q, a, G, thole_a=2.0)
    bp, bq, ba = s.backward_mu(T(G))
    assert relmax(N(bp), adj["grad_pos"]) < 1e-10
    assert relmax(N(bq), adj["grad_q"]) < 1e-10
    assert relmax(N(ba), adj["grad_alpha"]) < 1e-10


@pytest.mark.parametrize("pc", [0.0, 2.5])
def test_sites_fmm_matches_oracle_fmm(api, pc):
    """1,000 particles in a 20 A cube, a third polarisable, p = 4, ws = 1: the site tree's solve against
    the oracle's FMM on the same two trees."""
    print(f"[case] sites fmm pc={pc}", flush=True)
    from paper_1408_6527_amd import inputs
    ps = inputs.uniform_cube(1000)
    a = _third_polarisable(ps, 5)
    lw = 2.6
    s = api.Solver(order_p=4, ws=1, leaf_width=lw, scf_tol=1e-10, dipole_tree=1, precond_cutoff=pc)
    r = s.solve(T(ps.pos), T(ps.q), T(a))
    sites = np.nonzero(a > 0)[0]
    assert r.stats["n_sites"] == sites.size
    mu = N(r.mu)
    assert np.all(mu[a == 0] == 0.0)
    st1 = FM.fmm_fields(ps.pos, ps.q, None, a, 2.0, 4, lw, 1)
    sub = FM.fmm_fields(ps.pos[sites], None, mu[sites], a[sites], 2.0, 4, lw, 1)
    Eq = st1["E_d"][sites]
    res = np.linalg.norm(a[sites, None] * (Eq + sub["E_d"]) - mu[sites]) / np.linalg.norm(a[sites, None] * Eq)
    print(f"sites fmm: residual on the site tree {res:.2e}, iters {r.iters}", flush=True)
    assert res < 2e-10
    st3 = FM.fmm_fields(ps.pos, None, mu, a, 2.0, 4, lw, 1)
    ev = D.evaluate(ps.pos, ps.q, a, mu, 2.0, D.COULOMB_K, charge=(st1["phi"], st1["E_d"], st1["G_d"]),
                    dip=(st3["phi"], st3["E_u"], st3["E_d"], st3["G_d"]), want_grad_alpha=False)
    assert abs(r.U - ev["U"]) < 1e-10 * abs(ev["U"])
    assert relmax(N(r.forces), ev["F"]) < 1e-10
    assert relmax(N(r.phi), ev["phi"]) < 1e-10
    ref = D.solve(ps.pos, ps.q, a, thole_a=2.0)
    one = api.Solver(order_p=4, ws=1, leaf_width=lw, scf_tol=1e-10).solve(T(ps.pos), T(ps.q), T(a))
    e_sites, e_one = relnorm(N(r.forces), ref["F"]), relnorm(N(one.forces), ref["F"])
    print(f"sites fmm: force error {e_sites:.3e} (single tree {e_one:.3e}), dipole error "
          f"{relnorm(mu, ref['mu']):.3e}", flush=True)
    assert e_sites < 2 * e_one + 1e-3


def test_sites_fall_back_to_one_tree(api):
    print("[case] sites fallback", flush=True)
    from paper_1408_6527_amd import inputs
    ps = inputs.uniform_cube(1000)
    s = api.Solver(order_p=4, ws=1, leaf_width=2.6, scf_tol=1e-10, dipole_tree=1)
    plain = api.Solver(order_p=4, ws=1, leaf_width=2.6, scf_tol=1e-10)
    r = s.solve(T(ps.pos), T(ps.q), T(ps.alpha))
    r0 = plain.solve(T(ps.pos), T(ps.q), T(ps.alpha))
    assert r.stats["n_sites"] == ps.n
    assert np.array_equal(N(r.forces), N(r0.forces)) and r.U == r0.U
    z = s.solve(T(ps.pos), T(ps.q), T(np.zeros(ps.n)))
    assert z.stats["n_sites"] == ps.n and np.all(N(z.mu) == 0.0)
    with pytest.raises(api.PFMMError, match="INVALID_ARG"):
        s.set_exclusions(ps.n, [(0, 1)])
        s.solve(T(ps.pos), T(ps.q), T(_third_polarisable(ps, 6)))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_sites_globular_50k(api, precision):
    """50,000 clumped particles, a third polarisable, p = 6: the site tree's solve agrees with the
    single tree's to the FMM error, with fewer particles in the solve's evaluations."""
    print(f"[case] sites 50k {precision}", flush=True)
    import time
    import torch
    from paper_1408_6527_amd import inputs
    ps = inputs.globular(50_000)
    a = _third_polarisable(ps, 7)
    kw = dict(order_p=6, ws=2, leaf_width=4.0, scf_tol=1e-8, precond_cutoff=4.0, precision=precision)
    out = {}
    for tree in (0, 1):
        s = api.Solver(dipole_tree=tree, **kw)
        s.solve(T(ps.pos), T(ps.q), T(a))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = s.solve(T(ps.pos), T(ps.q), T(a))
        torch.cuda.synchronize()
        out[tree] = (r, time.perf_counter() - t0)
    (r0, t0), (r1, t1) = out[0], out[1]
    d = relnorm(N(r1.forces), N(r0.forces))
    print(f"sites 50k {precision}: n_sites {r1.stats['n_sites']}, force difference {d:.2e}, "
          f"{t0 * 1e3:.1f} ms (one tree) vs {t1 * 1e3:.1f} ms (site tree), iters {r0.iters} / {r1.iters}", flush=True)
    assert r1.stats["n_sites"] == int(np.sum(a > 0))
    assert d < 3e-4


def test_sites_relaxed_and_preconditioned_solve(api):
    """The benchmark's solver settings (per-offset orders, near-field preconditioner, relaxed
    evaluations) on the site tree: the stopping rule is checked with the site tree's own field at the
    full orders, so the solve converges, to the unrelaxed site-tree solve's dipoles within the
    tolerance."""
    print("[case] sites relaxed", flush=True)
    from paper_1408_6527_amd import inputs
    ps = inputs.globular(50_000)
    a = _third_polarisable(ps, 8)
    kw = dict(order_p=8, ws=2, leaf_width=5.0, scf_tol=1e-6, m2l_order_slack=2, precond_cutoff=4.0, dipole_tree=1)
    r0 = api.Solver(**kw).solve(T(ps.pos), T(ps.q), T(a))
    r1 = api.Solver(scf_relax=0.01, **kw).solve(T(ps.pos), T(ps.q), T(a))
    d = relnorm(N(r1.mu), N(r0.mu))
    print(f"sites relaxed: iters {r1.iters} (unrelaxed {r0.iters}), continuations {r1.stats['scf_restarts']}, "
          f"dipole difference {d:.2e}, full-tree residual {r1.residual:.2e}", flush=True)
    assert d < 3e-6
    assert r1.stats["m2l_order_cap_min"] < 8
