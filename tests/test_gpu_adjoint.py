"""The adjoint of the dipole equations on the GPU (pfmm_backward_mu through the C interface):
gradients of a loss that depends on the converged dipoles, against the oracle's adjoint
(oracle.direct.dipole_adjoint, pinned by finite differences of the dense solve).

* one leaf (everything direct): with and without field charges, plain and preconditioned solves,
  with Thole-damped pairs and a non-polarisable site: 1e-10;
* through the FMM (2,000 clumped particles, p = 8, four levels), both precision paths, against the
  stored dense adjoint (tests/golden/small_globular_2k_dense.npz): the method's truncation error;
* the autograd function returning (U, mu) against finite differences of the library's own solves;
* the adjoint leaves the saved state of the solve intact for the energy backward.
"""
import numpy as np
import pytest

from oracle import direct as D

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


def _cluster(n, side, seed):
    rng = np.random.default_rng(seed)
    pts = []
    while len(pts) < n:
        x = rng.uniform(0, side, 3)
        if all(np.sum((x - y) ** 2) >= 1.0 for y in pts):
            pts.append(x)
    X = np.array(pts)
    q = rng.normal(0, 0.5, n)
    a = rng.uniform(0.3, 2.0, n)
    a[4] = 0.0
    G = rng.normal(0, 1.0, (n, 3))
    return X, q, a, G


@pytest.mark.parametrize("pc", [0.0, 3.0])
def test_adjoint_one_leaf_equals_oracle(api, pc):
    print(f"[case] adjoint one leaf pc={pc}", flush=True)
    X, q, a, G = _cluster(120, 7.0, 21)
    ref = D.dipole_adjoint(X, q, a, G, thole_a=2.0)
    s = api.Solver(order_p=4, ws=1, leaf_width=50.0, scf_tol=1e-13, scf_max_iter=300, precond_cutoff=pc)
    r = s.solve(T(X), T(q), T(a))
    assert r.stats["levels"] == 0
    gp, gq, ga = s.backward_mu(T(G), solve_id=r.stats["solve_id"])
    assert relmax(N(gp), ref["grad_pos"]) < 1e-10
    assert relmax(N(gq), ref["grad_q"]) < 1e-10
    assert relmax(N(ga), ref["grad_alpha"]) < 1e-10


def test_adjoint_one_leaf_field_charges(api):
    print("[case] adjoint one leaf qE", flush=True)
    X, q, a, G = _cluster(100, 6.8, 22)
    qE = np.random.default_rng(23).normal(0, 0.7, X.shape[0])
    ref = D.dipole_adjoint(X, q, a, G, thole_a=2.0, qE=qE)
    s = api.Solver(order_p=4, ws=1, leaf_width=50.0, scf_tol=1e-13, scf_max_iter=300)
    s.solve(T(X), T(q), T(a), qE=T(qE))
    gp, gq, ga, ge = s.backward_mu(T(G), want_qE=True)
    assert np.all(N(gq) == 0.0)
    assert relmax(N(ge), ref["grad_qE"]) < 1e-10
    assert relmax(N(gp), ref["grad_pos"]) < 1e-10
    assert relmax(N(ga), ref["grad_alpha"]) < 1e-10


def test_adjoint_keeps_the_energy_backward(api):
    """The adjoint solve borrows the dipole buffers of the solve; the energy backward after it is
    bitwise the one before, and a second adjoint repeats the first."""
    print("[case] adjoint keeps state", flush=True)
    X, q, a, G = _cluster(300, 11.0, 24)
    s = api.Solver(order_p=6, ws=2, leaf_width=2.0, scf_tol=1e-10, precond_cutoff=2.5)
    r = s.solve(T(X), T(q), T(a))
    assert r.stats["levels"] >= 2
    b0 = [N(t) for t in s.backward(1.0)]
    a1 = [N(t) for t in s.backward_mu(T(G))]
    b1 = [N(t) for t in s.backward(1.0)]
    a2 = [N(t) for t in s.backward_mu(T(G))]
    for u, v in zip(b0, b1):
        assert np.array_equal(u, v)
    for u, v in zip(a1, a2):
        assert np.array_equal(u, v)
    z = s.backward_mu(T(np.zeros_like(G)))
    assert all(float(np.abs(N(t)).max()) == 0.0 for t in z)


@pytest.mark.parametrize("precision,gate", [("fp64", 3e-4), ("mixed", 3e-4)])
def test_adjoint_fmm_2k_vs_dense_oracle(api, precision, gate):
    """Through the FMM (four levels): gradients of L = sum G . mu against the dense oracle's adjoint."""
    print(f"[case] adjoint fmm 2k {precision}", flush=True)
    import os
    from paper_1408_6527_amd import inputs
    ps = inputs.small_globular(2000)
    ref = np.load(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "small_globular_2k_dense.npz"))
    s = api.Solver(order_p=8, ws=2, leaf_width=3.0, scf_tol=1e-10 if precision == "fp64" else 1e-7,
                   precision=precision, precond_cutoff=3.0)
    r = s.solve(T(ps.pos), T(ps.q), T(ps.alpha))
    assert r.stats["levels"] >= 3
    gp, gq, ga = s.backward_mu(T(ref["adj_G"]), solve_id=r.stats["solve_id"])
    e = dict(pos=relnorm(N(gp), ref["adj_grad_pos"]), q=relnorm(N(gq), ref["adj_grad_q"]),
             alpha=relnorm(N(ga), ref["adj_grad_alpha"]))
    print(f"adjoint fmm 2k {precision}: dL/dx {e['pos']:.3e} dL/dq {e['q']:.3e} dL/dalpha {e['alpha']:.3e}",
          flush=True)
    assert e["pos"] < gate and e["q"] < gate and e["alpha"] < gate


def test_polarizable_solve_autograd_against_finite_differences(api):
    """L = U + sum w . mu through PolarizableSolve: autograd gradients against central differences of
    the library's own solves (one leaf, tight tolerance)."""
    print("[case] PolarizableSolve fd", flush=True)
    X, q, a, G = _cluster(60, 5.5, 25)
    w = 300.0 * G  # comparable to U in size
    s = api.Solver(order_p=4, ws=1, leaf_width=50.0, scf_tol=1e-14, scf_max_iter=400)
    pos, qq, al = T(X).requires_grad_(True), T(q).requires_grad_(True), T(a).requires_grad_(True)
    U, mu = api.PolarizableSolve.apply(pos, qq, al, s)
    L = U + (mu * T(w)).sum()
    L.backward()

    def loss(X_, q_, a_):
        r = s.solve(T(X_), T(q_), T(a_))
        return r.U + float(np.sum(N(r.mu) * w))

    rng = np.random.default_rng(26)
    h = 1e-5
    for _ in range(5):
        i, c = int(rng.integers(60)), int(rng.integers(3))
        Xp = X.copy(); Xp[i, c] += h
        Xm = X.copy(); Xm[i, c] -= h
        fd = (loss(Xp, q, a) - loss(Xm, q, a)) / (2 * h)
        assert abs(fd - pos.grad[i, c].item()) < 1e-6 * max(1.0, abs(fd))
        qp = q.copy(); qp[i] += h
        qm = q.copy(); qm[i] -= h
        fd = (loss(X, qp, a) - loss(X, qm, a)) / (2 * h)
        assert abs(fd - qq.grad[i].item()) < 1e-6 * max(1.0, abs(fd))
        if a[i] > 0:
            ap = a.copy(); ap[i] += h
            am = a.copy(); am[i] -= h
            fd = (loss(X, q, ap) - loss(X, q, am)) / (2 * h)
            assert abs(fd - al.grad[i].item()) < 1e-6 * max(1.0, abs(fd))
