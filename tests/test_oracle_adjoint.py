"""Pins of the oracle's adjoint of the dipole equations (direct.dipole_adjoint): gradients of a loss
L(mu) through the induced dipoles.  No GPU.

* central finite differences of L = sum G . mu(x, q, alpha) with dense solves, on a 9-site cluster
  with Thole-damped pairs and a non-polarisable site (a second-order one-sided difference there,
  where alpha cannot go negative), for positions, charges and polarisabilities, with and without
  separate field charges q^E;
* the symmetry of the operator: lambda . E^q = G . mu exactly (lambda = A^-1 G, mu = A^-1 E^q);
* a closed form: one polarisable site in the field of a charge, mu = alpha E, dL/dalpha = G . E,
  dL/dq = G . E / q.
"""
import numpy as np
import pytest

from oracle import direct as D


def _cluster(n=9, seed=5, side=3.2):
    rng = np.random.default_rng(seed)
    pts = []
    while len(pts) < n:
        x = rng.uniform(0, side, 3)
        if all(np.linalg.norm(x - y) >= 1.0 for y in pts):
            pts.append(x)
    X = np.array(pts)
    q = rng.normal(0, 0.6, n)
    a = rng.uniform(0.5, 2.0, n)
    a[3] = 0.0
    G = rng.normal(0, 1, (n, 3))
    return X, q, a, G


def _loss(G, X, q, a, qE=None):
    E = None if qE is None else D.charge_fields(X, qE, want_grad=False)[1]
    return float(np.sum(G * D.solve_dipoles_dense(X, q, a, 2.0, E_q=E)))


def _fd_alpha(f, a, i, h):
    ap = a.copy(); ap[i] += h
    if a[i] > 0:
        am = a.copy(); am[i] -= h
        return (f(ap) - f(am)) / (2 * h)
    a2 = a.copy(); a2[i] += 2 * h
    return (-3 * f(a) + 4 * f(ap) - f(a2)) / (2 * h)


def relmax(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / np.abs(np.asarray(b)).max())


def test_adjoint_matches_finite_differences():
    X, q, a, G = _cluster()
    d = np.linalg.norm(X[:, None] - X[None], axis=2)
    np.fill_diagonal(d, 9.0)
    assert np.sum(d < 2.0 * np.cbrt(np.sqrt(a[:, None] * a[None]))) // 2 >= 5  # damped pairs present
    o = D.dipole_adjoint(X, q, a, G, 2.0)
    n = X.shape[0]
    fx = np.zeros((n, 3)); fq = np.zeros(n); fa = np.zeros(n)
    h = 1e-5
    for i in range(n):
        for c in range(3):
            Xp = X.copy(); Xp[i, c] += h
            Xm = X.copy(); Xm[i, c] -= h
            fx[i, c] = (_loss(G, Xp, q, a) - _loss(G, Xm, q, a)) / (2 * h)
        qp = q.copy(); qp[i] += h
        qm = q.copy(); qm[i] -= h
        fq[i] = (_loss(G, X, qp, a) - _loss(G, X, qm, a)) / (2 * h)
        fa[i] = _fd_alpha(lambda aa: _loss(G, X, q, aa), a, i, h)
    assert relmax(o["grad_pos"], fx) < 1e-8
    assert relmax(o["grad_q"], fq) < 1e-8
    assert relmax(o["grad_alpha"], fa) < 1e-7
    assert np.all(o["lam"][3] == 0.0) and np.all(o["mu"][3] == 0.0)


def test_adjoint_with_field_charges_matches_finite_differences():
    X, q, a, G = _cluster(seed=8)
    qE = np.random.default_rng(9).normal(0, 0.8, X.shape[0])
    o = D.dipole_adjoint(X, q, a, G, 2.0, qE=qE)
    assert np.all(o["grad_q"] == 0.0)
    n = X.shape[0]
    h = 1e-5
    fe = np.array([(_loss(G, X, q, a, qE + h * (np.arange(n) == i)) - _loss(G, X, q, a, qE - h * (np.arange(n) == i)))
                   / (2 * h) for i in range(n)])
    assert relmax(o["grad_qE"], fe) < 1e-8
    fx = np.zeros((n, 3))
    for i in range(n):
        for c in range(3):
            Xp = X.copy(); Xp[i, c] += h
            Xm = X.copy(); Xm[i, c] -= h
            fx[i, c] = (_loss(G, Xp, q, a, qE) - _loss(G, Xm, q, a, qE)) / (2 * h)
    assert relmax(o["grad_pos"], fx) < 1e-8


def test_adjoint_symmetry_of_the_operator():
    X, q, a, G = _cluster(seed=11)
    o = D.dipole_adjoint(X, q, a, G, 2.0)
    _, Eq, _ = D.charge_fields(X, q, want_grad=False)
    assert abs(np.sum(o["lam"] * Eq) - np.sum(G * o["mu"])) < 1e-13 * np.sum(np.abs(G * o["mu"]))


@pytest.mark.parametrize("r", [4.0, 1.3])
def test_adjoint_single_site_closed_form(r):
    """A charge and a polarisable site (the site alone carries a dipole, so no damping enters):
    mu = alpha E with E = q r_hat / r^2, and L = G . mu gives dL/dalpha = G . E and dL/dq = alpha G . E / q."""
    qq, al = 0.9, 1.7
    X = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, r]])
    G = np.array([[0.0, 0.0, 0.0], [0.3, -0.2, 0.7]])
    o = D.dipole_adjoint(X, np.array([qq, 0.0]), np.array([0.0, al]), G, 2.0)
    E = np.array([0.0, 0.0, qq / r**2])
    assert np.allclose(o["mu"][1], al * E, rtol=1e-15, atol=0)
    assert abs(o["grad_alpha"][1] - G[1] @ E) < 1e-15
    assert abs(o["grad_q"][0] - al * (G[1] @ E) / qq) < 1e-15
    # the radial derivative: L = alpha q G_z / r^2 -> dL/dz_site = -2 alpha q G_z / r^3
    assert abs(o["grad_pos"][1, 2] - (-2.0 * al * qq * G[1, 2] / r**3)) < 1e-14
