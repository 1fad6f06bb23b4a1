"""Pins of the matrix-free direct-sum oracle (oracle/native.py + liborcdirect.so) and of the
sampled-target fields of oracle/direct.py.  No GPU.

Each pin ties the code to something other than itself:
* the sampled-target fields (direct.fields_at) against the per-source-type sums written out
  separately (direct.charge_fields + direct.dipole_fields), with damped pairs and a zero alpha;
* the C++ sums against the NumPy sums (different language, loop order and summation) and against
  the dense matrix of the dipole tensor;
* the matrix-free solve against the dense LU solve of the scaled system at 2,000 particles, to 1e-12;
* closed forms: two charges (Coulomb's law), a charge and a polarisable site, two polarisable
  sites on an axis (the 2 x 2 closed form of the dipole equations).
"""
import numpy as np
import pytest

from oracle import direct as D
from oracle import native as NT


def relmax(a, b):
    a = np.asarray(a); b = np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def relnorm(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def _cloud(n, side, seed, a_zero=(5,)):
    """n points in a cube at least 0.9 A apart (so that Thole-damped pairs exist at a = 2)."""
    rng = np.random.default_rng(seed)
    pts = []
    while len(pts) < n:
        x = rng.uniform(0, side, 3)
        if all(np.sum((x - y) ** 2) >= 0.81 for y in pts):
            pts.append(x)
    X = np.array(pts)
    q = rng.normal(0, 0.5, n)
    a = rng.uniform(0.2, 2.0, n)
    for i in a_zero:
        a[i] = 0.0
    mu = rng.normal(0, 0.2, (n, 3))
    return X, q, a, mu


def _damped_pairs(X, a, thole_a=2.0):
    d = np.linalg.norm(X[:, None] - X[None], axis=2)
    s = thole_a * np.cbrt(np.sqrt(a[:, None] * a[None, :]))
    np.fill_diagonal(d, np.inf)
    return int(np.sum(d < s) // 2)


def test_fields_at_equals_charge_plus_dipole_fields():
    """direct.fields_at (used for sampled checks of large systems) at every target of a 60-particle
    system equals the charge and dipole sums evaluated separately."""
    X, q, a, mu = _cloud(60, 5.0, 1)
    assert _damped_pairs(X, a) > 5
    pq, Eq, Gq = D.charge_fields(X, q)
    pm, Eu, Ed, Gd = D.dipole_fields(X, mu, a, 2.0)
    idx = np.arange(60)
    phi, EU, ED, G = D.fields_at(idx, X, q, mu, a, 2.0)
    assert relmax(phi, pq + pm) < 1e-14
    assert relmax(EU, Eq + Eu) < 1e-14
    assert relmax(ED, Eq + Ed) < 1e-14
    assert relmax(G, Gq + Gd) < 1e-14
    # a subset in any order returns the same rows
    sub = np.array([17, 3, 59, 5, 0])
    s_phi, s_EU, s_ED, s_G = D.fields_at(sub, X, q, mu, a, 2.0)
    assert relmax(s_ED, ED[sub]) < 1e-15 and relmax(s_G, G[sub]) < 1e-15
    # no damping, no dipoles: Coulomb alone
    c_phi, c_EU, c_ED, c_G = D.fields_at(idx, X, q, None, None, 2.0)
    assert relmax(c_phi, pq) < 1e-14 and relmax(c_ED, Eq) < 1e-14 and relmax(c_G, Gq) < 1e-14


def test_native_fields_equal_numpy_sums():
    X, q, a, mu = _cloud(300, 8.5, 2)
    assert _damped_pairs(X, a) > 20
    pq, Eq, Gq = D.charge_fields(X, q)
    pm, Eu, Ed, Gd = D.dipole_fields(X, mu, a, 2.0)
    phi, EU, ED, G = NT.fields(X, q, mu, a, 2.0)
    assert relmax(phi, pq + pm) < 1e-13
    assert relmax(EU, Eq + Eu) < 1e-13
    assert relmax(ED, Eq + Ed) < 1e-13
    assert relmax(G, Gq + Gd) < 1e-13
    # sources one type at a time
    c = NT.fields(X, q=q, alpha=a, thole_a=2.0)
    assert relmax(c[0], pq) < 1e-13 and relmax(c[1], Eq) < 1e-13 and relmax(c[2], Eq) < 1e-13
    d = NT.fields(X, mu=mu, alpha=a, thole_a=2.0)
    assert relmax(d[1], Eu) < 1e-13 and relmax(d[2], Ed) < 1e-13 and relmax(d[3], Gd) < 1e-13
    # sampled targets return the rows of the full evaluation
    tg = np.array([299, 0, 150, 5, 7])
    s = NT.fields(X, q, mu, a, 2.0, targets=tg)
    for full, part in zip((phi, EU, ED, G), s):
        assert relmax(part, full[tg]) < 1e-15
    # the product of the dipole solve is the dense tensor times the dipoles
    T = D.dipole_matrix(X, a, 2.0)
    Tmu = (T @ mu.reshape(-1)).reshape(-1, 3)
    assert relmax(NT.dipole_field(X, a, 2.0, mu), Tmu) < 1e-13
    assert relmax(NT.dipole_field(X, a, 2.0, mu, targets=tg), Tmu[tg]) < 1e-13


def test_native_forces_at_equal_dense_forces_at_solution():
    X, q, a, _ = _cloud(150, 6.5, 3)
    ref = D.solve(X, q, a, thole_a=2.0)
    tg = np.array([0, 5, 33, 149])
    F, res = NT.forces_at(X, q, ref["mu"], a, tg, thole_a=2.0)
    assert relmax(F, ref["F"][tg]) < 1e-12
    assert np.abs(res).max() < 1e-12 * np.abs(ref["mu"]).max()


@pytest.mark.slow
def test_native_solve_equals_dense_solve_2k():
    """Matrix-free CG with direct-sum products to 1e-13 vs dense LU of the scaled system: 2,000
    clumped particles at protein density (many damped pairs)."""
    from paper_1408_6527_amd import inputs
    ps = inputs.small_globular(2000)
    ref = D.solve(ps.pos, ps.q, ps.alpha, thole_a=2.0)
    o = NT.solve(ps.pos, ps.q, ps.alpha, thole_a=2.0, tol=1e-13)
    assert o["residual"] < 1e-12
    assert relnorm(o["mu"], ref["mu"]) < 1e-12
    assert relnorm(o["F"], ref["F"]) < 1e-12
    assert relnorm(o["phi"], ref["phi"]) < 1e-12
    for k in ("U", "U_qq", "U_pol"):
        assert abs(o[k] - ref[k]) < 1e-12 * abs(ref[k])


def test_native_two_charges_coulomb():
    X = np.array([[0.0, 0.0, 0.0], [1.0, 2.0, 2.0]])  # r = 3
    q = np.array([0.7, -1.3])
    o = NT.solve(X, q, np.zeros(2), thole_a=2.0)
    ke = D.COULOMB_K
    assert abs(o["U"] - ke * 0.7 * -1.3 / 3.0) < 1e-15 * ke
    rhat = X[1] / 3.0
    assert np.allclose(o["F"][1], ke * 0.7 * -1.3 * rhat / 9.0, rtol=1e-15, atol=0)
    assert np.allclose(o["F"][0], -o["F"][1], rtol=1e-15, atol=0)


def test_native_charge_and_polarisable_site():
    """Charge q at the origin, site of polarisability alpha at distance r (beyond the Thole radius):
    mu = alpha q r_hat / r^2, U^pol = -alpha q^2 / (2 r^4), radial force -2 alpha q^2 / r^5."""
    r, qq, al = 4.0, 0.9, 1.7
    X = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, r]])
    o = NT.solve(X, np.array([qq, 0.0]), np.array([0.0, al]), thole_a=2.0, tol=1e-14)
    ke = D.COULOMB_K
    assert np.allclose(o["mu"][1], [0, 0, al * qq / r**2], rtol=1e-14, atol=1e-17)
    assert abs(o["U_pol"] - ke * (-al * qq**2 / (2 * r**4))) < 1e-14 * abs(o["U_pol"])
    assert abs(o["F"][1, 2] - ke * (-2.0 * al * qq**2 / r**5)) < 1e-13 * abs(o["F"][1, 2])


@pytest.mark.parametrize("r,damped", [(3.1, False), (1.5, True)])
def test_native_two_polarisable_sites_closed_form(r, damped):
    """Two charged polarisable sites on the z axis: the dipoles solve the 2 x 2 system
    mu1 = a1 (E1 + c a2-coupled mu2), with the axial coupling c = (3 f_t - f_e) / r^3 of the tensor
    (c = 2 / r^3 undamped; f_e = 4v^3 - 3v^4, f_t = v^4 inside the Thole radius)."""
    a1, a2, q1, q2, ta = 1.3, 0.9, 0.7, -0.4, 2.0
    X = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, r]])
    s = ta * (a1 * a2) ** (1.0 / 6.0)
    assert (r < s) == damped
    if r < s:
        v = r / s
        c = (3 * v**4 - (4 * v**3 - 3 * v**4)) / r**3
    else:
        c = 2.0 / r**3
    E1 = -q2 / r**2  # field of q2 at site 1 along +z (site 2 is at +z)
    E2 = q1 / r**2
    det = 1.0 - c * c * a1 * a2
    m1 = a1 * (E1 + c * a2 * E2) / det
    m2 = a2 * (E2 + c * a1 * E1) / det
    o = NT.solve(X, np.array([q1, q2]), np.array([a1, a2]), thole_a=ta, tol=1e-15)
    assert abs(o["mu"][0, 2] - m1) < 1e-14 * abs(m1)
    assert abs(o["mu"][1, 2] - m2) < 1e-14 * abs(m2)
    assert np.abs(o["mu"][:, :2]).max() < 1e-17


def test_native_coincident_and_bad_arguments():
    X = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 0.0]])
    with pytest.raises(ValueError, match="coincident"):
        NT.fields(X, q=np.ones(3))
    with pytest.raises(ValueError):
        NT.fields(X[:2], q=np.ones(2), targets=[0, 2])
    assert NT.threads() >= 1
