"""Pins of the CPU oracle against closed forms, invariants, finite differences, brute force in
high precision and the FMM error decay.  None of these tests needs a GPU.

Each test names the passage of arXiv:1408.6527 it pins.
"""
import itertools
import math

import numpy as np
import pytest

from oracle import direct as D
from oracle import fmm as FM

K = 1.0  # work in Gaussian units inside the pins; k_e scaling is pinned separately


def rand_system(n, seed, box=8.0, r_min=1.2, qsd=0.5, alo=0.5, ahi=2.0):
    rng = np.random.default_rng(seed)
    pts = []
    while len(pts) < n:
        x = rng.uniform(0, box, 3)
        if all(np.linalg.norm(x - y) >= r_min for y in pts):
            pts.append(x)
    X = np.array(pts)
    q = rng.normal(0, qsd, n)
    a = rng.uniform(alo, ahi, n)
    return X, q, a


# ---------------------------------------------------------------- closed forms (Sec. II.A)

def test_two_charges_closed_form():
    """U^{qq'} of two charges and the Coulomb force (Sec. II.A, U^{qq'} equation)."""
    X = np.array([[0.3, -0.2, 0.1], [1.9, 2.4, -0.8]])
    q = np.array([0.7, -1.3])
    out = D.solve(X, q, np.zeros(2), thole_a=2.0, k_e=D.COULOMB_K)
    r = np.linalg.norm(X[0] - X[1])
    assert out["U"] == pytest.approx(D.COULOMB_K * q[0] * q[1] / r, rel=1e-15)
    F0 = D.COULOMB_K * q[0] * q[1] * (X[0] - X[1]) / r**3
    assert np.allclose(out["F"][0], F0, rtol=1e-14, atol=0)
    assert np.allclose(out["F"][1], -F0, rtol=1e-14, atol=0)
    assert np.allclose(out["mu"], 0.0)


def test_charge_and_polarizable_site():
    """A charge next to one polarisable site: mu = alpha q r/r^3, U^pol = -alpha q^2/(2 r^4), attractive
    radial force 2 alpha q^2 / r^5 (Sec. II.A, dipole-moment and U^pol equations)."""
    q0, alpha, r = 0.9, 1.7, 3.3
    X = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, r]])
    out = D.solve(X, np.array([q0, 0.0]), np.array([0.0, alpha]), thole_a=2.0, k_e=1.0)
    assert np.allclose(out["mu"][1], [0, 0, alpha * q0 / r**2], rtol=1e-14)
    assert out["U_pol"] == pytest.approx(-alpha * q0**2 / (2 * r**4), rel=1e-14)
    assert out["F"][1][2] == pytest.approx(-2 * alpha * q0**2 / r**5, rel=1e-13)
    assert out["F"][0][2] == pytest.approx(2 * alpha * q0**2 / r**5, rel=1e-13)


@pytest.mark.parametrize("r,damped", [(3.1, False), (3.1, True), (1.4, True)])
def test_two_polarizable_sites_on_axis(r, damped):
    """Two charged polarisable sites on the z axis solve a 2x2 system in closed form:
    mu_1 = alpha_1 (E_1 + c alpha_2 E_2) / (1 - c^2 alpha_1 alpha_2) with c = (3 f_t - f_e)/r^3
    (c = 2/r^3 undamped).  Sec. II.A, dipole-moment equation; the Thole damping form is the
    linear model read for Sec. II.A."""
    q = np.array([0.7, -0.4]); a = np.array([1.3, 0.9])
    X = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, r]])
    thole = 2.0 if damped else 0.0
    out = D.solve(X, q, a, thole_a=thole, k_e=1.0)
    E1 = -q[1] / r**2   # field at site 1 (z component) from charge 2
    E2 = q[0] / r**2
    s = thole * (a[0] * a[1]) ** (1 / 6)
    v = min(r / s, 1.0) if s > 0 else 1.0
    ft, fe = v**4, 4 * v**3 - 3 * v**4
    c = (3 * ft - fe) / r**3
    mu1 = a[0] * (E1 + c * a[1] * E2) / (1 - c * c * a[0] * a[1])
    mu2 = a[1] * (E2 + c * a[0] * E1) / (1 - c * c * a[0] * a[1])
    assert out["mu"][0][2] == pytest.approx(mu1, rel=1e-14)
    assert out["mu"][1][2] == pytest.approx(mu2, rel=1e-14)
    assert np.allclose(out["mu"][:, :2], 0.0, atol=1e-16)
    if damped and r == 1.4:
        assert r < s  # the damped branch is exercised
    Upol = -0.5 * (mu1 * E1 + mu2 * E2)
    assert out["U_pol"] == pytest.approx(Upol, rel=1e-13)


def test_two_site_exact_rational_value():
    """An independent numeric value of the undamped two-site system (q = 0.7/-0.4, alpha = 1.3/0.9,
    r = 3.1) recomputed from the 2x2 closed form with exact rational steps."""
    from fractions import Fraction as Fr
    r = Fr(31, 10); q1, q2 = Fr(7, 10), Fr(-4, 10); a1, a2 = Fr(13, 10), Fr(9, 10)
    E1 = -q2 / r**2; E2 = q1 / r**2; c = 2 / r**3
    mu1 = a1 * (E1 + c * a2 * E2) / (1 - c * c * a1 * a2)
    X = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 3.1]])
    out = D.solve(X, np.array([0.7, -0.4]), np.array([1.3, 0.9]), thole_a=0.0, k_e=1.0)
    assert out["mu"][0][2] == pytest.approx(float(mu1), rel=1e-14)


# ---------------------------------------------------------------- derivative tensor (App. D, Sec. II.B)

def test_derivative_tensor_against_sympy():
    """D_n(R) = d^n (1/|R|) from the recurrence equals symbolic differentiation up to degree 10."""
    sp = pytest.importorskip("sympy")
    x, y, z = sp.symbols("x y z", real=True)
    f = 1 / sp.sqrt(x**2 + y**2 + z**2)
    R = np.array([[0.7, -1.3, 2.1]])
    P = 10
    Dn = FM.derivative_tensor(R, P)[0]
    mi = FM.MultiIndex(P)
    vals = {x: sp.Rational(7, 10), y: sp.Rational(-13, 10), z: sp.Rational(21, 10)}
    worst = 0.0
    for k, (a, b, c) in enumerate(mi.items):
        expr = f
        if a: expr = sp.diff(expr, x, a)
        if b: expr = sp.diff(expr, y, b)
        if c: expr = sp.diff(expr, z, c)
        ref = float(sp.N(expr.subs(vals), 30))
        if ref != 0:
            worst = max(worst, abs(Dn[k] - ref) / abs(ref))
        else:
            assert abs(Dn[k]) < 1e-12
    assert worst < 1e-12


def test_derivative_tensor_homogeneity():
    """D_n(w d) = w^-(|n|+1) D_n(d): the scaling used to share one table across tree levels."""
    d = np.array([[2.0, -1.0, 3.0]])
    w = 3.75
    P = 8
    mi = FM.MultiIndex(P)
    a = FM.derivative_tensor(w * d, P)[0]
    b = FM.derivative_tensor(d, P)[0] * w ** (-(mi.deg + 1.0))
    assert np.allclose(a, b, rtol=1e-13, atol=0)


# ---------------------------------------------------------------- FMM operators (Sec. II.B-II.C)

def _cell(seed, n=6, h=0.5):
    rng = np.random.default_rng(seed)
    return rng.uniform(-h, h, (n, 3)), rng.normal(0, 1, n), rng.normal(0, 0.3, (n, 3))


def test_m2m_is_exact_shift():
    """M2M of a child expansion equals P2M taken directly about the parent centre (exact identity)."""
    X, q, mu = _cell(1)
    p = 7
    zc = np.array([0.1, -0.2, 0.05]); zp = np.array([0.6, 0.3, -0.45])
    Mc = FM.p2m(p, zc, X, q, mu)
    Mp = FM.p2m(p, zp, X, q, mu)
    assert np.allclose(FM.m2m(p, Mc, zp - zc), Mp, rtol=1e-12, atol=1e-13)


def test_l2l_preserves_local_polynomial():
    """L2L re-expands the degree-p local polynomial exactly: L2P before and after agree."""
    rng = np.random.default_rng(3)
    p = 6
    F = rng.normal(size=FM.ncoef(p))
    zp = np.zeros(3); zc = np.array([0.25, -0.25, 0.25])
    Fc = FM.l2l(p, F, zc - zp)
    pts = zc + rng.uniform(-0.2, 0.2, (5, 3))
    a = FM.l2p(p, F, zp, pts)
    b = FM.l2p(p, Fc, zc, pts)
    for u, v in zip(a, b):
        assert np.allclose(u, v, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("with_dipoles", [False, True])
def test_single_interaction_converges_to_direct(with_dipoles):
    """P2M -> M2L -> L2P between two separated cells approaches the direct potential, field and field
    gradient, with an error falling geometrically in p (Sec. II.B two-centre expansion; dipoles as
    the delta-l -> 0 limit of Sec. II.C)."""
    X, q, mu = _cell(5)
    mu = mu if with_dipoles else None
    zA = np.zeros(3); zB = np.array([4.2, -2.6, 3.4])
    T = zB + np.random.default_rng(6).uniform(-0.5, 0.5, (4, 3))
    # direct
    phi = np.zeros(4); E = np.zeros((4, 3)); G = np.zeros((4, 3, 3))
    for i in range(4):
        rv = T[i] - X
        g, grad, H, T3 = D.hessian_and_third(rv)
        phi[i] = np.sum(q * g); E[i] = -np.sum(q[:, None] * grad, 0); G[i] = -np.sum(q[:, None, None] * H, 0)
        if mu is not None:
            phi[i] -= np.sum(mu * grad); E[i] += np.einsum("jab,jb->a", H, mu)
            G[i] += np.einsum("jabc,jc->ab", T3, mu)
    errs = []
    for p in (2, 4, 6, 8, 10):
        M = FM.p2m(p, zA, X, q, mu)
        F = FM.m2l(p, M[None], (zB - zA)[None])[0]
        ph, Ef, Gf = FM.l2p(p, F, zB, T)
        errs.append(max(np.abs(ph - phi).max() / np.abs(phi).max(),
                        np.abs(Ef - E).max() / np.abs(E).max(),
                        np.abs(Gf - G).max() / np.abs(G).max()))
    assert errs[-1] < 1e-4
    assert all(errs[i + 1] < errs[i] for i in range(len(errs) - 1))


def test_dipole_limit_matches_charge_pair():
    """The point-dipole P2M equals the +/- q^mu pair of Sec. II.C as delta-l -> 0 (error O(delta-l^2))."""
    p = 6
    rng = np.random.default_rng(9)
    x = rng.uniform(-0.4, 0.4, (1, 3)); mu = rng.normal(size=(1, 3))
    Mpt = FM.p2m(p, np.zeros(3), x, None, mu)
    errs = []
    for dl in (1e-2, 1e-3):
        u = mu[0] / np.linalg.norm(mu[0])
        qmu = np.linalg.norm(mu[0]) / (2 * dl)  # mu = 2 |q^mu| delta-l
        Xp = np.array([x[0] + dl * u, x[0] - dl * u])
        Mpair = FM.p2m(p, np.zeros(3), Xp, np.array([qmu, -qmu]))
        errs.append(np.abs(Mpair - Mpt).max())
    assert errs[1] < errs[0] / 50  # quadratic convergence in delta-l


def test_pair_p2m_axis_closed_form():
    """A dipole mu_a e_a at the expansion centre, taken as the +/- q^mu pair of Sec. II.C (charges
    +/- |mu| / (2 dl) at +/- dl mu/|mu|, so mu = 2 |q^mu| delta-l), has at any finite dl the
    multipoles M_{k e_a} = (-1)^k / k! q^mu (dl^k - (-dl)^k) s^k, s = sign(mu_a): -mu_a dl^(k-1) / k!
    for odd k, zero for even k and for every mixed multi-index."""
    p = 7
    items = FM._mi(p).items
    for a in range(3):
        for sgn in (1.0, -1.0):
            mu = np.zeros(3); mu[a] = 0.8 * sgn
            for dl in (0.3, 1e-2):
                M = FM.p2m_pair(p, np.zeros(3), np.zeros((1, 3)), mu[None], dl)
                expect = np.zeros(len(items))
                for k, n in enumerate(items):
                    if n[a] == sum(n) and n[a] % 2 == 1:
                        expect[k] = -mu[a] * dl ** (n[a] - 1) / math.factorial(n[a])
                np.testing.assert_allclose(M, expect, rtol=1e-13, atol=1e-15)


def test_pair_p2m_tends_to_point_dipole():
    """The pair multipoles approach the point-dipole P2M quadratically in dl (Sec. II.C: the point
    dipole is the pair's dl -> 0 limit); a zero dipole has no pair and adds nothing."""
    p = 6
    rng = np.random.default_rng(19)
    X = rng.uniform(-0.4, 0.4, (3, 3)); mu = rng.normal(size=(3, 3)); mu[1] = 0.0
    Mpt = FM.p2m(p, np.zeros(3), X, None, mu)
    errs = [np.abs(FM.p2m_pair(p, np.zeros(3), X, mu, dl) - Mpt).max() for dl in (1e-2, 1e-3)]
    assert 80 < errs[0] / errs[1] < 120
    assert not np.any(FM.p2m_pair(p, np.zeros(3), X, np.zeros((3, 3)), 1e-4))


def test_fmm_pair_dipoles_insensitive_to_dl():
    """FMM fields with the dipole multipoles built from the +/- q^mu pairs (order 5, as in the
    paper's sphere tests): for dl = 1e-5 .. 1e-3 A they differ from the point-dipole FMM by far less
    than the FMM's own error against the direct sums, so that error does not change with dl (the
    paper's finding over five decades of dl); the departure grows as dl^2."""
    X, q, a = rand_system(300, 83, box=14.0, r_min=1.0)
    mu = np.random.default_rng(5).normal(0, 0.2, (300, 3))
    _, Eq, _ = D.charge_fields(X, q)
    _, _, Ed, _ = D.dipole_fields(X, mu, a, 2.0)
    ref = Eq + Ed
    base = FM.fmm_fields(X, q, mu, a, 2.0, 5, 1.7, 1, want_grad=False)["E_d"]
    assert FM.Octree(X, 1.7, 1).L >= 3
    e0 = np.linalg.norm(base - ref) / np.linalg.norm(ref)
    dev = {}
    for dl in (1e-5, 1e-4, 1e-3, 1e-2):
        E = FM.fmm_fields(X, q, mu, a, 2.0, 5, 1.7, 1, want_grad=False, pair_dl=dl)["E_d"]
        dev[dl] = np.linalg.norm(E - base) / np.linalg.norm(ref)
        e = np.linalg.norm(E - ref) / np.linalg.norm(ref)
        if dl <= 1e-3:
            assert dev[dl] < 1e-4 * e0 and abs(e - e0) < 1e-4 * e0
    assert 60 < dev[1e-2] / dev[1e-3] < 140


# ---------------------------------------------------------------- identities and invariants

def test_energy_identity_at_convergence():
    """U^pol = A - sum Phi^{mu q} - 1/2 sum Phi^{mu mu} equals -1/2 sum mu.E^q at the solution
    (Sec. II.A, U^pol equation with the linear dipole equation)."""
    X, q, a = rand_system(9, 11)
    out = D.solve(X, q, a, thole_a=2.0, k_e=1.0)
    assert out["U_pol"] == pytest.approx(-0.5 * np.sum(out["mu"] * out["E_q"]), rel=1e-13)


@pytest.mark.parametrize("thole", [0.0, 2.0])
def test_newton_third_law_and_torque(thole):
    """Zero net force and zero net torque for an isolated system (momentum conservation,
    Sec. II.B and Sec. IV.B).  The torque includes mu x E since dipoles carry torque; with isotropic
    alpha, mu is parallel to E, so sum x_i x F_i = 0."""
    X, q, a = rand_system(12, 12)
    out = D.solve(X, q, a, thole_a=thole, k_e=1.0)
    F = out["F"]
    scale = np.abs(F).sum()
    assert np.abs(F.sum(0)).max() < 1e-12 * scale
    assert np.abs(np.cross(X, F).sum(0)).max() < 1e-12 * scale * np.abs(X).max()


def test_translation_rotation_scaling_invariance():
    """U is invariant under translation and rotation, forces and dipoles rotate with the system, and
    U(lambda X, q, lambda^3 alpha) = U / lambda (the damping radius scales with lambda)."""
    X, q, a = rand_system(8, 13)
    base = D.solve(X, q, a, thole_a=2.0, k_e=1.0)
    t = np.array([3.3, -7.1, 0.4])
    tr = D.solve(X + t, q, a, thole_a=2.0, k_e=1.0)
    assert tr["U"] == pytest.approx(base["U"], rel=1e-12)
    assert np.allclose(tr["F"], base["F"], rtol=1e-10, atol=1e-12)
    th = 0.7
    Rz = np.array([[math.cos(th), -math.sin(th), 0], [math.sin(th), math.cos(th), 0], [0, 0, 1]])
    Rx = np.array([[1, 0, 0], [0, math.cos(1.1), -math.sin(1.1)], [0, math.sin(1.1), math.cos(1.1)]])
    Rm = Rz @ Rx
    ro = D.solve(X @ Rm.T, q, a, thole_a=2.0, k_e=1.0)
    assert ro["U"] == pytest.approx(base["U"], rel=1e-12)
    assert np.allclose(ro["F"], base["F"] @ Rm.T, rtol=1e-10, atol=1e-12)
    assert np.allclose(ro["mu"], base["mu"] @ Rm.T, rtol=1e-10, atol=1e-13)
    lam = 1.37
    sc = D.solve(lam * X, q, lam**3 * a, thole_a=2.0, k_e=1.0)
    assert sc["U"] == pytest.approx(base["U"] / lam, rel=1e-12)


# ---------------------------------------------------------------- finite differences (stationarity, Sec. II.A/II.C)

@pytest.mark.parametrize("thole", [0.0, 2.0])
def test_forces_potentials_alpha_gradients_by_finite_differences(thole):
    """F = -dU/dx, phi = dU/dq and the dU/dalpha formula, at fixed converged dipoles, agree with
    central differences of the energy at re-converged dipoles (stationarity dU^pol/dmu = 0)."""
    X, q, a = rand_system(7, 21 if thole else 22, box=5.0, r_min=1.0)
    out = D.solve(X, q, a, thole_a=thole, k_e=1.0)
    if thole:
        r = np.linalg.norm(X[:, None] - X[None], axis=2)
        s = thole * np.cbrt(np.sqrt(a[:, None] * a[None]))
        assert ((r < s) & (r > 0)).sum() >= 2  # damped pairs exist
    h = 1e-5
    E = lambda X_, q_, a_: D.energy_only(X_, q_, a_, thole, 1.0)
    n = X.shape[0]
    Ffd = np.zeros((n, 3)); gq = np.zeros(n); ga = np.zeros(n)
    for i in range(n):
        for c in range(3):
            Xp = X.copy(); Xp[i, c] += h; Xm = X.copy(); Xm[i, c] -= h
            Ffd[i, c] = -(E(Xp, q, a) - E(Xm, q, a)) / (2 * h)
        qp = q.copy(); qp[i] += h; qm = q.copy(); qm[i] -= h
        gq[i] = (E(X, qp, a) - E(X, qm, a)) / (2 * h)
        ap = a.copy(); ap[i] += h; am = a.copy(); am[i] -= h
        ga[i] = (E(X, q, ap) - E(X, q, am)) / (2 * h)
    assert np.linalg.norm(Ffd - out["F"]) / np.linalg.norm(Ffd) < 1e-7
    assert np.linalg.norm(gq - out["phi"]) / np.linalg.norm(gq) < 1e-8
    assert np.linalg.norm(ga - out["grad_alpha"]) / np.linalg.norm(ga) < 1e-7


def test_field_charges_two_sites_closed_form():
    """Separate charges q^E for the polarising field (Sec. III): on the z axis the dipoles follow
    the 2x2 closed form with E_1 = -qE_2/r^2, E_2 = qE_1/r^2, and U = q_1 q_2 / r - 1/2 (mu_1 E_1 +
    mu_2 E_2); with q^E = q it is the plain system."""
    q = np.array([0.7, -0.4]); qE = np.array([-0.3, 0.5]); a = np.array([1.3, 0.9]); r = 3.1
    X = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, r]])
    out = D.solve(X, q, a, thole_a=0.0, k_e=1.0, qE=qE)
    E1, E2, c = -qE[1] / r**2, qE[0] / r**2, 2 / r**3
    mu1 = a[0] * (E1 + c * a[1] * E2) / (1 - c * c * a[0] * a[1])
    mu2 = a[1] * (E2 + c * a[0] * E1) / (1 - c * c * a[0] * a[1])
    assert out["mu"][0][2] == pytest.approx(mu1, rel=1e-14)
    assert out["mu"][1][2] == pytest.approx(mu2, rel=1e-14)
    assert out["U"] == pytest.approx(q[0] * q[1] / r - 0.5 * (mu1 * E1 + mu2 * E2), rel=1e-13)
    tied = D.solve(X, q, a, thole_a=0.0, k_e=1.0)
    same = D.solve(X, q, a, thole_a=0.0, k_e=1.0, qE=q.copy())
    assert same["U"] == pytest.approx(tied["U"], rel=1e-15)
    assert np.allclose(same["F"], tied["F"], rtol=1e-14, atol=0)
    assert np.allclose(same["phi"] + same["phi_E"], tied["phi"], rtol=1e-14, atol=0)


def test_zero_field_charges_leave_coulomb():
    """With every q^E zero no atom generates the polarising field: mu = 0, U = U^qq, F = q E^q."""
    X, q, a = rand_system(8, 31)
    out = D.solve(X, q, a, thole_a=2.0, k_e=1.0, qE=np.zeros_like(q))
    assert not np.any(out["mu"])
    phi, E, _ = D.charge_fields(X, q)
    assert out["U"] == pytest.approx(0.5 * np.sum(q * phi), rel=1e-14)
    assert np.allclose(out["F"], q[:, None] * E, rtol=1e-14, atol=0)


@pytest.mark.parametrize("thole", [0.0, 2.0])
def test_field_charges_gradients_by_finite_differences(thole):
    """With q^E != q: F = -dU/dx, dU/dq = phi, dU/dqE = phi_E = phi^mu and dU/dalpha agree with
    central differences of the energy at re-converged dipoles."""
    X, q, a = rand_system(6, 41 if thole else 42, box=5.0, r_min=1.0)
    qE = np.random.default_rng(43).normal(0, 0.6, q.size)
    out = D.solve(X, q, a, thole_a=thole, k_e=1.0, qE=qE)
    h = 1e-5
    E = lambda X_, q_, e_, a_: D.energy_only(X_, q_, a_, thole, 1.0, qE=e_)
    n = X.shape[0]
    Ffd = np.zeros((n, 3)); gq = np.zeros(n); ge = np.zeros(n); ga = np.zeros(n)
    for i in range(n):
        for c in range(3):
            Xp = X.copy(); Xp[i, c] += h; Xm = X.copy(); Xm[i, c] -= h
            Ffd[i, c] = -(E(Xp, q, qE, a) - E(Xm, q, qE, a)) / (2 * h)
        d = np.zeros(n); d[i] = h
        gq[i] = (E(X, q + d, qE, a) - E(X, q - d, qE, a)) / (2 * h)
        ge[i] = (E(X, q, qE + d, a) - E(X, q, qE - d, a)) / (2 * h)
        ga[i] = (E(X, q, qE, a + d) - E(X, q, qE, a - d)) / (2 * h)
    assert np.linalg.norm(Ffd - out["F"]) / np.linalg.norm(Ffd) < 1e-7
    assert np.linalg.norm(gq - out["phi"]) / np.linalg.norm(gq) < 1e-8
    assert np.linalg.norm(ge - out["phi_E"]) / np.linalg.norm(ge) < 1e-8
    assert np.linalg.norm(ga - out["grad_alpha"]) / np.linalg.norm(ga) < 1e-7


def test_exclusions_three_sites_closed_form():
    """Three sites on the z axis with the pair (0, 1) excluded (the starred sums of Sec. II.A):
    the charge energy keeps q0 q2 / r02 + q1 q2 / r12, site 2 is polarised by q0 and q1, sites 0 and
    1 by q2 only, and the dipoles couple 0-2 and 1-2 only (undamped on-axis coupling 2 / r^3), a
    3 x 3 linear system; U = U^qq - 1/2 sum mu E^q."""
    z = np.array([0.0, 2.2, 5.1]); q = np.array([0.6, -0.5, 0.3]); a = np.array([1.1, 0.7, 1.6])
    X = np.stack([np.zeros(3), np.zeros(3), z], axis=1)
    out = D.solve(X, q, a, thole_a=0.0, k_e=1.0, excl=[(0, 1)])
    r02, r12 = z[2] - z[0], z[2] - z[1]
    E = np.array([-q[2] / r02**2, -q[2] / r12**2, q[0] / r02**2 + q[1] / r12**2])
    C = np.zeros((3, 3))
    C[0, 2] = C[2, 0] = 2 / r02**3
    C[1, 2] = C[2, 1] = 2 / r12**3
    mu = np.linalg.solve(np.eye(3) - a[:, None] * C, a * E)
    np.testing.assert_allclose(out["mu"][:, 2], mu, rtol=1e-13)
    assert np.allclose(out["mu"][:, :2], 0.0, atol=1e-16)
    U = q[0] * q[2] / r02 + q[1] * q[2] / r12 - 0.5 * np.sum(mu * E)
    assert out["U"] == pytest.approx(U, rel=1e-13)


def test_excluding_every_pair_removes_all_interactions():
    X, q, a = rand_system(6, 51)
    allp = [(i, j) for i in range(6) for j in range(i + 1, 6)]
    out = D.solve(X, q, a, thole_a=2.0, k_e=1.0, excl=allp)
    assert out["U"] == 0.0 and not np.any(out["mu"]) and not np.any(out["F"]) and not np.any(out["phi"])


@pytest.mark.parametrize("thole", [0.0, 2.0])
def test_exclusions_gradients_by_finite_differences(thole):
    """With a chain of bonded (1-2) and angle (1-3) exclusions, F = -dU/dx, dU/dq = phi and
    dU/dalpha agree with central differences of the energy at re-converged dipoles."""
    X, q, a = rand_system(7, 52 if thole else 53, box=5.0, r_min=1.0)
    excl = [(i, i + 1) for i in range(6)] + [(i, i + 2) for i in range(5)]
    out = D.solve(X, q, a, thole_a=thole, k_e=1.0, excl=excl)
    h = 1e-5
    E = lambda X_, q_, a_: D.energy_only(X_, q_, a_, thole, 1.0, excl=excl)
    n = X.shape[0]
    Ffd = np.zeros((n, 3)); gq = np.zeros(n); ga = np.zeros(n)
    for i in range(n):
        for c in range(3):
            Xp = X.copy(); Xp[i, c] += h; Xm = X.copy(); Xm[i, c] -= h
            Ffd[i, c] = -(E(Xp, q, a) - E(Xm, q, a)) / (2 * h)
        d = np.zeros(n); d[i] = h
        gq[i] = (E(X, q + d, a) - E(X, q - d, a)) / (2 * h)
        ga[i] = (E(X, q, a + d) - E(X, q, a - d)) / (2 * h)
    assert np.linalg.norm(Ffd - out["F"]) / np.linalg.norm(Ffd) < 1e-7
    assert np.linalg.norm(gq - out["phi"]) / np.linalg.norm(gq) < 1e-8
    assert np.linalg.norm(ga - out["grad_alpha"]) / np.linalg.norm(ga) < 1e-7


def test_fmm_exclusions_match_direct():
    """The FMM with exclusions: with one leaf it is the direct sum with the pairs left out (to
    rounding); on a deeper tree it differs from it by the FMM's truncation error only."""
    X, q, a = rand_system(120, 54, box=9.0, r_min=1.0)
    mu = np.random.default_rng(55).normal(0, 0.2, (120, 3))
    excl = [(i, i + 1) for i in range(119)] + [(3, 60), (7, 100)]
    _, Eq, Gq = D.charge_fields(X, q, excl=excl)
    ph, Eu, Ed, Gd = D.dipole_fields(X, mu, a, 2.0, excl=excl)
    one = FM.fmm_fields(X, q, mu, a, 2.0, 4, 100.0, 1, excl=excl)
    assert one["tree"].L == 0
    assert np.abs(one["E_d"] - (Eq + Ed)).max() < 1e-12 * np.abs(Eq + Ed).max()
    assert np.abs(one["G_d"] - (Gq + Gd)).max() < 1e-12 * np.abs(Gq + Gd).max()
    deep = FM.fmm_fields(X, q, mu, a, 2.0, 6, 1.5, 2, excl=excl)
    plain = FM.fmm_fields(X, q, mu, a, 2.0, 6, 1.5, 2)
    assert deep["tree"].L >= 3
    err = np.linalg.norm(deep["E_d"] - (Eq + Ed)) / np.linalg.norm(Eq + Ed)
    err_plain = np.linalg.norm(plain["E_d"] - (Eq + Ed)) / np.linalg.norm(Eq + Ed)
    assert err < 1e-3 < err_plain  # the exclusions are really applied


def test_alpha_gradient_at_zero_polarizability():
    """For alpha_i = 0 the gradient is -|E_i|^2/2 (the limit of -|mu|^2/(2 alpha^2) with mu = alpha E)."""
    X, q, a = rand_system(6, 31)
    a[2] = 0.0
    out = D.solve(X, q, a, thole_a=2.0, k_e=1.0)
    h = 1e-6
    ap = a.copy(); ap[2] += h
    fd = (D.energy_only(X, q, ap, 2.0, 1.0) - D.energy_only(X, q, a, 2.0, 1.0)) / h
    assert out["grad_alpha"][2] == pytest.approx(fd, rel=1e-4)
    assert np.allclose(out["mu"][2], 0.0)


# ---------------------------------------------------------------- limits

def test_zero_polarizability_is_pure_coulomb():
    X, q, a = rand_system(10, 41)
    out = D.solve(X, q, np.zeros_like(a), thole_a=2.0, k_e=1.0)
    U = sum(q[i] * q[j] / np.linalg.norm(X[i] - X[j]) for i in range(10) for j in range(i + 1, 10))
    assert out["U"] == pytest.approx(U, rel=1e-13)
    assert out["U_pol"] == 0.0


def test_vanishing_thole_constant_is_undamped():
    X, q, a = rand_system(6, 42, box=4.0, r_min=1.0)
    T0 = D.dipole_matrix(X, a, 0.0)
    Tt = D.dipole_matrix(X, a, 1e-9)
    assert np.allclose(T0, Tt, rtol=1e-15, atol=0)
    Td = D.dipole_matrix(X, a, 2.0)
    assert not np.allclose(T0, Td)


def test_coulomb_constant_scaling():
    X, q, a = rand_system(5, 43)
    u1 = D.solve(X, q, a, 2.0, k_e=1.0)
    uk = D.solve(X, q, a, 2.0, k_e=D.COULOMB_K)
    assert uk["U"] == pytest.approx(D.COULOMB_K * u1["U"], rel=1e-14)
    assert np.allclose(uk["F"], D.COULOMB_K * u1["F"], rtol=1e-14)
    assert np.allclose(uk["mu"], u1["mu"], rtol=1e-14)


# ---------------------------------------------------------------- brute force in high precision

def test_brute_force_mpmath_tiny():
    """N = 3: fields built by high-precision numerical differentiation of the (smeared) potentials and
    a 50-digit linear solve reproduce the FP64 oracle's dipoles and energy."""
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 50
    X = np.array([[0.0, 0.0, 0.0], [1.6, 0.4, -0.3], [0.2, 1.9, 1.1]])
    q = np.array([0.6, -0.25, -0.35]); a = np.array([1.1, 1.8, 0.7]); thole = 2.0
    Xm = [[mp.mpf(float(v)) for v in row] for row in X]

    def g_smeared(r, s):
        if s > 0 and r < s:
            v = r / s
            return (2 - 2 * v**2 + v**3) / s
        return 1 / r

    def pot(x, j, s):  # potential at point x of a unit (smeared) charge at particle j
        r = mp.sqrt(sum((x[c] - Xm[j][c]) ** 2 for c in range(3)))
        return g_smeared(r, s)

    n = 3
    Eq = [[mp.mpf(0)] * 3 for _ in range(n)]
    for i in range(n):
        for j in range(n):
            if i == j:
                continue
            for c in range(3):
                f = lambda t, c=c: pot([Xm[i][k] + (t if k == c else 0) for k in range(3)], j, 0)
                Eq[i][c] -= mp.mpf(float(q[j])) * mp.diff(f, 0)
    A = mp.zeros(3 * n, 3 * n)
    for i in range(n):
        for c in range(3):
            A[3 * i + c, 3 * i + c] = 1 / mp.mpf(float(a[i]))
    for i in range(n):
        for j in range(n):
            if i == j:
                continue
            s = mp.mpf(thole) * (mp.mpf(float(a[i])) * mp.mpf(float(a[j]))) ** (mp.mpf(1) / 6)
            for c in range(3):
                for d in range(3):
                    def f2(t1, t2, c=c, d=d):
                        x = list(Xm[i]); x[c] += t1; x[d] += t2
                        return pot(x, j, s)
                    H = mp.diff(f2, (0, 0), (1, 1))
                    A[3 * i + c, 3 * j + d] = -H
    b = mp.matrix([Eq[i][c] for i in range(n) for c in range(3)])
    mu = mp.lu_solve(A, b)
    phi = [sum(mp.mpf(float(q[j])) / mp.sqrt(sum((Xm[i][c] - Xm[j][c]) ** 2 for c in range(3)))
               for j in range(n) if j != i) for i in range(n)]
    U = sum(mp.mpf(float(q[i])) * phi[i] for i in range(n)) / 2 - sum(mu[k] * b[k] for k in range(3 * n)) / 2
    out = D.solve(X, q, a, thole_a=thole, k_e=1.0)
    r = np.linalg.norm(X[:, None] - X[None], axis=2)
    s = thole * np.cbrt(np.sqrt(a[:, None] * a[None]))
    assert ((r < s) & (r > 0)).any()  # a damped pair is included
    assert out["U"] == pytest.approx(float(U), rel=1e-13)
    assert np.allclose(out["mu"].reshape(-1), [float(v) for v in mu], rtol=1e-12, atol=1e-15)


# ---------------------------------------------------------------- solvers

def test_dense_and_conjugate_gradient_agree():
    """The conjugate-gradient dipole solve on the scaled system reaches the dense solution."""
    X, q, a = rand_system(25, 51, box=9.0, r_min=1.0)
    a[3] = 0.0
    _, Eq, _ = D.charge_fields(X, q, want_grad=False)
    mu_d = D.solve_dipoles_dense(X, q, a, 2.0, E_q=Eq)
    T = D.dipole_matrix(X, a, 2.0)
    mu_c, it, res = D.cg_scaled(lambda m: (T @ m.reshape(-1)).reshape(-1, 3), Eq, a, tol=1e-13)
    assert res <= 1e-13 and it < 75
    assert np.allclose(mu_c, mu_d, rtol=1e-10, atol=1e-13)
    assert np.all(mu_c[3] == 0.0)


def test_fmm_error_decays_with_order_and_separation():
    """FMM fields approach the direct sums geometrically in p and faster with the wider separation
    ws = 2 (Sec. III, accuracy controlled by the expansion order and the separation parameter)."""
    rng = np.random.default_rng(61)
    n = 300
    X = rng.uniform(0, 14, (n, 3)); q = rng.normal(0, 0.4, n); q -= q.mean()
    a = rng.uniform(0.5, 2.0, n); mu = rng.normal(0, 0.1, (n, 3))
    phq, Eq, Gq = D.charge_fields(X, q)
    _, Eu, Ed, Gd = D.dipole_fields(X, mu, a, 2.0)
    ref = Eq + Ed
    errs = {}
    for ws in (1, 2):
        for p in (2, 4, 6):
            o = FM.fmm_fields(X, q, mu, a, 2.0, p, 2.0, ws)
            assert o["tree"].L == 3
            errs[(ws, p)] = np.linalg.norm(o["E_d"] - ref) / np.linalg.norm(ref)
    for ws in (1, 2):
        assert errs[(ws, 4)] < errs[(ws, 2)] / 2.5 and errs[(ws, 6)] < errs[(ws, 4)] / 2.5
    for p in (2, 4, 6):
        assert errs[(2, p)] < errs[(1, p)] / 3
    assert errs[(2, 6)] < 2e-4


def test_fmm_single_level_is_direct():
    """With the whole system in one leaf every pair is direct: FMM fields equal the direct sums."""
    X, q, a = rand_system(20, 71, box=6.0, r_min=1.0)
    mu = np.random.default_rng(7).normal(0, 0.2, (20, 3))
    o = FM.fmm_fields(X, q, mu, a, 2.0, 4, 100.0, 1)
    assert o["tree"].L == 0
    phq, Eq, Gq = D.charge_fields(X, q)
    phm, Eu, Ed, Gd = D.dipole_fields(X, mu, a, 2.0)
    assert np.allclose(o["phi"], phq + phm, rtol=1e-13, atol=1e-13)
    assert np.allclose(o["E_d"], Eq + Ed, rtol=1e-13, atol=1e-13)
    assert np.allclose(o["E_u"], Eq + Eu, rtol=1e-13, atol=1e-13)
    assert np.allclose(o["G_d"], Gq + Gd, rtol=1e-13, atol=1e-13)


def test_fmm_pair_accounting_is_complete():
    """Every ordered particle pair is covered exactly once, by the near field or by one M2L."""
    rng = np.random.default_rng(81)
    X = rng.uniform(0, 17, (150, 3))
    for ws in (1, 2):
        t = FM.Octree(X, 1.9, ws)
        cover = np.zeros((150, 150), int)
        for B, A in t.near_pairs():
            for i in t.leaves[B]:
                for j in t.leaves[A]:
                    cover[i, j] += 1
        for l in range(1, t.L + 1):
            sh = t.L - l
            members = {}
            for cc, idx in t.leaves.items():
                members.setdefault((cc[0] >> sh, cc[1] >> sh, cc[2] >> sh), []).extend(idx)
            for B, A in t.m2l_pairs(l):
                for i in members[B]:
                    for j in members[A]:
                        cover[i, j] += 1
        assert np.all(cover == 1)


# ------------------------------------------------------------------ per-offset truncation order

def _offsets(ws):
    """Every M2L offset d = oB - c - 2e of the ws lists, over all target octants."""
    out = set()
    for o in range(8):
        ob = ((o >> 2) & 1, (o >> 1) & 1, o & 1)
        for t in itertools.product(range(-2 * ws, 2 * ws + 2), repeat=3):
            d = tuple(ob[a] - t[a] for a in range(3))
            if max(abs(x) for x in d) > ws:
                out.add(d)
    return sorted(out)


@pytest.mark.parametrize("ws", [1, 2])
def test_offset_order_bound_is_the_smallest_order_meeting_it(ws):
    """slack 0: q is the least order whose bound (sqrt3/|d|)^(q+1) does not exceed the nearest
    offsets' bound at order p, (sqrt3/(ws+1))^(p+1) (checked in floating point away from ties);
    the nearest offsets keep order p; the order never grows with distance."""
    for p in (2, 6, 8, 10):
        ref = (p + 1) * math.log(math.sqrt(3) / (ws + 1))
        by_r2 = {}
        for d in _offsets(ws):
            q = FM.offset_order(d, p, ws, 0)
            r = math.sqrt(sum(x * x for x in d))
            lr = math.log(math.sqrt(3) / r)
            assert 0 <= q <= p
            if q < p:
                assert (q + 1) * lr <= ref + 1e-12          # bound met at q
            if q > 0:
                assert q * lr > ref - 1e-12                 # not met at q - 1
            if max(abs(x) for x in d) == ws + 1 and sum(x * x for x in d) == (ws + 1) ** 2:
                assert q == p
            by_r2.setdefault(sum(x * x for x in d), set()).add(q)
        qs = [max(v) for k, v in sorted(by_r2.items())]
        assert all(len(v) == 1 for v in by_r2.values())     # a function of |d| only
        assert all(a >= b for a, b in zip(qs, qs[1:]))       # non-increasing with distance


def test_offset_order_slack_limits():
    for d in _offsets(2):
        assert FM.offset_order(d, 8, 2, -1) == 8
        assert FM.offset_order(d, 8, 2, 8) == 8
        assert FM.offset_order(d, 8, 2, 1) == min(8, FM.offset_order(d, 8, 2, 0) + 1)


def test_m2l_with_orders_truncates_exactly():
    """Per-pair orders: q = p reproduces the plain M2L (to rounding: the masked product may be
    summed in another order); q < p keeps exactly the terms with |n| + |m| <= q (checked against a
    loop over the multi-indices)."""
    rng = np.random.default_rng(91)
    p = 5
    nc = FM.ncoef(p)
    Ms = rng.normal(size=(4, nc))
    R = rng.normal(size=(4, 3)) * 3 + np.array([5.0, 0.0, 0.0])
    plain = FM.m2l(p, Ms, R)
    assert np.allclose(FM.m2l(p, Ms, R, orders=[p] * 4), plain, rtol=1e-14, atol=1e-14 * np.abs(plain).max())
    qs = [0, 2, 3, 5]
    got = FM.m2l(p, Ms, R, orders=qs)
    mi = FM._mi(p).items
    D2 = FM.derivative_tensor(R, p)
    mi2 = FM._mi(2 * p).index
    for k, q in enumerate(qs):
        want = np.zeros(nc)
        for a, n in enumerate(mi):
            for b, m in enumerate(mi):
                if sum(n) + sum(m) <= q:
                    want[a] += D2[k, mi2[(n[0] + m[0], n[1] + m[1], n[2] + m[2])]] * Ms[k, b]
        assert np.allclose(got[k], want, rtol=1e-13, atol=1e-13 * np.abs(want).max())


def test_fmm_with_offset_orders_stays_near_the_fixed_order_error():
    """The per-offset orders with slack 2 keep the FMM field error within 1.5x of the fixed order
    (and slack >= p is the fixed order, to rounding)."""
    X, q, a = rand_system(300, 83, box=14.0, r_min=1.0)
    mu = np.random.default_rng(5).normal(0, 0.2, (300, 3))
    _, Eq, _ = D.charge_fields(X, q)
    _, _, Ed, _ = D.dipole_fields(X, mu, a, 2.0)
    ref = Eq + Ed
    fixed = FM.fmm_fields(X, q, mu, a, 2.0, 4, 1.7, 2, want_grad=False)
    assert fixed["tree"].L >= 3
    same = FM.fmm_fields(X, q, mu, a, 2.0, 4, 1.7, 2, want_grad=False, order_slack=4)
    assert np.allclose(same["E_d"], fixed["E_d"], rtol=1e-13, atol=1e-13 * np.abs(fixed["E_d"]).max())
    adapt = FM.fmm_fields(X, q, mu, a, 2.0, 4, 1.7, 2, want_grad=False, order_slack=2)
    e_fixed = np.linalg.norm(fixed["E_d"] - ref) / np.linalg.norm(ref)
    e_adapt = np.linalg.norm(adapt["E_d"] - ref) / np.linalg.norm(ref)
    assert e_adapt < 1.5 * e_fixed
