"""Direct-summation FP64 oracle for the polarizable electrostatics of Coles & Masella,
"The Fast Multipole Method and Point Dipole Moment Polarizable Force Fields" (arXiv:1408.6527).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import or call this module; it is
used by tests/, by the smoke check and by the CPU-baseline leg of the benchmark.  It shares no
code with the HIP library.

Everything here is the plain definition written out, in float64, one target at a time with the
sum over sources vectorised:

* static field and Coulomb potential: Sec. II.A, equations for U^{qq'} and E^q;
* induced-dipole field E^mu = sum_j T_ij mu_j with T the Hessian of the Green's function
  (Sec. II.A, dipolar-tensor equation; the sign is read so that the field of a dipole is the
  physical one) and a Thole short-range damping of the dipole-dipole tensor (Sec. II.A and
  Sec. III mention the damping but do not give its form; the linear "cone" model is used);
* the linear system mu_i = alpha_i (E^q_i + E^mu_i) (Sec. II.A, dipole-moment equation),
  solved densely in the symmetric scaled form (I - S T S) y = S E^q, mu = S y, S = diag(sqrt(alpha));
* U^pol = A(mu) - sum Phi^{mu q} - 1/2 sum Phi^{mu mu} with A = 1/2 sum |mu|^2/alpha
  (Sec. II.A, U^pol and A(mu) equations);
* forces and parameter gradients from the stationarity dU^pol/dmu = 0 (Sec. II.A and II.C):
  the derivative of U at fixed dipoles.

Units: lengths in Angstrom, charges in e, polarisabilities as volumes in Angstrom^3, fields in
e/Angstrom^2, dipoles in e*Angstrom.  Energies, forces and potentials are multiplied by the
Coulomb constant k_e at the end (default 332.06371 kcal*Angstrom/(mol*e^2)).
"""
from __future__ import annotations

import numpy as np

COULOMB_K = 332.06371
EANG_TO_DEBYE = 4.80320


# ----------------------------------------------------------------------------------------------
# Radial functions of the Green's function and of its Thole-smeared version.
# ----------------------------------------------------------------------------------------------

def radial_derivatives(r: np.ndarray, s: np.ndarray | float | None):
    """Return g, g', g'', g''' for the interaction kernel g(r).

    Undamped: g = 1/r (the Green's function of Sec. II.A).
    Damped (Thole linear model, used only between two dipoles): the potential of a unit charge
    smeared as a cone of radius s, g = (2 - 2 v^2 + v^3)/s for v = r/s < 1 and 1/r beyond.
    s = 0 means no damping.
    """
    r = np.asarray(r, dtype=np.float64)
    g = 1.0 / r
    g1 = -1.0 / r**2
    g2 = 2.0 / r**3
    g3 = -6.0 / r**4
    if s is None:
        return g, g1, g2, g3
    s = np.broadcast_to(np.asarray(s, dtype=np.float64), r.shape)
    inside = (s > 0) & (r < s)
    if np.any(inside):
        si = s[inside]
        v = r[inside] / si
        g = g.copy(); g1 = g1.copy(); g2 = g2.copy(); g3 = g3.copy()
        g[inside] = (2.0 - 2.0 * v**2 + v**3) / si
        g1[inside] = (-4.0 * v + 3.0 * v**2) / si**2
        g2[inside] = (-4.0 + 6.0 * v) / si**3
        g3[inside] = 6.0 / si**4
    return g, g1, g2, g3


def hessian_and_third(rvec: np.ndarray, s=None):
    """Second and third Cartesian derivatives of g(|r|) for each row of rvec (shape (m, 3)).

    Uses d_a d_b g = (g'' - g'/r) u_a u_b + (g'/r) delta_ab and
    d_a d_b d_c g = (g''' - 3 g''/r + 3 g'/r^2) u_a u_b u_c
                    + (g''/r - g'/r^2)(delta_ab u_c + delta_ac u_b + delta_bc u_a),  u = r/|r|.
    Returns (grad (m,3), H (m,3,3), T3 (m,3,3,3)).
    """
    r = np.linalg.norm(rvec, axis=1)
    u = rvec / r[:, None]
    g, g1, g2, g3 = radial_derivatives(r, s)
    eye = np.eye(3)
    grad = g1[:, None] * u
    H = (g2 - g1 / r)[:, None, None] * u[:, :, None] * u[:, None, :] + (g1 / r)[:, None, None] * eye
    A = g3 - 3.0 * g2 / r + 3.0 * g1 / r**2
    B = g2 / r - g1 / r**2
    uuu = u[:, :, None, None] * u[:, None, :, None] * u[:, None, None, :]
    sym = (eye[None, :, :, None] * u[:, None, None, :]
           + eye[None, :, None, :] * u[:, None, :, None]
           + eye[None, None, :, :] * u[:, :, None, None])
    T3 = A[:, None, None, None] * uuu + B[:, None, None, None] * sym
    return g, grad, H, T3


def thole_radius(alpha_i, alpha_j, thole_a):
    """s_ij = a (alpha_i alpha_j)^(1/6); zero disables damping for the pair."""
    if thole_a <= 0:
        return np.zeros_like(np.asarray(alpha_j, dtype=np.float64) * 1.0)
    return thole_a * np.cbrt(np.sqrt(np.asarray(alpha_i) * np.asarray(alpha_j)))


# ----------------------------------------------------------------------------------------------
# Fields by direct summation.
# ----------------------------------------------------------------------------------------------

def _check_distinct(X):
    n = X.shape[0]
    for i in range(n):
        d = np.linalg.norm(X - X[i], axis=1)
        d[i] = np.inf
        if np.min(d, initial=np.inf) == 0.0:
            raise ValueError("coincident particles")


def exclusion_matrix(n, excl=None):
    """n x n boolean matrix of the excluded pairs: the starred sums of Sec. II.A skip them (bonded
    pairs in a force field).  excl lists unordered pairs (i, j), i != j, as an (m, 2) array."""
    M = np.zeros((n, n), bool)
    if excl is not None and len(excl):
        e = np.asarray(excl, np.int64).reshape(-1, 2)
        M[e[:, 0], e[:, 1]] = True
        M[e[:, 1], e[:, 0]] = True
    return M


def _partners(n, i, ex):
    return (np.arange(n) != i) & ~ex[i]


def charge_fields(X: np.ndarray, q: np.ndarray, want_grad: bool = True, excl=None):
    """Potential, field and field gradient of the point charges at every particle, j != i and
    (i, j) not excluded.

    phi_i = sum*_j q_j / r_ij;  E_i = -grad phi_i = sum*_j q_j r_ij / r_ij^3;
    G_i[a, b] = d_a E_b.
    """
    X = np.asarray(X, np.float64); q = np.asarray(q, np.float64)
    n = X.shape[0]
    ex = exclusion_matrix(n, excl)
    phi = np.zeros(n); E = np.zeros((n, 3)); G = np.zeros((n, 3, 3))
    for i in range(n):
        mask = _partners(n, i, ex)
        rv = X[i] - X[mask]
        g, grad, H, _ = hessian_and_third(rv)
        phi[i] = np.sum(q[mask] * g)
        E[i] = -np.sum(q[mask][:, None] * grad, axis=0)
        if want_grad:
            G[i] = -np.sum(q[mask][:, None, None] * H, axis=0)
    return phi, E, G


def dipole_fields(X, mu, alpha, thole_a, want_grad: bool = True, excl=None):
    """Fields of the point dipoles mu_j at every particle, j != i and (i, j) not excluded.

    Returns phi (undamped potential mu_j . r / r^3), E_u (undamped field, what acts on charges),
    E_d (damped field T~ mu, what acts on dipoles) and G_d[a, b] = d_a (E_d)_b (damped).
    """
    X = np.asarray(X, np.float64); mu = np.asarray(mu, np.float64); alpha = np.asarray(alpha, np.float64)
    n = X.shape[0]
    ex = exclusion_matrix(n, excl)
    phi = np.zeros(n); Eu = np.zeros((n, 3)); Ed = np.zeros((n, 3)); Gd = np.zeros((n, 3, 3))
    for i in range(n):
        mask = _partners(n, i, ex)
        rv = X[i] - X[mask]
        m = mu[mask]
        _, grad_u, H_u, _ = hessian_and_third(rv)
        s = thole_radius(alpha[i], alpha[mask], thole_a)
        _, _, H_d, T3_d = hessian_and_third(rv, s)
        phi[i] = -np.sum(np.einsum("ja,ja->j", m, grad_u))
        Eu[i] = np.einsum("jab,jb->a", H_u, m)
        Ed[i] = np.einsum("jab,jb->a", H_d, m)
        if want_grad:
            Gd[i] = np.einsum("jabc,jc->ab", T3_d, m)
    return phi, Eu, Ed, Gd


def dipole_matrix(X, alpha, thole_a, excl=None):
    """Dense 3N x 3N damped dipole field tensor: E_d = T mu, block (i, j) = Hessian of g at x_i - x_j
    (zero for excluded pairs)."""
    X = np.asarray(X, np.float64); alpha = np.asarray(alpha, np.float64)
    n = X.shape[0]
    ex = exclusion_matrix(n, excl)
    T = np.zeros((3 * n, 3 * n))
    for i in range(n):
        mask = _partners(n, i, ex)
        idx = np.nonzero(mask)[0]
        rv = X[i] - X[mask]
        s = thole_radius(alpha[i], alpha[mask], thole_a)
        _, _, H, _ = hessian_and_third(rv, s)
        for k, j in enumerate(idx):
            T[3 * i:3 * i + 3, 3 * j:3 * j + 3] = H[k]
    return T


# ----------------------------------------------------------------------------------------------
# Induced dipoles.
# ----------------------------------------------------------------------------------------------

def solve_dipoles_dense(X, q, alpha, thole_a, E_q=None, excl=None):
    """Exact solution of mu = alpha (E^q + T~ mu) by a dense LU solve of the scaled system.

    (I - S T S) y = S E^q with S = diag(sqrt(alpha)) repeated per component; mu = S y.
    Polarisabilities equal to zero give mu_i = 0 exactly.
    """
    X = np.asarray(X, np.float64); alpha = np.asarray(alpha, np.float64)
    n = X.shape[0]
    if E_q is None:
        _, E_q, _ = charge_fields(X, q, want_grad=False, excl=excl)
    T = dipole_matrix(X, alpha, thole_a, excl)
    S = np.repeat(np.sqrt(alpha), 3)
    A = np.eye(3 * n) - S[:, None] * T * S[None, :]
    y = np.linalg.solve(A, S * E_q.reshape(-1))
    return (S * y).reshape(n, 3)


def cg_scaled(apply_T, E_q, alpha, tol=1e-12, max_iter=1000, mu0=None):
    """Conjugate gradients on the scaled system (I - S T S) y = S E^q (Hestenes-Stiefel).

    apply_T(mu) must return the damped dipole field T~ mu at every particle, shape (n, 3).
    Start from mu0 = alpha E^q unless given.  Stop when the preconditioned residual in dipole
    units, ||alpha E(mu) - mu||_2 / ||alpha E^q||_2, is at most tol.  This is conjugate gradients
    on the symmetric Jacobi-scaled system; the paper names an iterative scheme but gives its
    details elsewhere.  Returns (mu, iterations, final relative residual).
    """
    alpha = np.asarray(alpha, np.float64)
    n = alpha.shape[0]
    S = np.repeat(np.sqrt(alpha), 3)
    b = S * E_q.reshape(-1)

    def A(v):
        return v - S * apply_T((S * v).reshape(n, 3)).reshape(-1)

    if mu0 is None:
        y = b.copy()
    else:
        y = np.where(S > 0, np.asarray(mu0, np.float64).reshape(-1) / np.where(S > 0, S, 1.0), 0.0)
    r = b - A(y)
    bnorm = np.sqrt(np.sum((S * b) ** 2))
    if bnorm == 0.0:
        return np.zeros((n, 3)), 0, 0.0

    def resid(rr):
        return np.sqrt(np.sum((S * rr) ** 2)) / bnorm

    p = r.copy()
    rr = r @ r
    it = 0
    rel = resid(r)
    while rel > tol and it < max_iter:
        Ap = A(p)
        pAp = p @ Ap
        if pAp <= 0:
            raise np.linalg.LinAlgError("system is not positive definite")
        a = rr / pAp
        y = y + a * p
        r = r - a * Ap
        rr_new = r @ r
        p = r + (rr_new / rr) * p
        rr = rr_new
        it += 1
        rel = resid(r)
    return (S * y).reshape(n, 3), it, rel


# ----------------------------------------------------------------------------------------------
# Energy, forces and gradients at given dipoles.
# ----------------------------------------------------------------------------------------------

def evaluate(X, q, alpha, mu, thole_a=2.0, k_e=COULOMB_K, charge=None, dip=None, qE=None, charge_E=None,
             excl=None, want_grad_alpha=True):
    """Energies, forces, potentials and dU/dalpha for given dipoles (exact if mu is converged).

    The static field that polarises the dipoles comes from the charges q^E (Sec. III: they may
    differ from the Coulomb charges q; qE=None means q^E = q, the same charges):
    U^{qq'} = 1/2 sum_i q_i phi^q_i
    U^pol   = 1/2 sum |mu_i|^2/alpha_i - sum mu_i.E^{qE}_i - 1/2 sum mu_i.E^mu_i   (E^mu damped)
    F_i     = q_i E^q_i + qE_i E^mu_u,i + (mu_i . grad)(E^{qE} + E^mu_d)_i
              (charges feel the undamped dipole field; dipoles feel the damped one)
    phi_i   = dU/dq_i: phi^q_i + phi^mu_i when q^E = q, phi^q_i otherwise (both undamped)
    phi_E_i = dU/dqE_i = phi^mu_i (returned when qE is given)
    dU/dalpha_i = -|mu_i|^2/(2 alpha_i^2) (= -|E_i|^2/2 when alpha_i = 0, E = E^{qE} + E^mu_d)
                  - sum_{j: r_ij < s_ij} mu_i . (dT~_ij/ds_ij) mu_j * s_ij/(6 alpha_i)
    Energies, forces, potentials and gradients are multiplied by k_e.  want_grad_alpha=False skips
    dU/dalpha (its Thole term is a pairwise sum, too slow here for large systems).
    """
    X = np.asarray(X, np.float64); q = np.asarray(q, np.float64)
    alpha = np.asarray(alpha, np.float64); mu = np.asarray(mu, np.float64)
    n = X.shape[0]
    phi_q, E_q, G_q = charge if charge is not None else charge_fields(X, q, excl=excl)
    tied = qE is None
    if tied:
        qE = q
        E_e, G_e = E_q, G_q
    else:
        qE = np.asarray(qE, np.float64)
        _, E_e, G_e = charge_E if charge_E is not None else charge_fields(X, qE, excl=excl)
    phi_m, Eu_m, Ed_m, Gd_m = dip if dip is not None else dipole_fields(X, mu, alpha, thole_a, excl=excl)
    pos = alpha > 0
    U_qq = 0.5 * np.sum(q * phi_q)
    A_mu = 0.5 * np.sum(np.sum(mu[pos] ** 2, axis=1) / alpha[pos])
    U_pol = A_mu - np.sum(mu * E_e) - 0.5 * np.sum(mu * Ed_m)
    G = G_e + Gd_m
    F = q[:, None] * E_q + qE[:, None] * Eu_m + np.einsum("ia,iab->ib", mu, G)
    phi = phi_q + phi_m if tied else phi_q
    E_tot = E_e + Ed_m
    out = dict(U=k_e * (U_qq + U_pol), U_qq=k_e * U_qq, U_pol=k_e * U_pol, F=k_e * F, phi=k_e * phi,
               E_q=E_q, E_mu=Ed_m, E_mu_undamped=Eu_m, G=G)
    if want_grad_alpha:
        g_alpha = np.empty(n)
        g_alpha[pos] = -np.sum(mu[pos] ** 2, axis=1) / (2.0 * alpha[pos] ** 2)
        g_alpha[~pos] = -0.5 * np.sum(E_tot[~pos] ** 2, axis=1)
        g_alpha += thole_alpha_term(X, alpha, mu, thole_a, excl)
        out["grad_alpha"] = k_e * g_alpha
    if not tied:
        out.update(phi_E=k_e * phi_m, E_qE=E_e)
    return out


def thole_alpha_term(X, alpha, mu, thole_a, excl=None):
    """Second term of dU/dalpha_i: derivative of -1/2 sum mu.T~ mu through s_ij = a (alpha_i alpha_j)^(1/6).

    With v = r/s < 1: T~ = (3 v^4 u u - (4 v^3 - 3 v^4) I)/r^3, so
    dT~/ds = (-12 v^4 u u + 12 (v^3 - v^4) I)/(s r^3), and ds/dalpha_i = s/(6 alpha_i).
    """
    X = np.asarray(X, np.float64); alpha = np.asarray(alpha, np.float64); mu = np.asarray(mu, np.float64)
    n = X.shape[0]
    out = np.zeros(n)
    if thole_a <= 0:
        return out
    ex = exclusion_matrix(n, excl)
    for i in range(n):
        if alpha[i] <= 0:
            continue
        mask = _partners(n, i, ex)
        rv = X[i] - X[mask]
        r = np.linalg.norm(rv, axis=1)
        s = thole_radius(alpha[i], alpha[mask], thole_a)
        inside = (s > 0) & (r < s)
        if not np.any(inside):
            continue
        rv = rv[inside]; r = r[inside]; s = s[inside]; mj = mu[mask][inside]
        u = rv / r[:, None]
        v = r / s
        mi_u = u @ mu[i]
        mj_u = np.sum(mj * u, axis=1)
        mi_mj = mj @ mu[i]
        dTds = (-12.0 * v**4 * mi_u * mj_u + 12.0 * (v**3 - v**4) * mi_mj) / (s * r**3)
        out[i] = -np.sum(dTds * s / (6.0 * alpha[i]))
    return out


def solve(X, q, alpha, thole_a=2.0, k_e=COULOMB_K, qE=None, excl=None):
    """Full oracle: exact dipoles (dense LU), energies, forces, potentials and gradients.
    qE: the charges of the static field that polarises the dipoles (None: q).  excl: excluded
    pairs, left out of every sum (exclusion_matrix)."""
    X = np.asarray(X, np.float64)
    _check_distinct(X)
    charge = charge_fields(X, q, excl=excl)
    charge_E = None if qE is None else charge_fields(X, qE, excl=excl)
    mu = solve_dipoles_dense(X, q, alpha, thole_a, E_q=(charge if qE is None else charge_E)[1], excl=excl)
    dip = dipole_fields(X, mu, alpha, thole_a, excl=excl)
    out = evaluate(X, q, alpha, mu, thole_a, k_e, charge=charge, dip=dip, qE=qE, charge_E=charge_E, excl=excl)
    out["mu"] = mu
    return out


def energy_only(X, q, alpha, thole_a=2.0, k_e=COULOMB_K, qE=None, excl=None):
    """Total U at the exact dipoles; U^pol = -1/2 sum mu.E^{qE} holds at the solution (qE: the
    charges of the polarising field, None: q)."""
    phi_q, _, _ = charge_fields(X, q, want_grad=False, excl=excl)
    _, E_e, _ = charge_fields(X, q if qE is None else qE, want_grad=False, excl=excl)
    mu = solve_dipoles_dense(X, q, alpha, thole_a, E_q=E_e, excl=excl)
    return k_e * (0.5 * np.sum(np.asarray(q) * phi_q) - 0.5 * np.sum(mu * E_e))


def fields_at(idx, X, q=None, mu=None, alpha=None, thole_a=2.0):
    """Exact fields at the particles listed in idx from every other particle (sampled targets).

    Returns phi (undamped), E_u (undamped dipole part), E_d (damped dipole part) and G_d = d_a (E_d)_b,
    each restricted to the targets in idx.  Used to check large systems on a sample of outputs.
    """
    X = np.asarray(X, np.float64)
    n = X.shape[0]
    q = np.zeros(n) if q is None else np.asarray(q, np.float64)
    mu = np.zeros((n, 3)) if mu is None else np.asarray(mu, np.float64)
    alpha = np.zeros(n) if alpha is None else np.asarray(alpha, np.float64)
    idx = np.asarray(idx)
    m = idx.size
    phi = np.zeros(m); Eu = np.zeros((m, 3)); Ed = np.zeros((m, 3)); Gd = np.zeros((m, 3, 3))
    for k, i in enumerate(idx):
        mask = np.arange(n) != i
        rv = X[i] - X[mask]
        g, grad, H, T3 = hessian_and_third(rv)
        s = thole_radius(alpha[i], alpha[mask], thole_a)
        _, _, Hd, T3d = hessian_and_third(rv, s)
        qs = q[mask]; ms = mu[mask]
        phi[k] = np.sum(qs * g) - np.sum(ms * grad)
        Eq = -np.sum(qs[:, None] * grad, axis=0)
        Eu[k] = Eq + np.einsum("jab,jb->a", H, ms)
        Ed[k] = Eq + np.einsum("jab,jb->a", Hd, ms)
        Gd[k] = -np.sum(qs[:, None, None] * H, axis=0) + np.einsum("jabc,jc->ab", T3d, ms)
    return phi, Eu, Ed, Gd


# ----------------------------------------------------------------------------------------------
# Gradients of a loss that depends on the dipoles (the adjoint of the dipole equations).
# ----------------------------------------------------------------------------------------------

def thole_alpha_pair(X, alpha, a, b, thole_a, excl=None):
    """sum_j a_i . (dT~_ij/ds_ij) b_j * ds_ij/dalpha_i for every i (zero where alpha_i = 0), with
    s_ij = a (alpha_i alpha_j)^(1/6), ds_ij/dalpha_i = s_ij / (6 alpha_i); by the formula of
    thole_alpha_term, (a . dT~/ds b) = (-12 v^4 (a.u)(b.u) + 12 (v^3 - v^4) a.b) / (s r^3) for v = r/s < 1."""
    X = np.asarray(X, np.float64); alpha = np.asarray(alpha, np.float64)
    a = np.asarray(a, np.float64); b = np.asarray(b, np.float64)
    n = X.shape[0]
    out = np.zeros(n)
    if thole_a <= 0:
        return out
    ex = exclusion_matrix(n, excl)
    for i in range(n):
        if alpha[i] <= 0:
            continue
        mask = _partners(n, i, ex)
        rv = X[i] - X[mask]
        r = np.linalg.norm(rv, axis=1)
        s = thole_radius(alpha[i], alpha[mask], thole_a)
        inside = (s > 0) & (r < s)
        if not np.any(inside):
            continue
        rv = rv[inside]; r = r[inside]; s = s[inside]; bj = b[mask][inside]
        u = rv / r[:, None]
        v = r / s
        dTds = (-12.0 * v**4 * (u @ a[i]) * np.sum(bj * u, axis=1) + 12.0 * (v**3 - v**4) * (bj @ a[i])) / (s * r**3)
        out[i] = np.sum(dTds * s / (6.0 * alpha[i]))
    return out


def dipole_adjoint(X, q, alpha, G, thole_a=2.0, qE=None, excl=None):
    """Gradients of a loss L(mu) through the induced dipoles, given G = dL/dmu (n x 3) at the solution.

    The dipoles solve A mu = E^{qE} with A = diag(1/alpha) - T~ (Sec. II.A, dipole-moment equation;
    qE=None: the field of the charges q).  A is symmetric, so the adjoint lambda = A^-1 G solves the
    same system with G in place of E^{qE} (in the scaled form, (I - S T~ S) z = S G, lambda = S z,
    lambda_i = 0 where alpha_i = 0), and dL = lambda . (dE^{qE} + dT~ mu - d(diag(1/alpha)) mu):
      dL/dx_i     = qE_i E^lambda_u,i + (lambda_i . grad)(E^{qE} + E^mu_d)_i + (mu_i . grad) E^lambda_d,i
      dL/dqE_i    = -phi^lambda_i                      (minus the undamped potential of the dipoles lambda)
      dL/dalpha_i = (G_i + E^lambda_d,i) . E_i + sum_j [lambda_i . dT~_ij/ds mu_j + mu_i . dT~_ij/ds lambda_j] ds_ij/dalpha_i
    with E = E^{qE} + E^mu_d the total damped field (for alpha_i > 0, G_i + E^lambda_d,i = lambda_i / alpha_i).
    Returns dict(mu, lam, grad_pos, grad_q, grad_alpha[, grad_qE]); with qE given, L does not depend on q.
    """
    X = np.asarray(X, np.float64); q = np.asarray(q, np.float64); alpha = np.asarray(alpha, np.float64)
    G = np.asarray(G, np.float64).reshape(-1, 3)
    tied = qE is None
    qf = q if tied else np.asarray(qE, np.float64)
    _, E_e, G_e = charge_fields(X, qf, excl=excl)
    mu = solve_dipoles_dense(X, q, alpha, thole_a, E_q=E_e, excl=excl)
    lam = solve_dipoles_dense(X, q, alpha, thole_a, E_q=G, excl=excl)
    _, _, Ed_m, Gd_m = dipole_fields(X, mu, alpha, thole_a, excl=excl)
    phi_l, Eu_l, Ed_l, Gd_l = dipole_fields(X, lam, alpha, thole_a, excl=excl)
    gx = (qf[:, None] * Eu_l + np.einsum("ia,iab->ib", lam, G_e + Gd_m) + np.einsum("ia,iab->ib", mu, Gd_l))
    E_tot = E_e + Ed_m
    ga = np.sum((G + Ed_l) * E_tot, axis=1)
    ga += thole_alpha_pair(X, alpha, lam, mu, thole_a, excl) + thole_alpha_pair(X, alpha, mu, lam, thole_a, excl)
    out = dict(mu=mu, lam=lam, grad_pos=gx, grad_alpha=ga)
    if tied:
        out["grad_q"] = -phi_l
    else:
        out["grad_q"] = np.zeros_like(q)
        out["grad_qE"] = -phi_l
    return out
