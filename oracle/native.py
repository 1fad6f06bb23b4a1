"""Matrix-free direct-sum oracle for systems too large for the dense solve.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import or call this module; it is used
by tests/, the scripts under tests/golden/, the smoke check and the benchmark's CPU-baseline leg.
It shares no code with the HIP library.

The sums run in liborcdirect.so (oracle/csrc/direct_sum.cpp, C++/OpenMP on all host cores, float64,
compensated per-target totals); this module only marshals arrays and strings the steps together:

* fields(): potential, field (undamped and Thole-damped dipole part) and field gradient of
  given charges and point dipoles at every particle or at sampled targets (the definitions of
  Sec. II.A, as in direct.charge_fields / direct.dipole_fields / direct.fields_at);
* solve(): the induced dipoles mu = alpha (E^q + T~ mu) (Sec. II.A, dipole-moment equation) by
  conjugate gradients on the symmetric Jacobi-scaled system (direct.cg_scaled) with a direct-sum
  product T~ mu, then energy, forces and potentials at the solution (direct.evaluate).

Loading builds the library when it is missing (oracle/build.py).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import direct

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liborcdirect.so")

_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        from .build import build
        build(verbose=False)
    lib = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    lib.orc_threads.argtypes = []
    lib.orc_threads.restype = ctypes.c_int
    lib.orc_fields.argtypes = [ctypes.c_int64, vp, vp, vp, vp, ctypes.c_double, ctypes.c_int64, vp, vp, vp, vp, vp]
    lib.orc_fields.restype = ctypes.c_int
    lib.orc_dipole_field.argtypes = [ctypes.c_int64, vp, vp, ctypes.c_double, vp, ctypes.c_int64, vp, vp]
    lib.orc_dipole_field.restype = ctypes.c_int
    _lib = lib
    return lib


def threads() -> int:
    """Host threads the sums run on (OpenMP)."""
    return int(_load().orc_threads())


def _arr(x, shape=None, dtype=np.float64):
    if x is None:
        return None
    a = np.ascontiguousarray(x, dtype=dtype)
    if shape is not None and a.shape != shape:
        raise ValueError(f"expected shape {shape}, got {a.shape}")
    return a


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _status(st):
    if st == 3:
        raise ValueError("coincident particles")
    if st != 0:
        raise ValueError(f"invalid arguments to the direct-sum oracle (status {st})")


def fields(X, q=None, mu=None, alpha=None, thole_a=2.0, targets=None):
    """Exact fields of the charges q and point dipoles mu at the particles listed in targets (None:
    every particle), each source j != target i.

    Returns phi (undamped potential), E_u (dipole part undamped: what acts on charges), E_d (dipole
    part Thole-damped: what acts on dipoles) and G_d[a, b] = d_a (E_d)_b, restricted to the targets.
    """
    lib = _load()
    X = _arr(X)
    n = X.shape[0]
    X = _arr(X, (n, 3))
    q = _arr(q, (n,))
    mu = _arr(mu, (n, 3))
    alpha = _arr(alpha, (n,))
    tg = None if targets is None else _arr(targets, dtype=np.int64).reshape(-1)
    m = n if tg is None else tg.size
    phi = np.empty(m); Eu = np.empty((m, 3)); Ed = np.empty((m, 3)); G = np.empty((m, 3, 3))
    st = lib.orc_fields(n, _p(X), _p(q), _p(mu), _p(alpha), float(thole_a if alpha is not None else 0.0), m, _p(tg),
                        _p(phi), _p(Eu), _p(Ed), _p(G))
    _status(st)
    return phi, Eu, Ed, G


def dipole_field(X, alpha, thole_a, mu, targets=None):
    """Thole-damped field T~ mu of the point dipoles at every particle (or at the targets listed)."""
    lib = _load()
    X = _arr(X)
    n = X.shape[0]
    alpha = _arr(alpha, (n,))
    mu = _arr(mu, (n, 3))
    tg = None if targets is None else _arr(targets, dtype=np.int64).reshape(-1)
    m = n if tg is None else tg.size
    Ed = np.empty((m, 3))
    _status(lib.orc_dipole_field(n, _p(X), _p(alpha), float(thole_a), _p(mu), m, _p(tg), _p(Ed)))
    return Ed


def solve(X, q, alpha, thole_a=2.0, k_e=direct.COULOMB_K, tol=1e-12, max_iter=2000, log=None):
    """Full oracle without a dense matrix: the exact induced dipoles to the relative residual tol,
    energies, forces and potentials.

    Returns the dict of direct.evaluate (without dU/dalpha) plus mu, iters and residual, where
    residual = ||alpha (E^q + T~ mu) - mu||_2 / ||alpha E^q||_2 is recomputed from the final dipoles
    with one more direct-sum product.  log(msg) receives progress lines when given.
    """
    X = _arr(X); q = _arr(q); alpha = _arr(alpha)
    n = X.shape[0]
    charge = fields(X, q=q, alpha=alpha, thole_a=thole_a)
    phi_q, E_q, _, G_q = charge
    count = [0]

    def apply_T(m):
        count[0] += 1
        if log is not None and count[0] % 5 == 0:
            log(f"direct-sum product {count[0]}")
        return dipole_field(X, alpha, thole_a, m)

    mu, iters, _ = direct.cg_scaled(apply_T, E_q, alpha, tol=tol, max_iter=max_iter)
    dip = fields(X, mu=mu, alpha=alpha, thole_a=thole_a)
    res = np.linalg.norm(alpha[:, None] * (E_q + dip[2]) - mu) / max(np.linalg.norm(alpha[:, None] * E_q), 1e-300)
    out = direct.evaluate(X, q, alpha, mu, thole_a, k_e, charge=(phi_q, E_q, G_q), dip=dip, want_grad_alpha=False)
    out.update(mu=mu, iters=iters, residual=float(res), n=n)
    return out


def forces_at(X, q, mu, alpha, targets, thole_a=2.0, k_e=direct.COULOMB_K):
    """Exact forces F_i = k_e [q_i E_i + (mu_i . grad) E_i] (Sec. II.A at fixed dipoles; E on a charge
    with undamped dipole fields, on a dipole with damped ones) and the exact dipole residual
    alpha_i E_i(mu) - mu_i at the sampled targets, from every source, for given (e.g. a solver's)
    dipoles.  Returns (F (m, 3), residual vectors (m, 3))."""
    tg = np.asarray(targets, np.int64).reshape(-1)
    _, Eu, Ed, G = fields(X, q=q, mu=mu, alpha=alpha, thole_a=thole_a, targets=tg)
    q = np.asarray(q, np.float64); mu = np.asarray(mu, np.float64); alpha = np.asarray(alpha, np.float64)
    F = k_e * (q[tg, None] * Eu + np.einsum("ia,iab->ib", mu[tg], G))
    return F, alpha[tg, None] * Ed - mu[tg]
