"""Python interface of the pfmm library: argument marshalling only.

Every step of the computation runs in the HIP kernels of libpfmm.so; this module checks tensor
types, hands device pointers and PyTorch's current stream to the C interface and wraps the
results.  Tensors must be float64, contiguous and on the current HIP device.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass, field

import numpy as np
import torch

from . import _lib
from ._lib import lib

__all__ = ["PFMMError", "Solver", "SolveResult", "solve", "field_eval", "PolarizableEnergy", "PolarizableSolve",
           "config"]


class PFMMError(RuntimeError):
    def __init__(self, status: int, message: str):
        self.status = status
        self.code = _lib.STATUS.get(status, str(status))
        super().__init__(f"{self.code}: {message}")


def config(**kw) -> _lib.Config:
    """A pfmm_config with the library defaults, overridden by keyword arguments.

    Keywords: order_p, ws, leaf_width, precision ("fp64" | "mixed"), scf_tol, scf_max_iter,
    graph_iters, thole_a, coulomb_k, m2l_order_slack, precond_cutoff, precond_iters, scf_relax,
    dipole_pair_dl, dipole_tree (0 | 1), mac_theta (0, or the acceptance parameter in [0.3, 1)),
    mac_ndirect, mac_leaf_direct (0 | 1), adaptive_leaf_max (0, or the particles above which a cell
    of the adaptive octree is split),
    forces (bool), potentials (bool), save_for_backward (bool), warm_start (bool), timing (bool).
    """
    c = _lib.Config()
    lib.pfmm_config_default(ctypes.byref(c))
    prec = kw.pop("precision", None)
    if prec is not None:
        c.precision = {"fp64": _lib.PFMM_FP64, "mixed": _lib.PFMM_MIXED}[prec] if isinstance(prec, str) else int(prec)
    flagmap = {"forces": _lib.PFMM_WANT_FORCES, "potentials": _lib.PFMM_WANT_POTENTIALS,
               "save_for_backward": _lib.PFMM_SAVE_FOR_BACKWARD, "warm_start": _lib.PFMM_WARM_START,
               "timing": _lib.PFMM_TIMING}
    for k, bit in flagmap.items():
        if k in kw:
            if kw.pop(k):
                c.flags |= bit
            else:
                c.flags &= ~bit
    for k, v in kw.items():
        if not hasattr(c, k):
            raise TypeError(f"unknown pfmm option {k!r}")
        setattr(c, k, type(getattr(c, k))(v))
    return c


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _check_tensor(name, t, shape):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.dtype != torch.float64:
        raise TypeError(f"{name} must be float64, got {t.dtype}")
    if not t.is_cuda:
        raise ValueError(f"{name} must be on the GPU")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


@dataclass
class SolveResult:
    U: float
    U_qq: float
    U_pol: float
    mu: torch.Tensor
    forces: torch.Tensor | None
    phi: torch.Tensor | None
    iters: int
    residual: float
    residual_max_debye: float
    stats: dict = field(default_factory=dict)
    phi_E: torch.Tensor | None = None  # dU/dqE with separate field charges (potentials wanted)


def exclusion_rows(n, pairs):
    """CSR rows (ptr of n + 1, idx) of the unordered pairs: each pair in both of its rows, the
    partners of a row in increasing order (the form pfmm_set_exclusions takes)."""
    e = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
    rows = np.concatenate([e[:, 0], e[:, 1]])
    cols = np.concatenate([e[:, 1], e[:, 0]])
    order = np.lexsort((cols, rows))
    rows, cols = rows[order], cols[order]
    ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(ptr, rows + 1, 1)
    return np.cumsum(ptr).astype(np.int32), np.ascontiguousarray(cols, dtype=np.int32)


class Solver:
    """Owns one pfmm handle (device tables and workspace) for a fixed configuration."""

    def __init__(self, **kw):
        if not torch.cuda.is_available():
            raise RuntimeError("pfmm needs a GPU (HIP device); none is available")
        self.cfg = config(**kw)
        h = ctypes.c_void_p()
        st = lib.pfmm_create(ctypes.byref(self.cfg), ctypes.byref(h))
        if st != 0:
            raise PFMMError(st, "pfmm_create failed: " + lib.pfmm_status_string(st).decode())
        self._h = h
        self.last_result = None

    def close(self):
        if getattr(self, "_h", None):
            lib.pfmm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _raise(self, st):
        raise PFMMError(st, lib.pfmm_last_error(self._h).decode())

    def solve(self, pos, q, alpha, mu_init=None, allow_unconverged=False, qE=None) -> SolveResult:
        """qE: separate charges of the static field that polarises the dipoles (None: q)."""
        n = pos.shape[0]
        _check_tensor("pos", pos, (n, 3))
        _check_tensor("q", q, (n,))
        _check_tensor("alpha", alpha, (n,))
        if qE is not None:
            _check_tensor("qE", qE, (n,))
        want_f = bool(self.cfg.flags & _lib.PFMM_WANT_FORCES)
        want_p = bool(self.cfg.flags & _lib.PFMM_WANT_POTENTIALS)
        mu = torch.empty((n, 3), dtype=torch.float64, device=pos.device)
        if self.cfg.flags & _lib.PFMM_WARM_START:
            if mu_init is None:
                raise ValueError("warm_start needs mu_init")
            _check_tensor("mu_init", mu_init, (n, 3))
            mu.copy_(mu_init)
        F = torch.empty((n, 3), dtype=torch.float64, device=pos.device) if want_f else None
        phi = torch.empty((n,), dtype=torch.float64, device=pos.device) if want_p else None
        phiE = torch.empty((n,), dtype=torch.float64, device=pos.device) if (want_p and qE is not None) else None
        res = _lib.Result()
        st = lib.pfmm_solve_qe(self._h, n, _ptr(pos), _ptr(q), _ptr(qE), _ptr(alpha), _ptr(mu), _ptr(F),
                               _ptr(phi), _ptr(phiE), ctypes.byref(res), _stream())
        if st != 0 and not (allow_unconverged and st == 4):
            self._raise(st)
        self.last_result = res
        self._n_last = n
        stats = dict(levels=res.levels, leaf_width=res.leaf_width, n_leaves=res.n_leaves,
                     n_cells=res.n_cells, n_m2l=res.n_m2l, n_p2p=res.n_p2p, m2l_flops=res.m2l_flops, n_evals=res.n_evals,
                     m2l_flops_total=res.m2l_flops_total, m2l_order_cap_min=res.m2l_order_cap_min,
                     scf_restarts=res.scf_restarts, solve_id=res.solve_id, n_sites=res.n_sites,
                     m2l_split=dict(ms=list(res.t_m2l_split_ms), launches=list(res.m2l_split_launches),
                                    flops=list(res.m2l_split_flops)),
                     t_phase_ms=list(res.t_phase_ms), status=_lib.STATUS[st],
                     t_kernel_ms=dict(zip(_lib.KERNEL_CLASSES, res.t_kernel_ms)),
                     kernel_launches=dict(zip(_lib.KERNEL_CLASSES, res.kernel_launches)))
        return SolveResult(res.U_total, res.U_qq, res.U_pol, mu, F, phi, res.iters, res.residual,
                           res.residual_max_debye, stats, phiE)

    def set_exclusions(self, n, pairs):
        """Exclude the unordered particle pairs (an (m, 2) integer array, or None to clear) from every
        sum of later solves and field evaluations of n particles."""
        if pairs is None:
            st = lib.pfmm_set_exclusions(self._h, 0, None, None)
        else:
            ptr, idx = exclusion_rows(n, pairs)
            ip = ctypes.POINTER(ctypes.c_int)
            st = lib.pfmm_set_exclusions(self._h, int(n), ptr.ctypes.data_as(ip),
                                         idx.ctypes.data_as(ip) if idx.size else None)
        if st != 0:
            self._raise(st)

    def backward(self, g=1.0, want_pos=True, want_q=True, want_alpha=True, n=None, want_qE=False, solve_id=0):
        """Gradients of g U: (grad_pos, grad_q, grad_alpha), plus grad_qE last with want_qE (after a
        solve with qE).  solve_id (SolveResult.stats["solve_id"]) names the solve whose gradients are
        wanted; the library refuses (PFMM_ERR_NO_STATE) when the handle has solved again since.
        0: the last successful solve."""
        n = n if n is not None else self._n_last
        dev = torch.device("cuda", torch.cuda.current_device())
        gp = torch.empty((n, 3), dtype=torch.float64, device=dev) if want_pos else None
        gq = torch.empty((n,), dtype=torch.float64, device=dev) if want_q else None
        ga = torch.empty((n,), dtype=torch.float64, device=dev) if want_alpha else None
        ge = torch.empty((n,), dtype=torch.float64, device=dev) if want_qE else None
        st = lib.pfmm_backward_qe(self._h, int(solve_id), float(g), _ptr(gp), _ptr(gq), _ptr(ge), _ptr(ga),
                                  _stream())
        if st != 0:
            self._raise(st)
        return (gp, gq, ga, ge) if want_qE else (gp, gq, ga)

    def backward_mu(self, g_mu, want_pos=True, want_q=True, want_alpha=True, want_qE=False, solve_id=0):
        """Gradients of a loss L through the converged dipoles, given g_mu = dL/dmu (n x 3): (grad_pos,
        grad_q, grad_alpha), plus grad_qE last with want_qE.  One adjoint solve with the same operator."""
        n = self._n_last
        _check_tensor("g_mu", g_mu, (n, 3))
        dev = g_mu.device
        gp = torch.empty((n, 3), dtype=torch.float64, device=dev) if want_pos else None
        gq = torch.empty((n,), dtype=torch.float64, device=dev) if want_q else None
        ga = torch.empty((n,), dtype=torch.float64, device=dev) if want_alpha else None
        ge = torch.empty((n,), dtype=torch.float64, device=dev) if want_qE else None
        st = lib.pfmm_backward_mu(self._h, int(solve_id), _ptr(g_mu), _ptr(gp), _ptr(gq), _ptr(ge), _ptr(ga),
                                  _stream())
        if st != 0:
            self._raise(st)
        return (gp, gq, ga, ge) if want_qE else (gp, gq, ga)

    def field(self, pos, q=None, mu=None, alpha=None):
        """phi, E (undamped dipole part), E_damped and grad E_damped (n x 3 x 3) of the sources."""
        n = pos.shape[0]
        _check_tensor("pos", pos, (n, 3))
        if q is not None:
            _check_tensor("q", q, (n,))
        if mu is not None:
            _check_tensor("mu", mu, (n, 3))
        if alpha is None:
            alpha = torch.zeros(n, dtype=torch.float64, device=pos.device)
        _check_tensor("alpha", alpha, (n,))
        phi = torch.empty(n, dtype=torch.float64, device=pos.device)
        E = torch.empty((n, 3), dtype=torch.float64, device=pos.device)
        Ed = torch.empty((n, 3), dtype=torch.float64, device=pos.device)
        G = torch.empty((n, 3, 3), dtype=torch.float64, device=pos.device)
        st = lib.pfmm_field(self._h, n, _ptr(pos), _ptr(q), _ptr(mu), _ptr(alpha), _ptr(phi), _ptr(E),
                            _ptr(Ed), _ptr(G), _stream())
        if st != 0:
            self._raise(st)
        return phi, E, Ed, G


def solve(pos, q, alpha, **kw) -> SolveResult:
    """One-shot polarizable solve: dipoles, energies, forces and potentials."""
    s = Solver(**kw)
    try:
        return s.solve(pos, q, alpha)
    finally:
        s.close()


def field_eval(pos, q=None, mu=None, alpha=None, **kw):
    s = Solver(**kw)
    try:
        return s.field(pos, q, mu, alpha)
    finally:
        s.close()


class PolarizableEnergy(torch.autograd.Function):
    """U(pos, q, alpha) = U^{qq'} + U^pol at the converged dipoles, differentiable in all three inputs.

    The backward uses the stationarity of U^pol in the dipoles, so the dipole solve itself is not
    differentiated; gradients of mu or of the forces are not available through this function.
    The backward reads the state the solver's handle saved for this forward's solve: another solve
    on the same Solver in between makes the backward raise (PFMM_ERR_NO_STATE) rather than return
    the later system's gradients.
    """

    @staticmethod
    def forward(ctx, pos, q, alpha, solver: Solver):
        pos_c, q_c, a_c = pos.detach().contiguous(), q.detach().contiguous(), alpha.detach().contiguous()
        res = solver.solve(pos_c, q_c, a_c)
        ctx.solver = solver
        ctx.n = pos.shape[0]
        ctx.solve_id = res.stats["solve_id"]
        ctx.mark_non_differentiable()
        return torch.tensor(res.U, dtype=torch.float64, device=pos.device)

    @staticmethod
    def backward(ctx, gU):
        g = float(gU.item())
        gp, gq, ga = ctx.solver.backward(g, ctx.needs_input_grad[0], ctx.needs_input_grad[1],
                                         ctx.needs_input_grad[2], n=ctx.n, solve_id=ctx.solve_id)
        return gp, gq, ga, None


class PolarizableSolve(torch.autograd.Function):
    """(U, mu): the energy U^{qq'} + U^pol and the converged dipoles, both differentiable in pos, q and
    alpha.  The gradient through U uses the stationarity of U^pol in the dipoles (pfmm_backward); the
    gradient through mu, for a loss that depends on the dipoles themselves, comes from the adjoint
    solve with the same operator (pfmm_backward_mu).  Another solve on the same Solver before the
    backward makes it raise (PFMM_ERR_NO_STATE).
    """

    @staticmethod
    def forward(ctx, pos, q, alpha, solver: Solver):
        ctx.set_materialize_grads(False)
        pos_c, q_c, a_c = pos.detach().contiguous(), q.detach().contiguous(), alpha.detach().contiguous()
        res = solver.solve(pos_c, q_c, a_c)
        ctx.solver = solver
        ctx.n = pos.shape[0]
        ctx.solve_id = res.stats["solve_id"]
        return torch.tensor(res.U, dtype=torch.float64, device=pos.device), res.mu

    @staticmethod
    def backward(ctx, gU, gmu):
        need = ctx.needs_input_grad[:3]
        out = [None, None, None]

        def add(parts):
            for k in range(3):
                if parts[k] is not None:
                    out[k] = parts[k] if out[k] is None else out[k] + parts[k]

        if gU is not None:
            add(ctx.solver.backward(float(gU.item()), need[0], need[1], need[2], n=ctx.n, solve_id=ctx.solve_id))
        if gmu is not None:
            add(ctx.solver.backward_mu(gmu.detach().contiguous(), need[0], need[1], need[2], solve_id=ctx.solve_id))
        return out[0], out[1], out[2], None
