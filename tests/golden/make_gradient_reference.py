"""Writes small_globular_2k_dense.npz: the exact solution and gradients of the 2,000-particle
clumped ball at protein density (radius 16.8 A) by the dense oracle: induced dipoles by LU of the
scaled 6,000 x 6,000 system (Sec. II.A, dipole-moment equation), energies, forces F = -dU/dx,
potentials phi = dU/dq and dU/dalpha (stationarity of U^pol in the dipoles, Sec. II.A), Thole a = 2;
and the gradients of the loss L = sum_i G_i . mu_i for a seeded G through the dipoles (the adjoint of
the dipole equations, oracle.direct.dipole_adjoint).

Calls only the oracle and the input generator:
    python tests/golden/make_gradient_reference.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import direct as D  # noqa: E402
from paper_1408_6527_amd import inputs  # noqa: E402
from make_large_reference import fingerprint  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def main():
    ps = inputs.small_globular(2000)
    ref = D.solve(ps.pos, ps.q, ps.alpha, thole_a=2.0)
    out = dict(mu=ref["mu"], F=ref["F"], phi=ref["phi"], grad_alpha=ref["grad_alpha"], U=np.array(ref["U"]),
               U_qq=np.array(ref["U_qq"]), U_pol=np.array(ref["U_pol"]), fingerprint=np.array(fingerprint(ps)))
    # gradients of the loss L = sum G . mu through the dipoles (the adjoint), for a seeded G
    G = np.random.default_rng(1408).normal(0.0, 1.0, (ps.n, 3))
    adj = D.dipole_adjoint(ps.pos, ps.q, ps.alpha, G, thole_a=2.0)
    out.update(adj_G=G, adj_grad_pos=adj["grad_pos"], adj_grad_q=adj["grad_q"], adj_grad_alpha=adj["grad_alpha"])
    path = os.path.join(HERE, "small_globular_2k_dense.npz")
    np.savez_compressed(path, **out)
    print(f"small_globular_2k: U = {ref['U']:.12e} -> {path}", flush=True)


if __name__ == "__main__":
    main()
