"""Writes <workload>_oracle.npz: the exact solution of a large synthetic workload by the
matrix-free direct-sum oracle (oracle/native.py): induced dipoles to a relative residual of 1e-12
(Sec. II.A, dipole-moment equation, conjugate gradients on the Jacobi-scaled system with
direct-sum products), then energies (U, U^{qq'}, U^pol), forces and potentials at the solution,
Thole a = 2.

Calls only the oracle and the input generator:
    python tests/golden/make_large_reference.py globular_50k [hexamer_shell_160k scaling_250k ...]

Stored per workload: mu, F (n x 3), phi (n, for the 50k workload only), the energies, the CG
iteration count, the recomputed residual, the host threads and wall time, and a SHA-256 of the
generator's positions, charges and polarisabilities so that a test can tell if the generator has
changed since.
"""
import hashlib
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import native as NT  # noqa: E402
from paper_1408_6527_amd import inputs  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
TOL = 1e-12
THOLE_A = 2.0
WITH_PHI = {"globular_50k"}


def fingerprint(ps) -> str:
    h = hashlib.sha256()
    for a in (ps.pos, ps.q, ps.alpha):
        h.update(np.ascontiguousarray(a, dtype=np.float64).tobytes())
    return h.hexdigest()[:16]


def main(names):
    for name in names:
        t0 = time.time()
        ps = inputs.make(name)
        print(f"{name}: n = {ps.n}, generated in {time.time() - t0:.1f} s, {NT.threads()} threads", flush=True)
        t0 = time.time()
        o = NT.solve(ps.pos, ps.q, ps.alpha, thole_a=THOLE_A, tol=TOL,
                     log=lambda m: print(f"  {name}: {m} ({time.time() - t0:.0f} s)", flush=True))
        wall = time.time() - t0
        out = dict(mu=o["mu"], F=o["F"], U=np.array(o["U"]), U_qq=np.array(o["U_qq"]), U_pol=np.array(o["U_pol"]),
                   iters=np.array(o["iters"]), residual=np.array(o["residual"]), tol=np.array(TOL),
                   thole_a=np.array(THOLE_A), threads=np.array(NT.threads()), wall_s=np.array(wall),
                   fingerprint=np.array(fingerprint(ps)))
        if name in WITH_PHI:
            out["phi"] = o["phi"]
        path = os.path.join(HERE, f"{name}_oracle.npz")
        np.savez_compressed(path, **out)
        print(f"{name}: U = {o['U']:.12e}, iters {o['iters']}, residual {o['residual']:.2e}, {wall:.0f} s -> {path}",
              flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["globular_50k"])
