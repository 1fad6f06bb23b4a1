"""Writes sphere_4096_direct.npz: the exact (direct-sum, dense-solve) forces and energy of
the paper's random sphere (Sec. IV.A; 4,096 points in a 45 A ball, minimum separation 2 A, +/-1 e)
for the polarisabilities alpha = 0, 1, 2, 3 A^3 of its polarisation test, Thole a = 2, with the
sphere's separate field charges qE polarising the dipoles.

Calls only the oracle and the input generator:
    python tests/golden/make_sphere_reference.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import direct as D  # noqa: E402
from paper_1408_6527_amd import inputs  # noqa: E402

ALPHAS = (0.0, 1.0, 2.0, 3.0)


def main():
    out = {}
    for a in ALPHAS:
        ps = inputs.sphere(4096, alpha=a)
        ref = D.solve(ps.pos, ps.q, ps.alpha, thole_a=2.0, qE=ps.qE)
        key = f"a{int(a)}"
        out[f"F_{key}"] = ref["F"]
        out[f"U_{key}"] = np.array(ref["U"])
        print(f"alpha {a}: U = {ref['U']:.10e}", flush=True)
    np.savez_compressed(os.path.join(os.path.dirname(os.path.abspath(__file__)), "sphere_4096_direct.npz"), **out)


if __name__ == "__main__":
    main()
