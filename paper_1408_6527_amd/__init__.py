"""pfmm: polarizable fast multipole method on AMD MI355X (gfx950).

Cartesian FMM evaluation of the field of point charges and induced point dipoles inside the
self-consistent dipole solve, followed by energy, forces and parameter gradients
(Coles & Masella, arXiv:1408.6527), as HIP kernels behind the C interface of include/pfmm.h.

The GPU entry points (`Solver`, `solve`, `field_eval`, `PolarizableEnergy`, `config`) are loaded on
first use from `paper_1408_6527_amd.api`; `paper_1408_6527_amd.inputs` draws synthetic inputs and
needs neither PyTorch nor the library.
"""

_API = {"Solver", "SolveResult", "solve", "field_eval", "PolarizableEnergy", "config", "PFMMError"}


def __getattr__(name):
    if name in _API:
        from . import api
        return getattr(api, name)
    raise AttributeError(name)
