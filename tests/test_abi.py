"""The C interface: every function declared in include/pfmm.h is exported by libpfmm.so, and the
host-only entry points behave as documented.  No GPU call is made here."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pfmm.h")
LIB = os.path.join(ROOT, "paper_1408_6527_amd", "libpfmm.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pfmm_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    import torch  # noqa: F401  (same load order as the product path)
    assert os.path.exists(LIB), "libpfmm.so is not built"
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for f in ["pfmm_config_default", "pfmm_create", "pfmm_destroy", "pfmm_solve", "pfmm_backward",
              "pfmm_field", "pfmm_status_string", "pfmm_last_error", "pfmm_version"]:
        assert f in names


def test_every_declared_symbol_is_exported(lib):
    missing = [f for f in declared_functions() if not hasattr(lib, f)]
    assert not missing, missing


def test_status_strings_and_defaults(lib):
    from paper_1408_6527_amd import _lib
    lib.pfmm_status_string.restype = ctypes.c_char_p
    for code in range(9):
        assert lib.pfmm_status_string(code)
    c = _lib.Config()
    lib.pfmm_config_default(ctypes.byref(c))
    assert (c.order_p, c.ws, c.precision, c.scf_max_iter) == (6, 2, 0, 200)
    assert c.scf_tol == 1e-6 and c.thole_a == 2.0 and c.coulomb_k == 332.06371
    assert (c.m2l_order_slack, c.precond_cutoff, c.precond_iters, c.scf_relax) == (-1, 0.0, 4, 0.0)
    assert c.dipole_pair_dl == 0.0


@pytest.mark.parametrize("field,value", [("order_p", 0), ("order_p", 13), ("ws", 3), ("precision", 5),
                                         ("scf_tol", 0.0), ("scf_max_iter", 0), ("thole_a", -1.0),
                                         ("leaf_width", -2.0), ("m2l_order_slack", -2),
                                         ("precond_cutoff", -1.0), ("scf_relax", -0.1), ("scf_relax", 1.0),
                                         ("dipole_pair_dl", -1e-4), ("dipole_pair_dl", 1.5),
                                         ("dipole_pair_dl", float("nan"))])
def test_create_rejects_bad_config(lib, field, value):
    from paper_1408_6527_amd import _lib
    c = _lib.Config()
    lib.pfmm_config_default(ctypes.byref(c))
    setattr(c, field, value)
    h = ctypes.c_void_p()
    assert lib.pfmm_create(ctypes.byref(c), ctypes.byref(h)) == 1
    assert not h.value


def test_null_handle_is_rejected(lib):
    lib.pfmm_solve.restype = ctypes.c_int
    assert lib.pfmm_solve(None, 0, None, None, None, None, None, None, None, None) == 1
    vp = ctypes.c_void_p
    lib.pfmm_solve_qe.restype = ctypes.c_int
    lib.pfmm_solve_qe.argtypes = [vp, ctypes.c_int64] + [vp] * 10
    assert lib.pfmm_solve_qe(None, 0, *([None] * 10)) == 1
    lib.pfmm_backward_qe.restype = ctypes.c_int
    lib.pfmm_backward_qe.argtypes = [vp, ctypes.c_int64, ctypes.c_double] + [vp] * 5
    assert lib.pfmm_backward_qe(None, 0, 1.0, *([None] * 5)) == 1
    lib.pfmm_set_exclusions.restype = ctypes.c_int
    lib.pfmm_set_exclusions.argtypes = [vp, ctypes.c_int64, vp, vp]
    assert lib.pfmm_set_exclusions(None, 0, None, None) == 1
    lib.pfmm_destroy(None)


def test_struct_layout_matches_header(tmp_path):
    """The ctypes mirrors of pfmm_config and pfmm_result have the C layout of include/pfmm.h: every
    field at the same offset, the same total size (checked with the host C compiler)."""
    import shutil
    import subprocess
    from paper_1408_6527_amd import _lib
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "pfmm.h"', "int main(void) {"]
    for cname, cls in [("pfmm_config", _lib.Config), ("pfmm_result", _lib.Result)]:
        lines.append(f'  printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append("  return 0;\n}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, cls in [("pfmm_config", _lib.Config), ("pfmm_result", _lib.Result)]:
        assert got[(cname, "sizeof")] == ctypes.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert got[(cname, fname)] == getattr(cls, fname).offset, (cname, fname)


def test_exclusion_rows_are_symmetric_csr():
    """The binding's CSR form of excluded pairs: each pair in both rows, partners sorted, empty rows
    kept (the form pfmm_set_exclusions validates)."""
    import numpy as np
    from paper_1408_6527_amd.api import exclusion_rows
    ptr, idx = exclusion_rows(5, [(0, 1), (3, 1), (4, 0)])
    assert ptr.tolist() == [0, 2, 4, 4, 5, 6]
    assert idx.tolist() == [1, 4, 0, 3, 1, 0]
    assert ptr.dtype == np.int32 and idx.dtype == np.int32
    ptr, idx = exclusion_rows(3, np.zeros((0, 2), np.int64))
    assert ptr.tolist() == [0, 0, 0, 0] and idx.size == 0
