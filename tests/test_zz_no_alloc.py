"""pfmm_field_noalloc through the C interface: the allocation-free variant of pfmm_field (for callers
that cannot allocate) gives bitwise the results of pfmm_field on the same inputs, on two calls in a
row (the second smaller), takes no device memory, and refuses an evaluation larger than its scratch;
with the well-separation lists and with the adaptive octree's walk."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _cloud(n, density, seed):
    rng = np.random.default_rng(seed)
    side = (n / density) ** (1.0 / 3.0)
    X = rng.uniform(0.0, side, (n, 3))
    q = rng.normal(0.0, 0.4, n)
    a = rng.uniform(0.2, 2.0, n)
    mu = rng.normal(0.0, 0.1, (n, 3))
    return X, q, a, mu


def _noalloc(lib):
    vp = ctypes.c_void_p
    f = lib.pfmm_field_noalloc
    f.argtypes = [vp, ctypes.c_int64, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    f.restype = ctypes.c_int
    return f


@pytest.mark.parametrize("lists", ["ws", "adaptive"])
def test_field_noalloc_matches_field_and_allocates_nothing(lists):
    import torch
    from paper_1408_6527_amd import api
    from paper_1408_6527_amd._lib import lib
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    f = _noalloc(lib)
    dev = torch.device("cuda", 0)
    T = lambda x: torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=dev)
    kw = dict(order_p=6, ws=2, leaf_width=4.0, thole_a=2.0)
    if lists == "adaptive":
        # the dual walk's lists, whose near rows grow level by level inside the scratch
        kw.update(adaptive_leaf_max=12)
    ref_solver = api.Solver(**kw)
    na_solver = api.Solver(**kw)  # a fresh handle: only its tables are allocated
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    # (the walk's frontiers, split-partner table and near rows take more workspace per particle)
    sizes = ((40_000, 1), (7_000, 2)) if lists == "ws" else ((10_000, 1), (2_500, 2))
    for n, seed in sizes:
        print(f"[case] noalloc field {lists} n={n}", flush=True)
        X, q, a, mu = _cloud(n, 0.05, seed)
        pos, qq, al, mm = T(X), T(q), T(a), T(mu)
        ref = ref_solver.field(pos, qq, mm, al)
        out = [torch.full((n,), np.nan, dtype=torch.float64, device=dev),
               torch.full((n, 3), np.nan, dtype=torch.float64, device=dev),
               torch.full((n, 3), np.nan, dtype=torch.float64, device=dev),
               torch.full((n, 3, 3), np.nan, dtype=torch.float64, device=dev)]
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        st = f(na_solver._h, n, *(ctypes.c_void_p(t.data_ptr()) for t in (pos, qq, mm, al)),
               *(ctypes.c_void_p(t.data_ptr()) for t in out), stream)
        torch.cuda.synchronize()
        free1 = torch.cuda.mem_get_info()[0]
        assert st == 0, lib.pfmm_last_error(na_solver._h).decode()
        assert free1 == free0, f"device memory taken by the call: {free0 - free1} bytes"
        for r, o in zip(ref, out):
            assert torch.equal(r, o)
    # too large for the scratch: refused with the maximum named, nothing written
    n = 600_000
    X, q, a, mu = _cloud(n, 0.1, 3)
    pos, qq, al, mm = T(X), T(q), T(a), T(mu)
    out = [torch.zeros((n,), dtype=torch.float64, device=dev), torch.zeros((n, 3), dtype=torch.float64, device=dev),
           torch.zeros((n, 3), dtype=torch.float64, device=dev), torch.zeros((n, 3, 3), dtype=torch.float64, device=dev)]
    st = f(na_solver._h, n, *(ctypes.c_void_p(t.data_ptr()) for t in (pos, qq, mm, al)),
           *(ctypes.c_void_p(t.data_ptr()) for t in out), stream)
    assert st == 1
    assert "scratch maximum" in lib.pfmm_last_error(na_solver._h).decode()
    assert all(float(t.abs().max()) == 0.0 for t in out)
