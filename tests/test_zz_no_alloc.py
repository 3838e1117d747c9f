"""The allocation-free entry point sem_norm_noalloc against sem_norm, called
through the C-ABI: two calls in a row on one GPU, the second on a smaller
array (a second handle on a coarser mesh), each equal to sem_norm's result
(same kernels, same partial-sum order: bit-identical)."""
import ctypes

import numpy as np
import pytest

from paper_1512_02390_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _norms(nel, p, seed):
    from paper_1512_02390_amd import sem
    xb = W.uniform_breaks(nel, 1.0)
    s = sem.Solver(xb, xb, p, 0, 1, 1, 5)
    try:
        x = torch.tensor(W.random_nodal(s.shape(), 0, seed), dtype=torch.float64, device="cuda")
        lib = sem.load_library()
        a, b = ctypes.c_double(), ctypes.c_double()
        assert lib.sem_norm_noalloc(s.h, ctypes.c_void_p(x.data_ptr()), ctypes.byref(a)) == 0
        assert lib.sem_norm(s.h, ctypes.c_void_p(x.data_ptr()), ctypes.byref(b)) == 0
        ref = float(np.linalg.norm(x.cpu().numpy()))
        return a.value, b.value, ref
    finally:
        s.close()


def test_norm_noalloc_matches_sem_norm_twice():
    print("[gpu-noalloc] 48x48 p=8, then 6x6 p=4", flush=True)
    for nel, p, seed in ((48, 8, 41), (6, 4, 42)):
        got, want, ref = _norms(nel, p, seed)
        assert got == want
        assert abs(got - ref) <= 1e-12 * ref


def test_norm_noalloc_rejects_null_arguments():
    from paper_1512_02390_amd import sem
    lib = sem.load_library()
    out = ctypes.c_double()
    assert lib.sem_norm_noalloc(None, None, ctypes.byref(out)) == -1
