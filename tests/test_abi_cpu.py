"""Host-only checks of the C-ABI boundary: the shared library loads, exports
every function declared in include/sem.h, the header is valid C, and error
handling that needs no device works."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sem.h")
LIB = os.path.join(ROOT, "paper_1512_02390_amd", "libsem.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sem3?_[a-z_0-9]+)\s*\(", text)))


def test_header_is_c():
    src = f'#include "{HEADER}"\nint main(void) {{ return 0; }}\n'
    r = subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-x", "c", "-fsyntax-only", "-"],
                       input=src, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


@pytest.mark.skipif(not os.path.exists(LIB), reason="libsem.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    names = declared_functions()
    assert "sem_setup" in names and "sem_pcg_solve" in names
    for n in names:
        assert hasattr(lib, n), n
    from paper_1512_02390_amd import sem
    assert sorted(sem.EXPORTS) == names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libsem.so not built")
def test_error_paths_without_device():
    lib = ctypes.CDLL(LIB)
    lib.sem_strerror.restype = ctypes.c_char_p
    lib.sem_strerror.argtypes = [ctypes.c_int32]
    assert lib.sem_strerror(-5) == b"no convergence within imax"
    # null handle / null output are rejected before any device call
    lib.sem_setup.restype = ctypes.c_int32
    assert lib.sem_setup(None, 4, None, None, None, 0, None, None) == -1
    lib.sem_destroy.restype = ctypes.c_int32
    assert lib.sem_destroy(None) == -1
    lib.sem_norm.restype = ctypes.c_int32
    assert lib.sem_norm(None, None, None) == -1


def test_solver_refuses_missing_library(tmp_path):
    from paper_1512_02390_amd import sem
    saved = sem._lib
    sem._lib = None
    try:
        with pytest.raises(OSError):
            sem.load_library(str(tmp_path / "missing.so"))
    finally:
        sem._lib = saved


def test_bench_refuses_more_than_one_gpu():
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    res = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert res.returncode != 0
    assert "one GPU" in res.stderr


def test_precision_enum_matches_binding():
    text = open(HEADER).read()
    body = re.search(r"typedef enum \{([^}]*)\} sem_precision;", text).group(1)
    vals = {k: int(v) for k, v in re.findall(r"(SEM_\w+)\s*=\s*(\d+)", body)}
    from paper_1512_02390_amd import sem
    assert vals == {"SEM_FP64": sem.FP64, "SEM_MIXED_FP32": sem.MIXED_FP32,
                    "SEM_MIXED_BF16": sem.MIXED_BF16, "SEM_MIXED_FP16": sem.MIXED_FP16}


@pytest.mark.skipif(not os.path.exists(LIB), reason="libsem.so not built")
def test_setup_rejects_unknown_precision_without_device():
    lib = ctypes.CDLL(LIB)
    lib.sem_setup.restype = ctypes.c_int32
    h = ctypes.c_void_p(1)
    for prec in (-1, 4):
        # checked before the mesh is read or the device touched
        assert lib.sem_setup(None, 4, None, None, None, prec, None, ctypes.byref(h)) == -1
        assert h.value is None


@pytest.mark.skipif(not os.path.exists(LIB), reason="libsem.so not built")
def test_setup_validation_without_device():
    """Argument checks of sem_setup that precede every device call: bad
    order, element counts, boundary condition, periodic size, overlap,
    weight function, width scales (EINVAL) and non-increasing breaks (EDOM)."""
    import numpy as np
    from paper_1512_02390_amd import sem as S
    C = ctypes
    lib = ctypes.CDLL(LIB)
    lib.sem_setup.restype = C.c_int32

    def setup(nx=3, ny=3, p=4, bc=0, rule=1, n_o=1, wf=5, xb=None, yb=None, alpha=None,
              elem=None, local=0):
        xb = np.linspace(0.0, 1.0, nx + 1) if xb is None else np.asarray(xb, dtype=np.float64)
        yb = np.linspace(0.0, 1.0, ny + 1) if yb is None else np.asarray(yb, dtype=np.float64)
        dp = C.POINTER(C.c_double)
        mesh = S._Mesh(nx, ny, xb.ctypes.data_as(dp), yb.ctypes.data_as(dp), bc)
        ov = S._Overlap(rule, n_o, None)
        ax = None if alpha is None else np.asarray(alpha, dtype=np.float64)
        ep = None if elem is None else np.asarray(elem, dtype=np.float32).reshape(-1)
        w = S._Weights(wf, None if ax is None else ax.ctypes.data_as(dp), None,
                       None if ep is None else ep.ctypes.data_as(C.POINTER(C.c_float)), local)
        h = C.c_void_p(1)
        st = lib.sem_setup(C.byref(mesh), p, C.byref(ov), C.byref(w), None, 0, None, C.byref(h))
        assert h.value is None
        return st

    EINVAL, EDOM = -1, -2
    assert setup(p=0) == EINVAL
    assert setup(nx=0) == EINVAL
    assert setup(bc=7) == EINVAL
    assert setup(bc=1, nx=2) == EINVAL            # periodic needs 3 elements
    assert setup(rule=0, n_o=-1) == EINVAL
    assert setup(wf=4) == EINVAL                  # even kappa
    assert setup(alpha=[1.0, 0.0, 1.0, 1.0]) == EINVAL
    assert setup(alpha=[1.0, 1.5, 1.0, 1.0]) == EINVAL
    good = [[0.5, 0.25]] * 9
    bad_alpha = [[0.5, 0.25]] * 8 + [[0.0, 0.25]]
    big_alpha = [[0.5, 0.25]] * 8 + [[1.5, 0.25]]
    bad_rho = [[0.5, 0.25]] * 8 + [[0.5, -0.1]]
    nan_rho = [[0.5, 0.25]] * 8 + [[0.5, float("nan")]]
    for e in (bad_alpha, big_alpha, bad_rho, nan_rho):
        assert setup(elem=e) == EINVAL
    assert setup(elem=good, alpha=[1.0, 1.0, 1.0, 1.0]) == EINVAL   # one or the other
    assert setup(local=2) == EINVAL                      # unknown local solve
    assert setup(wf=-3, alpha=[1.0, 1.0, 1.0, 1.0]) == -7   # multiplicative: paper weights only
    assert setup(wf=-4) == EINVAL                        # no such weight function
    assert setup(local=1) == EINVAL                      # separable needs a variable nu
    assert setup(xb=[0.0, 0.5, 0.5, 1.0]) == EDOM
    assert setup(yb=[0.0, 0.7, 0.4, 1.0]) == EDOM
