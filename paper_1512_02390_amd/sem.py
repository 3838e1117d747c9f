"""Python binding of libsem (include/sem.h): argument marshalling only.

Every numerical step runs in the HIP library; this module converts torch
device tensors to pointers and host numpy arrays to C arrays.  If the shared
library is missing, importing works but creating a Solver raises, so that no
code path silently falls back to anything else.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsem.so")

BC_DIRICHLET, BC_PERIODIC = 0, 1
W_TOPHAT, W_ARITH, W_MULT = -1, -2, -3
NO_FIXED, NO_CEIL_P8, NO_FLOOR_P8, NO_CEIL_P2 = 0, 1, 2, 3
FP64, MIXED_FP32, MIXED_BF16, MIXED_FP16 = 0, 1, 2, 3

STATUS = {0: "SEM_OK", -1: "SEM_EINVAL", -2: "SEM_EDOM", -3: "SEM_ENOMEM", -4: "SEM_EHIP",
          -5: "SEM_ENOCONV", -6: "SEM_ENAN", -7: "SEM_EUNSUP"}

EXPORTS = ["sem_setup", "sem_destroy", "sem_num_levels", "sem_level_info", "sem_node_coords",
           "sem_mass", "sem_residual", "sem_schwarz_smooth", "sem_restrict", "sem_prolong_add",
           "sem_coarse_solve", "sem_vcycle", "sem_pcg_solve", "sem_norm", "sem_strerror",
           "sem_last_error", "sem_timing_enable", "sem_timing_read", "sem_timing_read_all",
           "sem_elem_features",
           "sem_mlp_num_params", "sem_mlp_create", "sem_mlp_destroy", "sem_mlp_forward",
           "sem_mlp_gradient", "sem_mlp_train_step", "sem_mlp_get_params",
           "sem_learned_params", "sem_norm_noalloc",
           "sem3_setup", "sem3_destroy", "sem3_num_levels", "sem3_level_info", "sem3_residual",
           "sem3_schwarz_smooth", "sem3_restrict", "sem3_prolong_add", "sem3_coarse_solve",
           "sem3_vcycle", "sem3_pcg_solve", "sem3_last_error"]


class SemError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class _Mesh(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("xb", C.POINTER(C.c_double)),
                ("yb", C.POINTER(C.c_double)), ("bc", C.c_int32)]


class _Overlap(C.Structure):
    _fields_ = [("rule", C.c_int32), ("n_o", C.c_int32), ("per_level", C.POINTER(C.c_int32))]


class _Mesh3(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("xb", C.POINTER(C.c_double)), ("yb", C.POINTER(C.c_double)),
                ("zb", C.POINTER(C.c_double))]


class _Weights(C.Structure):
    _fields_ = [("wf", C.c_int32), ("alpha_x", C.POINTER(C.c_double)),
                ("alpha_y", C.POINTER(C.c_double)), ("elem_params", C.POINTER(C.c_float)),
                ("local_solve", C.c_int32)]


LOCAL_MEAN, LOCAL_SEPARABLE = 0, 1


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libsem.so (raises OSError if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise OSError(f"{path} not found: build it with python -m paper_1512_02390_amd.build")
    lib = C.CDLL(path)
    P, I32, I64, D = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    lib.sem_setup.argtypes = [C.POINTER(_Mesh), I32, C.POINTER(_Overlap), C.POINTER(_Weights),
                              C.POINTER(D), I32, P, C.POINTER(P)]
    lib.sem_destroy.argtypes = [P]
    lib.sem_num_levels.argtypes = [P, C.POINTER(I32)]
    lib.sem_level_info.argtypes = [P, I32, C.POINTER(I32), C.POINTER(I32), C.POINTER(I64),
                                   C.POINTER(I64)]
    lib.sem_node_coords.argtypes = [P, I32, C.POINTER(D), C.POINTER(D)]
    lib.sem_mass.argtypes = [P, P, P]
    lib.sem_residual.argtypes = [P, I32, P, P, P]
    lib.sem_schwarz_smooth.argtypes = [P, I32, P, P, I32]
    lib.sem_restrict.argtypes = [P, I32, P, P]
    lib.sem_prolong_add.argtypes = [P, I32, P, P]
    lib.sem_coarse_solve.argtypes = [P, P, P]
    lib.sem_vcycle.argtypes = [P, P, P, C.POINTER(I32), C.POINTER(I32)]
    lib.sem_pcg_solve.argtypes = [P, P, P, I32, D, C.POINTER(I32), C.POINTER(I32),
                                  C.POINTER(I32), C.POINTER(D)]
    lib.sem_norm.argtypes = [P, P, C.POINTER(D)]
    lib.sem_norm_noalloc.argtypes = [P, P, C.POINTER(D)]
    lib.sem3_setup.argtypes = [C.POINTER(_Mesh3), I32, C.POINTER(_Overlap), I32, P, C.POINTER(P)]
    lib.sem3_destroy.argtypes = [P]
    lib.sem3_num_levels.argtypes = [P, C.POINTER(I32)]
    lib.sem3_level_info.argtypes = [P, I32, C.POINTER(I32), C.POINTER(I32), C.POINTER(I64)]
    lib.sem3_residual.argtypes = [P, I32, P, P, P]
    lib.sem3_schwarz_smooth.argtypes = [P, I32, P, P, I32]
    lib.sem3_restrict.argtypes = [P, I32, P, P]
    lib.sem3_prolong_add.argtypes = [P, I32, P, P]
    lib.sem3_coarse_solve.argtypes = [P, P, P]
    lib.sem3_vcycle.argtypes = [P, P, P, P, P]
    lib.sem3_pcg_solve.argtypes = [P, P, P, I32, D, P, P, C.POINTER(I32), C.POINTER(D)]
    lib.sem3_last_error.argtypes = [P]
    lib.sem3_last_error.restype = C.c_char_p
    lib.sem_timing_enable.argtypes = [P, I32, I32]
    lib.sem_timing_read.argtypes = [P, C.POINTER(I64), C.POINTER(D)]
    lib.sem_timing_read_all.argtypes = [P, C.POINTER(I64), C.POINTER(D)]
    F = C.POINTER(C.c_float)
    lib.sem_elem_features.argtypes = [P, P]
    lib.sem_mlp_num_params.argtypes = [I32, I32, I32, C.POINTER(I64)]
    lib.sem_mlp_create.argtypes = [I32, I32, I32, F, P, C.POINTER(P)]
    lib.sem_mlp_destroy.argtypes = [P]
    lib.sem_mlp_forward.argtypes = [P, P, I64, P]
    lib.sem_mlp_gradient.argtypes = [P, P, P, I64, P, F]
    lib.sem_mlp_train_step.argtypes = [P, P, P, I64, C.c_float, F]
    lib.sem_mlp_get_params.argtypes = [P, F]
    lib.sem_learned_params.argtypes = [F, I32, I32, I32, I32, C.POINTER(I32), C.POINTER(D),
                                       C.POINTER(D)]
    lib.sem_strerror.argtypes = [I32]
    lib.sem_strerror.restype = C.c_char_p
    lib.sem_last_error.argtypes = [P]
    lib.sem_last_error.restype = C.c_char_p
    for name in EXPORTS:
        if name not in ("sem_strerror", "sem_last_error"):
            getattr(lib, name).restype = C.c_int32
    _lib = lib
    return lib


def _ptr(t) -> int:
    if t is None:
        return None
    if not (t.is_cuda and t.is_contiguous()):
        raise ValueError("expected a contiguous device tensor")
    return t.data_ptr()


def _i32_array(v):
    if v is None:
        return None
    a = (C.c_int32 * len(v))(*[int(x) for x in v])
    return a


class Solver:
    """Handle of one SEM problem (all multigrid levels) on the current device."""

    def __init__(self, xb, yb, p: int, bc: int = BC_DIRICHLET, overlap_rule: int = NO_FIXED,
                 n_o: int = 1, wf: int = 5, nu=None, precision: int = FP64, alpha_x=None,
                 alpha_y=None, stream=None, overlaps=None, elem_params=None,
                 local_solve: int = LOCAL_MEAN):
        """elem_params: optional (n_e, 2) array of per-element (alpha_e, rho_e),
        e = ey * nx + ex (see sem_weights in include/sem.h)."""
        import torch
        self.lib = load_library()
        self.torch = torch
        self._xb = np.ascontiguousarray(xb, dtype=np.float64)
        self._yb = np.ascontiguousarray(yb, dtype=np.float64)
        dp = C.POINTER(C.c_double)
        mesh = _Mesh(len(self._xb) - 1, len(self._yb) - 1, self._xb.ctypes.data_as(dp),
                     self._yb.ctypes.data_as(dp), bc)
        self._ovl = None if overlaps is None else _i32_array(overlaps)
        ov = _Overlap(overlap_rule, n_o, self._ovl)
        self._ax = None if alpha_x is None else np.ascontiguousarray(alpha_x, dtype=np.float64)
        self._ay = None if alpha_y is None else np.ascontiguousarray(alpha_y, dtype=np.float64)
        self._ep = None if elem_params is None else np.ascontiguousarray(
            elem_params, dtype=np.float32).reshape(-1)
        wts = _Weights(wf, None if self._ax is None else self._ax.ctypes.data_as(dp),
                       None if self._ay is None else self._ay.ctypes.data_as(dp),
                       None if self._ep is None else self._ep.ctypes.data_as(C.POINTER(C.c_float)),
                       int(local_solve))
        nu_host = None
        if nu is not None:
            nu_host = np.ascontiguousarray(nu, dtype=np.float64)
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        self.stream = stream
        h = C.c_void_p()
        st = self.lib.sem_setup(C.byref(mesh), p, C.byref(ov), C.byref(wts),
                                None if nu_host is None else nu_host.ctypes.data_as(dp),
                                precision, C.c_void_p(stream), C.byref(h))
        if st != 0:
            raise SemError(st, self.lib.sem_last_error(None).decode())
        self.h = h
        self.p = p
        self.bc = bc
        n = C.c_int32()
        self.lib.sem_num_levels(self.h, C.byref(n))
        self.nlevels = n.value
        self.L = self.nlevels - 1

    def _check(self, st):
        if st != 0:
            raise SemError(st, self.lib.sem_last_error(self.h).decode())
        return st

    def close(self):
        if getattr(self, "h", None):
            self.lib.sem_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- layout ---------------------------------------------------------------
    def level_info(self, level: int):
        pl, no = C.c_int32(), C.c_int32()
        r, c = C.c_int64(), C.c_int64()
        self._check(self.lib.sem_level_info(self.h, level, C.byref(pl), C.byref(no), C.byref(r),
                                            C.byref(c)))
        return pl.value, no.value, r.value, c.value

    def shape(self, level: int | None = None):
        _, _, r, c = self.level_info(self.L if level is None else level)
        return r, c

    def node_coords(self, level: int | None = None):
        level = self.L if level is None else level
        r, c = self.shape(level)
        x = np.zeros(c)
        y = np.zeros(r)
        dp = C.POINTER(C.c_double)
        self._check(self.lib.sem_node_coords(self.h, level, x.ctypes.data_as(dp),
                                             y.ctypes.data_as(dp)))
        return x, y

    def zeros(self, level: int | None = None):
        return self.torch.zeros(self.shape(level), dtype=self.torch.float64, device="cuda")

    # -- operations -------------------------------------------------------------
    def mass(self, f_nodal, b):
        self._check(self.lib.sem_mass(self.h, _ptr(f_nodal), _ptr(b)))

    def residual(self, level: int, u, f, r):
        self._check(self.lib.sem_residual(self.h, level, _ptr(u), _ptr(f), _ptr(r)))

    def schwarz_smooth(self, level: int, u, f, n_it: int = 1):
        self._check(self.lib.sem_schwarz_smooth(self.h, level, _ptr(u), _ptr(f), n_it))

    def restrict(self, level: int, r_fine, f_coarse):
        self._check(self.lib.sem_restrict(self.h, level, _ptr(r_fine), _ptr(f_coarse)))

    def prolong_add(self, level: int, u_coarse, u_fine):
        self._check(self.lib.sem_prolong_add(self.h, level, _ptr(u_coarse), _ptr(u_fine)))

    def coarse_solve(self, f0, u0):
        self._check(self.lib.sem_coarse_solve(self.h, _ptr(f0), _ptr(u0)))

    def vcycle(self, u, f, ns1=None, ns2=None):
        self._check(self.lib.sem_vcycle(self.h, _ptr(u), _ptr(f), _i32_array(ns1),
                                        _i32_array(ns2)))

    def pcg_solve(self, u, f, imax: int = 100, rtol: float = 1e-10, ns1=None, ns2=None):
        """Returns (iterations, residual history, converged)."""
        it = C.c_int32()
        hist = np.zeros(imax + 1)
        st = self.lib.sem_pcg_solve(self.h, _ptr(u), _ptr(f), imax, rtol, _i32_array(ns1),
                                    _i32_array(ns2), C.byref(it),
                                    hist.ctypes.data_as(C.POINTER(C.c_double)))
        if st not in (0, -5):
            self._check(st)
        return it.value, hist[: it.value + 1], st == 0

    def timing_enable(self, level: int, on: bool = True):
        self._check(self.lib.sem_timing_enable(self.h, level, 1 if on else 0))

    def timing_read(self):
        """(number of timed Schwarz-kernel launches, summed milliseconds)."""
        n, ms = C.c_int64(), C.c_double()
        self._check(self.lib.sem_timing_read(self.h, C.byref(n), C.byref(ms)))
        return n.value, ms.value

    TIME_KINDS = ("schwarz", "residual", "restrict", "prolong", "apply")

    def timing_read_all(self):
        """{kind: (number of timed launches, summed milliseconds)} for the
        Schwarz, residual, restriction, prolongation and operator-product
        kernels of the timed level (the record is cleared)."""
        n = (C.c_int64 * len(self.TIME_KINDS))()
        ms = (C.c_double * len(self.TIME_KINDS))()
        self._check(self.lib.sem_timing_read_all(self.h, n, ms))
        return {k: (n[i], ms[i]) for i, k in enumerate(self.TIME_KINDS)}

    def norm(self, x) -> float:
        out = C.c_double()
        self._check(self.lib.sem_norm(self.h, _ptr(x), C.byref(out)))
        return out.value

    def norm_noalloc(self, x) -> float:
        """norm() through the allocation-free entry point."""
        out = C.c_double()
        self._check(self.lib.sem_norm_noalloc(self.h, _ptr(x), C.byref(out)))
        return out.value

    def elem_features(self):
        """Device tensor (n_e, 8) of FP32 element features, e = ey * nx + ex."""
        ne = (len(self._xb) - 1) * (len(self._yb) - 1)
        out = self.torch.empty((ne, 8), dtype=self.torch.float32, device="cuda")
        self._check(self.lib.sem_elem_features(self.h, _ptr(out)))
        return out


def _raise(st, what):
    if st != 0:
        raise SemError(st, what)


class MLP:
    """Device MLP d_in -> 64 -> 64 -> d_out (tanh, logistic output) trained with
    the library's own forward / backward / Adam kernels."""

    def __init__(self, params, d_in: int = 8, width: int = 64, d_out: int = 2, stream=None):
        import torch
        self.lib = load_library()
        self.torch = torch
        self.d_in, self.width, self.d_out = d_in, width, d_out
        n = C.c_int64()
        _raise(self.lib.sem_mlp_num_params(d_in, width, d_out, C.byref(n)), "mlp dimensions")
        self.np = n.value
        p = np.ascontiguousarray(params, dtype=np.float32)
        if p.size != self.np:
            raise ValueError(f"expected {self.np} parameters, got {p.size}")
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        h = C.c_void_p()
        _raise(self.lib.sem_mlp_create(d_in, width, d_out, p.ctypes.data_as(C.POINTER(C.c_float)),
                                       C.c_void_p(stream), C.byref(h)), "sem_mlp_create")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.sem_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def forward(self, x):
        y = self.torch.empty((x.shape[0], self.d_out), dtype=self.torch.float32, device="cuda")
        _raise(self.lib.sem_mlp_forward(self.h, _ptr(x), x.shape[0], _ptr(y)), "sem_mlp_forward")
        return y

    def gradient(self, x, t):
        """(loss, gradient as a device tensor)."""
        g = self.torch.empty(self.np, dtype=self.torch.float32, device="cuda")
        loss = C.c_float()
        _raise(self.lib.sem_mlp_gradient(self.h, _ptr(x), _ptr(t), x.shape[0], _ptr(g),
                                         C.byref(loss)), "sem_mlp_gradient")
        return loss.value, g

    def train_step(self, x, t, lr: float, want_loss: bool = False):
        loss = C.c_float()
        _raise(self.lib.sem_mlp_train_step(self.h, _ptr(x), _ptr(t), x.shape[0], lr,
                                           C.byref(loss) if want_loss else None),
               "sem_mlp_train_step")
        return loss.value if want_loss else None

    def get_params(self) -> np.ndarray:
        out = np.zeros(self.np, dtype=np.float32)
        _raise(self.lib.sem_mlp_get_params(self.h, out.ctypes.data_as(C.POINTER(C.c_float))),
               "sem_mlp_get_params")
        return out


def learned_params(pred, nx: int, ny: int, p: int, bc: int):
    """Reduce per-element predictions (n_e, 2) = (alpha_e, q_e) to
    (overlaps per level, alpha per x grid line, alpha per y grid line)."""
    lib = load_library()
    pr = np.ascontiguousarray(pred, dtype=np.float32).reshape(-1)
    levels = 1
    q = p
    while q > 1:
        q = (q + 1) // 2
        levels += 1
    ov = (C.c_int32 * levels)()
    ax = np.zeros(nx + 1)
    ay = np.zeros(ny + 1)
    dp = C.POINTER(C.c_double)
    _raise(lib.sem_learned_params(pr.ctypes.data_as(C.POINTER(C.c_float)), nx, ny, p, bc, ov,
                                  ax.ctypes.data_as(dp), ay.ctypes.data_as(dp)),
           "sem_learned_params")
    return list(ov), ax, ay


class Solver3:
    """Handle of one 3-D Poisson problem (all multigrid levels) on the current
    device: the sem3_* entry points, argument marshalling only."""

    def __init__(self, xb, yb, zb, p: int, overlap_rule: int = NO_FIXED, n_o: int = 1,
                 wf: int = 5, stream=None):
        import torch
        self.lib = load_library()
        self.torch = torch
        self._b = [np.ascontiguousarray(b, dtype=np.float64) for b in (xb, yb, zb)]
        dp = C.POINTER(C.c_double)
        mesh = _Mesh3(len(self._b[0]) - 1, len(self._b[1]) - 1, len(self._b[2]) - 1,
                      *[b.ctypes.data_as(dp) for b in self._b])
        ov = _Overlap(overlap_rule, n_o, None)
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        self.stream = stream
        h = C.c_void_p()
        st = self.lib.sem3_setup(C.byref(mesh), p, C.byref(ov), wf, C.c_void_p(stream), C.byref(h))
        if st != 0:
            raise SemError(st, "sem3_setup failed")
        self.h = h
        n = C.c_int32()
        self._check(self.lib.sem3_num_levels(self.h, C.byref(n)))
        self.L = n.value - 1

    def _check(self, st):
        if st != 0:
            raise SemError(st, self.lib.sem3_last_error(self.h).decode())
        return st

    def close(self):
        if getattr(self, "h", None):
            self.lib.sem3_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def level_info(self, level: int):
        """(p_l, n_o, (nodes z, y, x))."""
        p, no = C.c_int32(), C.c_int32()
        nodes = (C.c_int64 * 3)()
        self._check(self.lib.sem3_level_info(self.h, level, C.byref(p), C.byref(no), nodes))
        return p.value, no.value, (nodes[2], nodes[1], nodes[0])

    def zeros(self, level: int | None = None):
        shape = self.level_info(self.L if level is None else level)[2]
        return self.torch.zeros(shape, dtype=self.torch.float64, device="cuda")

    def residual(self, level: int, u, f, r):
        self._check(self.lib.sem3_residual(self.h, level, _ptr(u), _ptr(f), _ptr(r)))

    def schwarz_smooth(self, level: int, u, f, n_it: int = 1):
        self._check(self.lib.sem3_schwarz_smooth(self.h, level, _ptr(u), _ptr(f), n_it))

    def restrict(self, level: int, rf, fc):
        self._check(self.lib.sem3_restrict(self.h, level, _ptr(rf), _ptr(fc)))

    def prolong_add(self, level: int, uc, uf):
        self._check(self.lib.sem3_prolong_add(self.h, level, _ptr(uc), _ptr(uf)))

    def coarse_solve(self, f0, u0):
        self._check(self.lib.sem3_coarse_solve(self.h, _ptr(f0), _ptr(u0)))

    def vcycle(self, u, f, ns1=None, ns2=None):
        self._check(self.lib.sem3_vcycle(self.h, _ptr(u), _ptr(f), _i32_array(ns1), _i32_array(ns2)))

    def pcg_solve(self, u, f, imax: int = 100, rtol: float = 1e-10, ns1=None, ns2=None):
        """Returns (iterations, residual history, converged)."""
        it = C.c_int32()
        hist = np.zeros(imax + 1)
        st = self.lib.sem3_pcg_solve(self.h, _ptr(u), _ptr(f), imax, rtol, _i32_array(ns1),
                                     _i32_array(ns2), C.byref(it),
                                     hist.ctypes.data_as(C.POINTER(C.c_double)))
        if st not in (0, -5):
            self._check(st)
        return it.value, hist[: it.value + 1], st == 0
